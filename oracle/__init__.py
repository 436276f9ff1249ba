"""FP64 CPU oracle for the stereo path (Sec. 2.2, Eq. 1-2) -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``libbp_oracle.so`` (plain C, FP64, built from
``bp_oracle.c`` by ``oracle/build.py``) with numpy arrays.  It imports nothing
from the GPU library and the GPU library imports nothing from it.

Message arrays use the layout [4][L][H][W]; slot k holds the message a pixel
received from its neighbour on side k (0 left, 1 right, 2 up, 3 down).

Parity pins: every function here is pinned by the ``-m "not gpu"`` tests
(brute force, chain and tree dynamic programming, enumeration, closed forms,
worked examples under tests/golden).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libbp_oracle.so")
# Compiler flags of the library (oracle/build.py), reported with CPU timings.
BUILD_FLAGS = "gcc -std=c11 -O3 -march=x86-64-v3 -ffp-contract=off -fopenmp"
_lib = None

STORE_F64, STORE_F16, STORE_BF16, STORE_F32 = 0, 1, 2, 3
_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i32p = ctypes.POINTER(ctypes.c_int32)


def lib():
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        i = ctypes.c_int
        d = ctypes.c_double
        L.bpo_downsample.argtypes = [_u8p, i, i, i, i, _u8p]
        L.bpo_cost_volume.argtypes = [_u8p, _u8p, i, i, i, i, d, i, _dp]
        L.bpo_dt.argtypes = [_dp, i, d, d, _dp]
        L.bpo_dt.restype = None
        L.bpo_dt_brute.argtypes = [_dp, i, d, d, _dp]
        L.bpo_dt_brute.restype = None
        L.bpo_run.argtypes = [_dp, i, i, i, i, i, d, d, i, i, _u8p, _dp, _dp, _i32p, _dp, d, i]
        L.bpo_pyramid.argtypes = [_dp, i, i, i, i, _dp]
        L.bpo_upsample.argtypes = [_i32p, i, i, _u8p, i, i, i, d, d, i, _dp, i]
        L.bpo_triangulate.argtypes = [_dp, i, i, d, d, d, d, d, d, d, _dp]
        L.bpo_undistort.argtypes = [_u8p, i, i, i, ctypes.POINTER(ctypes.c_float), _u8p]
        _i64p = ctypes.POINTER(ctypes.c_int64)
        L.bpo_harris_response.argtypes = [_u8p, i, i, _i64p]
        L.bpo_harris_cells.argtypes = [_i64p, i, i, i, ctypes.c_int64, _i64p]
        L.bpo_zssd_match.argtypes = [_u8p, _u8p, i, i, _i64p, i, i, i, _i64p]
        _fp = ctypes.POINTER(ctypes.c_float)
        L.bpo_icp_correspond.argtypes = [_fp, i, _fp, i, _fp, _fp, ctypes.c_float, _fp,
                                         ctypes.POINTER(ctypes.c_int32), _fp]
        L.bpo_round_f16.argtypes = [d]
        L.bpo_round_f16.restype = d
        L.bpo_round_bf16.argtypes = [d]
        L.bpo_round_bf16.restype = d
        L.bpo_max_threads.restype = i
        L.bpo_backward.argtypes = [_dp, i, i, i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, i]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


def _img(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    if a.ndim == 2:
        return a, a.shape[0], a.shape[1], 1
    return a, a.shape[0], a.shape[1], a.shape[2]


def downsample(img, s: int):
    a, H, W, C = _img(img)
    out = np.empty((H // s, W // s) + ((C,) if img.ndim == 3 else ()), dtype=np.uint8)
    _check(lib().bpo_downsample(_p(a, _u8p), W, H, C, s, _p(out, _u8p)), "downsample")
    return out


def cost_volume(left, right, num_labels: int, data_trunc: float = 20.0, rgb_mode: int = 0):
    """Truncated absolute-difference cost [L][H][W] (float64)."""
    a, H, W, C = _img(left)
    b, _, _, _ = _img(right)
    out = np.empty((num_labels, H, W), dtype=np.float64)
    _check(lib().bpo_cost_volume(_p(a, _u8p), _p(b, _u8p), W, H, C, num_labels, float(data_trunc),
                                 int(rgb_mode), _p(out, _dp)), "cost_volume")
    return out


def dt(h, lam: float, tau: float, brute: bool = False):
    """One normalised message: min_g h(g) + lam*min(|f-g|, tau), minus its minimum."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    out = np.empty_like(h)
    fn = lib().bpo_dt_brute if brute else lib().bpo_dt
    fn(_p(h, _dp), h.shape[0], float(lam), float(tau), _p(out, _dp))
    return out


def pyramid(cost, level: int):
    cost = np.ascontiguousarray(cost, dtype=np.float64)
    L, H, W = cost.shape
    w, h = W, H
    for _ in range(level):
        w, h = (w + 1) // 2, (h + 1) // 2
    out = np.empty((L, h, w), dtype=np.float64)
    _check(lib().bpo_pyramid(_p(cost, _dp), W, H, L, level, _p(out, _dp)), "pyramid")
    return out


def run(cost, levels: int = 1, iters: int = 10, lam: float = 10.0, tau: float = 2.0, *,
        store_mode: int = STORE_F64, brute: bool = False, edges=None, msgs_init=None,
        want_msgs: bool = False, want_soft: bool = False, temperature: float = 0.5,
        nthreads: int = 0):
    """Hierarchical checkerboard BP.  Returns dict(disp, soft?, msgs?)."""
    cost = np.ascontiguousarray(cost, dtype=np.float64)
    L, H, W = cost.shape
    disp = np.empty((H, W), dtype=np.int32)
    soft = np.empty((H, W), dtype=np.float64) if want_soft else None
    msgs = np.empty((4, L, H, W), dtype=np.float64) if want_msgs else None
    if edges is not None:
        edges = np.ascontiguousarray(edges, dtype=np.uint8)
    if msgs_init is not None:
        msgs_init = np.ascontiguousarray(msgs_init, dtype=np.float64)
    rc = lib().bpo_run(_p(cost, _dp), W, H, L, int(levels), int(iters), float(lam), float(tau),
                       int(store_mode), 1 if brute else 0, _p(edges, _u8p), _p(msgs_init, _dp),
                       _p(msgs, _dp), _p(disp, _i32p), _p(soft, _dp), float(temperature),
                       int(nthreads))
    _check(rc, "run")
    out = {"disp": disp}
    if want_soft:
        out["soft"] = soft
    if want_msgs:
        out["msgs"] = msgs
    return out


def upsample(disp_lo, guide, sigma_s: float = 8.0, sigma_r: float = 12.0, radius: int = -1,
             nthreads: int = 0):
    """Joint bilateral upsampling (Eq. 2) -> float64 [H_hi][W_hi] in label units."""
    d = np.ascontiguousarray(disp_lo, dtype=np.int32)
    g, hh, wh, C = _img(guide)
    hl, wl = d.shape
    out = np.empty((hh, wh), dtype=np.float64)
    _check(lib().bpo_upsample(_p(d, _i32p), wl, hl, _p(g, _u8p), wh, hh, C, float(sigma_s),
                              float(sigma_r), int(radius), _p(out, _dp), int(nthreads)), "upsample")
    return out


def triangulate(disp, scale: float, baseline: float, focal: float, du: float, dv: float, u0: float, v0: float):
    """Eq. 3: camera-frame points [H][W][3] of a full-resolution disparity map
    (in 1/scale pixel units); NaN where the disparity is not positive."""
    dd = np.ascontiguousarray(disp, dtype=np.float64)
    h, w = dd.shape
    out = np.empty((h, w, 3), dtype=np.float64)
    _check(lib().bpo_triangulate(_p(dd, _dp), w, h, float(scale), float(baseline), float(focal), float(du),
                                 float(dv), float(u0), float(v0), _p(out, _dp)), "triangulate")
    return out


def undistort(img, fx: float, fy: float, cx: float, cy: float, k1: float = 0.0, k2: float = 0.0, k3: float = 0.0):
    """Radial-only undistortion with bilinear sampling (Sec. 2.1), u8 in, u8 out."""
    g, h, w, C = _img(img)
    K = np.array([fx, fy, cx, cy, k1, k2, k3], dtype=np.float32)
    out = np.empty_like(g)
    _check(lib().bpo_undistort(_p(g, _u8p), w, h, C, K.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                               _p(out, _u8p)), "undistort")
    return out


def harris_response(img):
    """25 R of Eq. 5 (k = 1/25) per pixel of a grey u8 frame, int64 [H][W]."""
    g, h, w, C = _img(img)
    if C != 1:
        raise ValueError("grey frames only")
    out = np.empty((h, w), dtype=np.int64)
    _check(lib().bpo_harris_response(_p(g, _u8p), w, h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
           "harris_response")
    return out


def harris_cells(r25, grid: int = 30, threshold: int = 0):
    """Per-cell corners of a g x g grid: int64 [g*g][3] (x, y, 25 R); x = -1 if none."""
    r = np.ascontiguousarray(r25, dtype=np.int64)
    h, w = r.shape
    out = np.empty((grid * grid, 3), dtype=np.int64)
    P = ctypes.POINTER(ctypes.c_int64)
    _check(lib().bpo_harris_cells(r.ctypes.data_as(P), w, h, grid, int(threshold), out.ctypes.data_as(P)),
           "harris_cells")
    return out


def zssd_match(a, b, corners, patch_radius: int, search_radius: int):
    """ZSSD matches of the corners (rows x, y, ...) of frame a in frame b:
    int64 [n][3] (x2, y2, n_pix * ZSSD); x2 = -1 if none."""
    ga, h, w, _ = _img(a)
    gb, _, _, _ = _img(b)
    c = np.ascontiguousarray(corners, dtype=np.int64)
    out = np.empty((c.shape[0], 3), dtype=np.int64)
    P = ctypes.POINTER(ctypes.c_int64)
    _check(lib().bpo_zssd_match(_p(ga, _u8p), _p(gb, _u8p), w, h, c.ctypes.data_as(P), c.shape[0],
                                int(patch_radius), int(search_radius), out.ctypes.data_as(P)), "zssd_match")
    return out


def icp_correspond(src, dst, R, T, dmax: float):
    """One ICP correspondence step in FP32: moved points R p + T, index of the
    nearest target within dmax (-1 if none, lowest index on ties), and the
    squared distance."""
    F = ctypes.POINTER(ctypes.c_float)
    s = np.ascontiguousarray(src, dtype=np.float32)
    d = np.ascontiguousarray(dst, dtype=np.float32)
    r = np.ascontiguousarray(R, dtype=np.float32).reshape(9)
    t = np.ascontiguousarray(T, dtype=np.float32).reshape(3)
    moved = np.empty_like(s)
    corr = np.empty(s.shape[0], dtype=np.int32)
    d2 = np.empty(s.shape[0], dtype=np.float32)
    dm2 = np.float32(dmax) * np.float32(dmax)
    _check(lib().bpo_icp_correspond(s.ctypes.data_as(F), s.shape[0], d.ctypes.data_as(F), d.shape[0],
                                    r.ctypes.data_as(F), t.ctypes.data_as(F), float(dm2), moved.ctypes.data_as(F),
                                    corr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), d2.ctypes.data_as(F)),
           "icp_correspond")
    return moved, corr, d2


def kabsch(p, q):
    """Least-squares rotation and translation taking points p onto q
    (centroids and the SVD of the cross-covariance, FP64, with the
    determinant correction that excludes reflections)."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    pc, qc = p.mean(axis=0), q.mean(axis=0)
    H = (p - pc).T @ (q - qc)
    U, _, Vt = np.linalg.svd(H)
    D = np.diag([1.0, 1.0, np.sign(np.linalg.det(Vt.T @ U.T))])
    R = Vt.T @ D @ U.T
    return R, qc - R @ pc


def icp(src, dst, R0, T0, iters: int, dmax: float):
    """Point-to-point ICP (Sec. 2.3 fine registration): per iteration the
    FP32 correspondence step, then the FP64 least-squares update over the
    accepted pairs composed onto the pose (left unchanged by an iteration
    with fewer than 3 pairs).  Returns (R, T, rms per iteration, pairs per
    iteration, the last iteration's correspondences)."""
    R = np.asarray(R0, dtype=np.float64)
    T = np.asarray(T0, dtype=np.float64)
    rms, npairs = [], []
    dst64 = np.asarray(dst, dtype=np.float64)
    corr = None
    for _ in range(iters):
        moved, corr, d2 = icp_correspond(src, dst, R.astype(np.float32), T.astype(np.float32), dmax)
        ok = corr >= 0
        npairs.append(int(ok.sum()))
        rms.append(float(np.sqrt(d2[ok].astype(np.float64).mean())) if ok.any() else 0.0)
        if ok.sum() < 3:
            continue
        Ri, Ti = kabsch(moved[ok].astype(np.float64), dst64[corr[ok]])
        R, T = Ri @ R, Ri @ T + Ti
    return R, T, rms, npairs, corr


def round_f16(x: float) -> float:
    return lib().bpo_round_f16(float(x))


def round_bf16(x: float) -> float:
    return lib().bpo_round_bf16(float(x))


def max_threads() -> int:
    return lib().bpo_max_threads()


def backward(cost, iters: int, lam: float, tau: float, temperature: float, grad_soft, nthreads: int = 0):
    """Single-level BP with soft-argmin readout and its reverse-mode derivative.

    Returns (soft [H][W], grad_cost [L][H][W], grad_lambda, grad_tau) for the
    loss sum(grad_soft * soft).
    """
    cost = np.ascontiguousarray(cost, dtype=np.float64)
    L, H, W = cost.shape
    g = np.ascontiguousarray(grad_soft, dtype=np.float64)
    soft = np.empty((H, W), dtype=np.float64)
    gc = np.empty_like(cost)
    gl = ctypes.c_double(0.0)
    gt = ctypes.c_double(0.0)
    rc = lib().bpo_backward(_p(cost, _dp), W, H, L, int(iters), float(lam), float(tau), float(temperature),
                            _p(g, _dp), _p(soft, _dp), _p(gc, _dp), ctypes.byref(gl), ctypes.byref(gt),
                            int(nthreads))
    _check(rc, "backward")
    return soft, gc, gl.value, gt.value
