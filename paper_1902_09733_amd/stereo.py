"""PyTorch-facing binding of libbpstereo.

Every function marshals torch tensors (device memory) and the current HIP
stream into the C ABI of include/bp.h; all arithmetic runs in the library's
HIP kernels.  Nothing here computes a stereo result on the host, and there is
no fallback: a missing library or a non-GPU tensor raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _abi

MSG_DTYPES = {"f32": _abi.BP_MSG_F32, "f16": _abi.BP_MSG_F16, "bf16": _abi.BP_MSG_BF16}


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need_gpu(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("libbpstereo works on GPU tensors only")
        if t is not None and not t.is_contiguous():
            raise ValueError("tensors must be contiguous")


def _img_dims(img):
    if img.dim() == 2:
        return img.shape[1], img.shape[0], 1
    return img.shape[1], img.shape[0], img.shape[2]


def downsample(img: torch.Tensor, factor: int, stream=None) -> torch.Tensor:
    """s x s block mean (rounded half up) of a u8 [H][W] or [H][W][3] image."""
    _need_gpu(img)
    w, h, c = _img_dims(img)
    out = torch.empty((h // factor, w // factor) + ((c,) if img.dim() == 3 else ()), dtype=torch.uint8,
                      device=img.device)
    st = _abi.lib().bp_downsample(_ptr(img), w, h, c, w * c, factor, _ptr(out), _stream(stream))
    _abi.check("bp_downsample", st)
    return out


def cost_volume(left: torch.Tensor, right: torch.Tensor, num_labels: int, data_trunc: float = 20.0,
                downsample: int = 1, rgb_mode: int = 0, out: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
    """Truncated absolute-difference data term, float32 [L][H/s][W/s]."""
    _need_gpu(left, right)
    if left.dtype != torch.uint8 or right.dtype != torch.uint8 or left.shape != right.shape:
        raise ValueError("left/right must be u8 images of the same shape")
    w, h, c = _img_dims(left)
    if out is None:
        out = torch.empty((num_labels, h // downsample, w // downsample), dtype=torch.float32, device=left.device)
    _need_gpu(out)
    st = _abi.lib().bp_cost_volume(_ptr(left), _ptr(right), w, h, c, w * c, downsample, num_labels,
                                   float(data_trunc), rgb_mode, _ptr(out), _stream(stream))
    _abi.check("bp_cost_volume", st)
    return out


@dataclass
class Pair:
    """A rectified u8 pair ([H][W] or [H][W][3]) standing in for a cost volume
    in ``run``: the library computes the finest-level data term itself (the
    values ``cost_volume`` gives for the same arguments) straight into its
    internal layout, without a planar volume in memory."""
    left: torch.Tensor
    right: torch.Tensor
    num_labels: int
    data_trunc: float = 20.0
    downsample: int = 1
    rgb_mode: int = 0

    @property
    def shape(self):
        w, h, _ = _img_dims(self.left)
        return (self.num_labels, h // self.downsample, w // self.downsample)

    @property
    def device(self):
        return self.left.device

    def c(self):
        _need_gpu(self.left, self.right)
        if self.left.dtype != torch.uint8 or self.right.dtype != torch.uint8 or self.left.shape != self.right.shape:
            raise ValueError("left/right must be u8 images of the same shape")
        w, _, ch = _img_dims(self.left)
        return _abi.BpPair(self.left.data_ptr(), self.right.data_ptr(), ch, self.downsample, w * ch,
                           float(self.data_trunc), self.rgb_mode)


@dataclass
class BPParams:
    levels: int = 1
    iters: int = 10
    lam: float = 10.0
    tau: float = 2.0
    msg_dtype: str = "f32"
    temperature: float = 0.5
    checkpoint_every: int = 0
    variant: int = 0
    pm_from: int = -1

    def c(self) -> _abi.BpParams:
        return _abi.BpParams(self.levels, self.iters, self.lam, self.tau, MSG_DTYPES[self.msg_dtype],
                             self.temperature, self.checkpoint_every, self.variant, self.pm_from)


class Workspace:
    """Reusable device scratch buffer (grows on demand; 256-byte aligned)."""

    def __init__(self, device=None):
        self.device = device
        self.buf = None

    def get(self, nbytes: int, device) -> torch.Tensor:
        need = nbytes + 256
        if self.buf is None or self.buf.numel() < need or self.buf.device != device:
            self.buf = torch.empty(need, dtype=torch.uint8, device=device)
        off = (-self.buf.data_ptr()) % 256
        return self.buf[off:off + nbytes] if nbytes else self.buf[:0]


_default_ws = Workspace()


def _problems(costs, disps, softs, msgs):
    probs = (_abi.BpProblem * len(costs))()
    pairs = []                       # BpPair structs, kept alive with the array
    for i, c in enumerate(costs):
        L, h, w = c.shape
        probs[i].width, probs[i].height, probs[i].num_labels = w, h, L
        if isinstance(c, Pair):
            pairs.append(c.c())
            probs[i].cost = None
            probs[i].pair = ctypes.pointer(pairs[-1])
        else:
            probs[i].cost = c.data_ptr()
        probs[i].disparity = disps[i].data_ptr() if disps[i] is not None else None
        probs[i].soft_disparity = softs[i].data_ptr() if softs[i] is not None else None
        probs[i].messages_out = msgs[i].data_ptr() if msgs[i] is not None else None
    probs._pairs = pairs
    return probs


def workspace_bytes(costs, params: BPParams) -> int:
    costs = list(costs)
    probs = _problems(costs, [None] * len(costs), [None] * len(costs), [None] * len(costs))
    p = params.c()
    return _abi.lib().bp_workspace_size(probs, len(costs), ctypes.byref(p))


def run(costs, params: BPParams, *, want_disp: bool = True, want_soft: bool = False, want_msgs: bool = False,
        workspace: Workspace | None = None, checkpoints: torch.Tensor | None = None, outputs=None,
        stream=None):
    """Hierarchical checkerboard BP on one cost volume [L][H][W] (or a
    ``Pair``), or on a list of them.

    Returns a dict (or a list of dicts for a list input) with ``disp`` (int32
    [H][W]), ``soft`` (float32 [H][W]) and ``msgs`` (float32 [4][L][H][W]).
    ``outputs`` may pass preallocated dicts of the same form.
    """
    single, costs, outputs, probs, p = _run_args(costs, params, want_disp, want_soft, want_msgs, outputs)
    lib = _abi.lib()
    nbytes = lib.bp_workspace_size(probs, len(costs), ctypes.byref(p))
    if nbytes == 0:
        raise ValueError("bp_workspace_size rejected the problem description")
    ws = (workspace or _default_ws).get(nbytes, costs[0].device)
    ck_ptr, ck_bytes = _ckpt(checkpoints)
    st = lib.bp_run(probs, len(costs), ctypes.byref(p), _ptr(ws), nbytes, ck_ptr, ck_bytes, _stream(stream))
    _abi.check("bp_run", st)
    outs = [{k: v for k, v in o.items() if v is not None} for o in outputs]
    return outs[0] if single else outs


def run_noalloc(costs, params: BPParams, *, want_disp: bool = True, want_soft: bool = False,
                want_msgs: bool = False, checkpoints: torch.Tensor | None = None, outputs=None, stream=None):
    """``run`` through bp_run_noalloc: the library's fixed per-GPU scratch
    array replaces the workspace, so the call allocates no device memory when
    ``outputs`` (and ``checkpoints``, if any) are passed in."""
    single, costs, outputs, probs, p = _run_args(costs, params, want_disp, want_soft, want_msgs, outputs)
    ck_ptr, ck_bytes = _ckpt(checkpoints)
    st = _abi.lib().bp_run_noalloc(probs, len(costs), ctypes.byref(p), ck_ptr, ck_bytes, _stream(stream))
    _abi.check("bp_run_noalloc", st)
    outs = [{k: v for k, v in o.items() if v is not None} for o in outputs]
    return outs[0] if single else outs


def _ckpt(checkpoints):
    if checkpoints is None:
        return None, 0
    _need_gpu(checkpoints)
    return _ptr(checkpoints), checkpoints.numel() * checkpoints.element_size()


def _run_args(costs, params, want_disp, want_soft, want_msgs, outputs):
    """Problem descriptors and output tensors of a run call."""
    single = isinstance(costs, (torch.Tensor, Pair))
    costs = [costs] if single else list(costs)
    for c in costs:
        if isinstance(c, Pair):
            continue
        _need_gpu(c)
        if c.dtype != torch.float32 or c.dim() != 3:
            raise ValueError("cost volumes must be float32 [L][H][W]")
    dev = costs[0].device
    if outputs is None:
        outputs = []
        for c in costs:
            L, h, w = c.shape
            outputs.append({
                "disp": torch.empty((h, w), dtype=torch.int32, device=dev) if want_disp else None,
                "soft": torch.empty((h, w), dtype=torch.float32, device=dev) if want_soft else None,
                "msgs": torch.empty((4, L, h, w), dtype=torch.float32, device=dev) if want_msgs else None,
            })
    else:
        if len(outputs) != len(costs):
            raise ValueError("outputs must hold one dict per problem")
        for c, o in zip(costs, outputs):
            L, h, w = c.shape
            for key, dt, shape in (("disp", torch.int32, (h, w)), ("soft", torch.float32, (h, w)),
                                   ("msgs", torch.float32, (4, L, h, w))):
                t = o.get(key)
                if t is None:
                    continue
                _need_gpu(t)
                if t.device != dev or t.dtype != dt or tuple(t.shape) != shape or not t.is_contiguous():
                    raise ValueError(f"outputs['{key}'] must be a contiguous {dt} tensor of shape {shape} on {dev}")
    probs = _problems(costs, [o.get("disp") for o in outputs], [o.get("soft") for o in outputs],
                      [o.get("msgs") for o in outputs])
    return single, costs, outputs, probs, params.c()


def checkpoint_bytes(costs, params: BPParams) -> int:
    """Bytes of the checkpoint buffer a forward call with checkpoint_every > 0 fills."""
    costs = [costs] if isinstance(costs, torch.Tensor) else list(costs)
    probs = _problems(costs, [None] * len(costs), [None] * len(costs), [None] * len(costs))
    p = params.c()
    return _abi.lib().bp_checkpoint_size(probs, len(costs), ctypes.byref(p))


def backward(costs, params: BPParams, checkpoints: torch.Tensor, grad_soft, workspace: Workspace | None = None,
             stream=None, grad_out: torch.Tensor | None = None):
    """Gradient of sum(grad_soft * soft_disparity) with respect to the cost
    volumes, lambda and tau, from the checkpoints of a forward ``run`` with the
    same costs and params.  ``grad_soft`` is a tensor [H][W] (or a list).
    ``grad_out`` may pass a contiguous float32 tensor holding every cost
    gradient back to back (e.g. [B][L][H][W] for a batch of equal volumes).
    Returns (grad_costs (tensor or list, views of grad_out when given),
    grad_lambda [1], grad_tau [1])."""
    single = isinstance(costs, torch.Tensor)
    costs = [costs] if single else list(costs)
    grads_soft = [grad_soft] if single else list(grad_soft)
    dev = costs[0].device
    for c, g in zip(costs, grads_soft):
        _need_gpu(c, g)
    gs = torch.cat([g.reshape(-1).float() for g in grads_soft]).contiguous()
    total = sum(c.numel() for c in costs)
    if grad_out is None:
        gc = torch.empty(total, dtype=torch.float32, device=dev)
    else:
        _need_gpu(grad_out)
        if grad_out.dtype != torch.float32 or not grad_out.is_contiguous() or grad_out.numel() != total:
            raise ValueError("grad_out must be a contiguous float32 tensor with one entry per cost entry")
        gc = grad_out.view(-1)
    gl = torch.empty(1, dtype=torch.float32, device=dev)
    gt = torch.empty(1, dtype=torch.float32, device=dev)
    probs = _problems(costs, [None] * len(costs), [None] * len(costs), [None] * len(costs))
    p = params.c()
    lib = _abi.lib()
    nbytes = lib.bp_backward_workspace_size(probs, len(costs), ctypes.byref(p))
    if nbytes == 0:
        raise ValueError("bp_backward_workspace_size rejected the problem description")
    ws = (workspace or Workspace()).get(nbytes, dev)
    st = lib.bp_backward(probs, len(costs), ctypes.byref(p), _ptr(checkpoints),
                         checkpoints.numel() * checkpoints.element_size(), _ptr(gs), _ptr(gc), _ptr(gl), _ptr(gt),
                         _ptr(ws), nbytes, _stream(stream))
    _abi.check("bp_backward", st)
    outs, off = [], 0
    for c in costs:
        outs.append(gc[off:off + c.numel()].view(c.shape))
        off += c.numel()
    return (outs[0] if single else outs), gl, gt


def upsample(disp_lo: torch.Tensor, guide: torch.Tensor, sigma_s: float = 8.0, sigma_r: float = 12.0,
             radius: int = -1, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Joint bilateral upsampling (Eq. 2) -> float32 [H][W] in low-res label units."""
    _need_gpu(disp_lo, guide)
    if disp_lo.dtype != torch.int32 or guide.dtype != torch.uint8:
        raise ValueError("disp_lo must be int32 and guide u8")
    hl, wl = disp_lo.shape
    w, h, c = _img_dims(guide)
    if out is None:
        out = torch.empty((h, w), dtype=torch.float32, device=guide.device)
    st = _abi.lib().bp_upsample(_ptr(disp_lo), wl, hl, _ptr(guide), w, h, c, w * c, float(sigma_s),
                                float(sigma_r), int(radius), _ptr(out), _stream(stream))
    _abi.check("bp_upsample", st)
    return out


def _records(raw: torch.Tensor):
    """(x, y, value) views of an array of {int32 x, y; int64 value} records."""
    v = raw.view(torch.int32).view(-1, 4)
    return v[:, 0], v[:, 1], v[:, 2:4].contiguous().view(torch.int64).view(-1)


def harris(img: torch.Tensor, grid: int = 30, threshold: int = 0, stream=None):
    """Harris response (25 R, int64 [H][W]) and per-cell corners of a grey u8
    frame (Eq. 4-5).  Returns a dict: response, x, y, corner_response (the
    last three with grid*grid entries, x = -1 for a cell without a corner)."""
    _need_gpu(img)
    if img.dtype != torch.uint8 or img.dim() != 2:
        raise ValueError("harris works on grey u8 [H][W] frames")
    h, w = img.shape
    resp = torch.empty((h, w), dtype=torch.int64, device=img.device)
    raw = torch.empty((grid * grid, 2), dtype=torch.int64, device=img.device)
    st = _abi.lib().bp_harris(_ptr(img), w, h, w, int(grid), int(threshold), _ptr(resp), _ptr(raw), _stream(stream))
    _abi.check("bp_harris", st)
    x, y, r = _records(raw)
    return {"response": resp, "x": x, "y": y, "corner_response": r, "raw": raw}


def zssd_match(a: torch.Tensor, b: torch.Tensor, corners_raw: torch.Tensor, patch_radius: int = 5,
               search_radius: int = 16, stream=None):
    """ZSSD matches in frame b of the corners (the `raw` records from harris)
    of frame a.  Returns a dict: x, y, cost (n * ZSSD), x = -1 when none."""
    _need_gpu(a, b, corners_raw)
    if a.dtype != torch.uint8 or b.shape != a.shape or a.dim() != 2:
        raise ValueError("zssd_match works on two grey u8 [H][W] frames of one size")
    h, w = a.shape
    n = corners_raw.numel() * corners_raw.element_size() // 16
    raw = torch.empty((n, 2), dtype=torch.int64, device=a.device)
    st = _abi.lib().bp_zssd_match(_ptr(a), _ptr(b), w, h, w, _ptr(corners_raw), n, int(patch_radius),
                                  int(search_radius), _ptr(raw), _stream(stream))
    _abi.check("bp_zssd_match", st)
    x, y, c = _records(raw)
    return {"x": x, "y": y, "cost": c}


def icp(src: torch.Tensor, dst: torch.Tensor, pose: torch.Tensor, iters: int = 30, dmax: float = 1.0,
        want_corr: bool = False, workspace: Workspace | None = None, stream=None):
    """Point-to-point ICP of float32 [n][3] onto [m][3] from the float64 pose
    [12] (R row-major, T).  Returns a dict: pose (float64 [12]), rms (float64
    [iters]), pairs (int32 [iters]) and, if asked, corr (int32 [n])."""
    _need_gpu(src, dst, pose)
    if src.dtype != torch.float32 or dst.dtype != torch.float32 or pose.dtype != torch.float64:
        raise ValueError("points must be float32 [N][3] and the pose float64 [12]")
    if src.dim() != 2 or src.shape[1] != 3 or dst.dim() != 2 or dst.shape[1] != 3 or pose.numel() != 12:
        raise ValueError("points must be float32 [N][3] and the pose float64 [12]")
    n, m = src.shape[0], dst.shape[0]
    lib = _abi.lib()
    nbytes = lib.bp_icp_workspace_size(n, m)
    ws = (workspace or Workspace()).get(nbytes, src.device)
    dev = src.device
    out = {"pose": torch.empty(12, dtype=torch.float64, device=dev),
           "rms": torch.empty(max(iters, 1), dtype=torch.float64, device=dev),
           "pairs": torch.empty(max(iters, 1), dtype=torch.int32, device=dev)}
    if want_corr:
        out["corr"] = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    st = lib.bp_icp(_ptr(src), n, _ptr(dst), m, _ptr(pose), int(iters), float(dmax), _ptr(out["pose"]),
                    _ptr(out["rms"]), _ptr(out["pairs"]), _ptr(out["corr"]) if want_corr else None, _ptr(ws),
                    nbytes, _stream(stream))
    _abi.check("bp_icp", st)
    out["rms"], out["pairs"] = out["rms"][:iters], out["pairs"][:iters]
    if want_corr:
        out["corr"] = out["corr"][:n]
    return out


@dataclass
class Intrinsics:
    """Distorted-frame intrinsics (pixels) with radial coefficients only."""
    fx: float
    fy: float
    cx: float
    cy: float
    k1: float = 0.0
    k2: float = 0.0
    k3: float = 0.0

    def c(self):
        return _abi.BpIntrinsics(self.fx, self.fy, self.cx, self.cy, self.k1, self.k2, self.k3)


def undistort(img: torch.Tensor, intrinsics: Intrinsics, out: torch.Tensor | None = None, stream=None):
    """Radial-only undistortion with bilinear sampling of a u8 [H][W] or [H][W][3] frame."""
    _need_gpu(img)
    if img.dtype != torch.uint8:
        raise ValueError("undistort works on u8 images")
    w, h, c = _img_dims(img)
    if out is None:
        out = torch.empty_like(img)
    _need_gpu(out)
    K = intrinsics.c()
    st = _abi.lib().bp_undistort(_ptr(img), w, h, c, w * c, ctypes.byref(K), _ptr(out), w * c, _stream(stream))
    _abi.check("bp_undistort", st)
    return out


@dataclass
class Camera:
    """Pinhole camera of the full-resolution frame (Eq. 3): baseline B, focal
    length f and pixel pitch du, dv in one length unit, principal point (u0, v0)
    in pixels."""
    baseline: float
    focal: float
    du: float
    dv: float
    u0: float
    v0: float

    def c(self):
        return _abi.BpCamera(self.baseline, self.focal, self.du, self.dv, self.u0, self.v0)


def upsample_points(disp_lo: torch.Tensor, guide: torch.Tensor, camera: Camera, sigma_s: float = 8.0,
                    sigma_r: float = 12.0, radius: int = -1, want_disp: bool = True, out=None, stream=None):
    """Joint bilateral upsampling fused with triangulation (Eq. 2 + Eq. 3).
    Returns (disp_hi float32 [H][W] or None, points float32 [H][W][3])."""
    _need_gpu(disp_lo, guide)
    if disp_lo.dtype != torch.int32 or guide.dtype != torch.uint8:
        raise ValueError("disp_lo must be int32 and guide u8")
    hl, wl = disp_lo.shape
    w, h, c = _img_dims(guide)
    disp_hi, pts = out if out is not None else (None, None)
    if want_disp and disp_hi is None:
        disp_hi = torch.empty((h, w), dtype=torch.float32, device=guide.device)
    if pts is None:
        pts = torch.empty((h, w, 3), dtype=torch.float32, device=guide.device)
    cam = camera.c()
    st = _abi.lib().bp_upsample_points(_ptr(disp_lo), wl, hl, _ptr(guide), w, h, c, w * c, float(sigma_s),
                                       float(sigma_r), int(radius), ctypes.byref(cam),
                                       _ptr(disp_hi) if want_disp else None, _ptr(pts), _stream(stream))
    _abi.check("bp_upsample_points", st)
    return (disp_hi if want_disp else None), pts


def variant_count(num_labels: int) -> int:
    return _abi.lib().bp_variant_count(num_labels)
