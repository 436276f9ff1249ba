"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Integer-valued inputs (u8 images, integer truncation, lambda and lambda*tau)
keep every BP quantity an integer below 2^24, so FP32 on the GPU must equal
the FP64 oracle bit for bit: cost volumes, messages and labels.  Real-valued
inputs use the stated tolerances: max |message error| <= 1e-4 * lambda * tau
and at most 0.5% of pixels whose label differs by more than one.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import aerial, slanted_planes, workload

pytestmark = pytest.mark.gpu

MSG_TOL_REL = 1e-4        # max message error relative to lambda*tau (real-valued inputs)
BAD_PIXEL_MAX = 0.005     # fraction of pixels off by more than one label


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1902_09733_amd as bp
    bp.stereo._abi.lib()
    return torch.device("cuda:0")


def bp_mod():
    import paper_1902_09733_amd as bp
    return bp


def gpu_run(cost_np, dev, **kw):
    bp = bp_mod()
    want_soft = kw.pop("want_soft", False)
    p = bp.BPParams(**kw)
    c = torch.from_numpy(np.ascontiguousarray(cost_np, dtype=np.float32)).to(dev)
    out = bp.run(c, p, want_disp=True, want_soft=want_soft, want_msgs=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def oracle_run(cost_np, levels, iters, lam, tau, **kw):
    return oracle.run(np.asarray(cost_np, dtype=np.float64), levels, iters, lam, tau, want_msgs=True, **kw)


def assert_exact(g, o, what=""):
    np.testing.assert_array_equal(g["disp"], o["disp"], err_msg=f"labels {what}")
    np.testing.assert_array_equal(g["msgs"].astype(np.float64), o["msgs"], err_msg=f"messages {what}")


def int_cost(w, h, L, seed, rgb=True):
    left, right, _ = aerial(w, h, L, seed, channels=3 if rgb else 1)
    return oracle.cost_volume(left, right, L, 20.0)


# ---------------------------------------------------------------- a1, a2

def test_cost_volume_grey_exact(dev):
    bp = bp_mod()
    w = workload("planes160x120_L32")
    g = bp.cost_volume(torch.from_numpy(w["left"]).to(dev), torch.from_numpy(w["right"]).to(dev), 32, 20.0)
    o = oracle.cost_volume(w["left"], w["right"], 32, 20.0)
    np.testing.assert_array_equal(g.cpu().numpy().astype(np.float64), o)


@pytest.mark.parametrize("rgb_mode", [0, 1])
@pytest.mark.parametrize("L", [7, 64, 130])
def test_cost_volume_rgb_downsampled(dev, rgb_mode, L):
    bp = bp_mod()
    left, right, _ = aerial(332, 236, 40, 11, channels=3, disparity_scale=4.0)
    g = bp.cost_volume(torch.from_numpy(left).to(dev), torch.from_numpy(right).to(dev), L, 20.0,
                       downsample=4, rgb_mode=rgb_mode)
    o = oracle.cost_volume(oracle.downsample(left, 4), oracle.downsample(right, 4), L, 20.0, rgb_mode=rgb_mode)
    # Mode 1 computes the exact channel mean rounded once to FP32.
    np.testing.assert_array_equal(g.cpu().numpy(), o.astype(np.float32))


@pytest.mark.parametrize("shape", [(16, 12, 1), (44, 20, 3), (2704, 1520, 3)])
def test_downsample_exact(dev, shape):
    bp = bp_mod()
    w, h, c = shape
    rng = np.random.default_rng(w)
    img = rng.integers(0, 256, size=(h, w, c) if c == 3 else (h, w), dtype=np.uint8)
    g = bp.downsample(torch.from_numpy(img).to(dev), 4)
    np.testing.assert_array_equal(g.cpu().numpy(), oracle.downsample(img, 4))


# ---------------------------------------------------------------- a3-a6, integer exactness

@pytest.mark.parametrize("variant,pm_from", [(0, -1), (1, 1), (2, 1), (3, 1), (0, 0)])
def test_planes160_exact(dev, variant, pm_from):
    w = workload("planes160x120_L32")
    cost = oracle.cost_volume(w["left"], w["right"], 32, 20.0)
    o = oracle_run(cost, 1, 10, 10.0, 2.0)
    g = gpu_run(cost, dev, levels=1, iters=10, lam=10.0, tau=2.0, variant=variant, pm_from=pm_from)
    assert_exact(g, o, f"variant {variant} pm_from {pm_from}")


@pytest.mark.parametrize("w,h,L,levels", [
    (77, 53, 16, 3), (77, 53, 32, 4), (64, 48, 48, 3), (101, 67, 64, 5), (45, 31, 96, 3),
    (58, 39, 128, 4), (33, 21, 100, 2), (29, 17, 200, 2), (19, 23, 256, 2), (40, 30, 2, 3),
    (37, 25, 5, 2), (24, 16, 17, 2),
])
def test_multilevel_exact(dev, w, h, L, levels):
    cost = int_cost(w, h, L, w * 7 + L)
    o = oracle_run(cost, levels, 6, 10.0, 2.0)
    # Every label-major kernel variant, and every split between label-major
    # and pixel-major levels.
    for variant in range(bp_mod().variant_count(L) + 1):
        g = gpu_run(cost, dev, levels=levels, iters=6, lam=10.0, tau=2.0, variant=variant, pm_from=levels)
        assert_exact(g, o, f"{w}x{h} L{L} n{levels} v{variant} label-major")
    for pm_from in range(levels):
        g = gpu_run(cost, dev, levels=levels, iters=6, lam=10.0, tau=2.0, pm_from=pm_from)
        assert_exact(g, o, f"{w}x{h} L{L} n{levels} pixel-major from {pm_from}")
    # Every pixel-major kernel variant at every level.
    for variant in range(1, bp_mod().variant_count(L) + 1):
        g = gpu_run(cost, dev, levels=levels, iters=6, lam=10.0, tau=2.0, variant=variant, pm_from=0)
        assert_exact(g, o, f"{w}x{h} L{L} n{levels} v{variant} pixel-major")


@pytest.mark.parametrize("K", [0, 1, 2, 3, 7])
@pytest.mark.parametrize("levels", [1, 2, 3])
def test_iteration_counts_exact(dev, K, levels):
    cost = int_cost(41, 27, 32, 5)
    o = oracle_run(cost, levels, K, 10.0, 2.0)
    for pm_from in sorted({0, levels - 1, levels}):
        g = gpu_run(cost, dev, levels=levels, iters=K, lam=10.0, tau=2.0, pm_from=pm_from)
        assert_exact(g, o, f"K{K} n{levels} pm_from {pm_from}")


@pytest.mark.parametrize("w,h", [(1, 1), (1, 9), (9, 1), (2, 2), (3, 5), (2, 7), (130, 1), (1, 70)])
def test_degenerate_grids_exact(dev, w, h):
    rng = np.random.default_rng(w * 100 + h)
    cost = rng.integers(0, 21, size=(16, h, w)).astype(np.float64)
    levels = 3 if min(w, h) > 1 else 2
    o = oracle_run(cost, levels, 5, 10.0, 2.0)
    for pm_from in (0, levels):
        g = gpu_run(cost, dev, levels=levels, iters=5, lam=10.0, tau=2.0, pm_from=pm_from)
        assert_exact(g, o, f"{w}x{h} pm_from {pm_from}")


@pytest.mark.parametrize("lam,tau", [(0.0, 2.0), (10.0, 0.5), (3.0, 40.0), (1.0, 3.0)])
def test_parameter_edges_exact(dev, lam, tau):
    cost = int_cost(50, 34, 32, 3)
    o = oracle_run(cost, 3, 6, lam, tau)
    for pm_from in (0, 3):
        g = gpu_run(cost, dev, levels=3, iters=6, lam=lam, tau=tau, pm_from=pm_from)
        assert_exact(g, o, f"lam {lam} tau {tau} pm_from {pm_from}")


@pytest.mark.parametrize("L", [64, 128])
@pytest.mark.parametrize("lam,tau", [(2.0, 1.0), (2.0, 1.5), (1.0, 2.0), (2.0, 2.5), (1.0, 3.0), (2.0, 3.5)])
def test_transform_forms_exact(dev, L, lam, tau):
    """The truncated-linear transform's forms at 16 lanes per pixel: three
    labels (tau <= 2), five labels (2 < tau <= 3, four labels per lane) and the
    two-pass scans (tau > 3, or eight labels per lane), on integer costs with
    dyadic lambda and tau, where every form is exact: bit-exact against the
    oracle's sequential two-pass transform."""
    cost = int_cost(44, 30, L, 7)
    o = oracle_run(cost, 2, 4, lam, tau)
    g = gpu_run(cost, dev, levels=2, iters=4, lam=lam, tau=tau)
    assert_exact(g, o, f"L {L} lam {lam} tau {tau}")
    g1 = gpu_run(cost, dev, levels=2, iters=3, lam=lam, tau=tau)
    assert_exact(g1, oracle_run(cost, 2, 3, lam, tau), f"L {L} lam {lam} tau {tau} K 3")


# ---------------------------------------------------------------- real-valued inputs

def real_case(w=96, h=64, L=64, seed=3):
    left, right, _ = aerial(w, h, L, seed, channels=3)
    cost = oracle.cost_volume(left, right, L, 20.0, rgb_mode=1)
    rng = np.random.default_rng(seed)
    cost = (cost + rng.uniform(0.0, 0.5, size=cost.shape)).astype(np.float32).astype(np.float64)
    return cost


@pytest.mark.parametrize("levels,pm_from,variant", [(1, 1, 0), (3, 3, 0), (1, 0, 0), (3, 1, 0), (1, 0, 3), (3, 0, 4)])
def test_real_valued_tolerance(dev, levels, pm_from, variant):
    lam, tau = 7.3, 2.6
    cost = real_case()
    o = oracle_run(cost, levels, 8, lam, tau)
    g = gpu_run(cost, dev, levels=levels, iters=8, lam=lam, tau=tau, pm_from=pm_from, variant=variant)
    err = np.abs(g["msgs"].astype(np.float64) - o["msgs"]).max()
    assert err <= MSG_TOL_REL * lam * tau, err
    bad = (np.abs(g["disp"] - o["disp"]) > 1).mean()
    assert bad <= BAD_PIXEL_MAX, bad


@pytest.mark.parametrize("pm_from", [0, 1])
def test_soft_argmin(dev, pm_from):
    lam, tau, T = 7.3, 2.6, 0.5
    cost = real_case(64, 48, 32, 9)
    o = oracle_run(cost, 1, 6, lam, tau, want_soft=True, temperature=T)
    g = gpu_run(cost, dev, levels=1, iters=6, lam=lam, tau=tau, temperature=T, want_soft=True, pm_from=pm_from)
    # Soft-argmin of beliefs within 1e-4*lambda*tau of the oracle's; the
    # readout's label-space error is then bounded by L * that / T (loose).
    err = np.abs(g["soft"].astype(np.float64) - o["soft"]).max()
    assert err <= 2e-3, err
    np.testing.assert_array_equal(g["disp"], o["disp"])


# ---------------------------------------------------------------- precision form

@pytest.mark.parametrize("pm_from", [0, 2, 4])
@pytest.mark.parametrize("fmt,mode", [("f16", oracle.STORE_F16), ("bf16", oracle.STORE_BF16)])
def test_16bit_messages_integer_exact(dev, fmt, mode, pm_from):
    cost = int_cost(88, 50, 64, 21)
    o = oracle_run(cost, 4, 6, 10.0, 2.0, store_mode=mode)
    g = gpu_run(cost, dev, levels=4, iters=6, lam=10.0, tau=2.0, msg_dtype=fmt, pm_from=pm_from)
    assert_exact(g, o, f"{fmt} pm_from {pm_from}")


@pytest.mark.parametrize("fmt,mode", [("f16", oracle.STORE_F16), ("bf16", oracle.STORE_BF16)])
def test_16bit_messages_real(dev, fmt, mode):
    lam, tau = 7.3, 2.6
    cost = real_case(96, 64, 64, 5)
    o16 = oracle_run(cost, 3, 8, lam, tau, store_mode=mode)
    o64 = oracle_run(cost, 3, 8, lam, tau)
    ulp = 2.0 ** -10 if fmt == "f16" else 2.0 ** -7
    for pm_from in (0, 3):
        g = gpu_run(cost, dev, levels=3, iters=8, lam=lam, tau=tau, msg_dtype=fmt, pm_from=pm_from)
        err = np.abs(g["msgs"].astype(np.float64) - o16["msgs"]).max()
        # Within a few storage ulps of the emulated-storage oracle.
        assert err <= 8 * ulp * lam * tau, (pm_from, err)
        assert (np.abs(g["disp"] - o64["disp"]) > 1).mean() <= BAD_PIXEL_MAX


# ---------------------------------------------------------------- a7

@pytest.mark.parametrize("s,R,ch", [(4, 4, 3), (2, 3, 1), (1, 2, 3), (3, 5, 3), (5, 8, 3), (17, 1, 3), (20, 0, 1)])
def test_upsample_parity(dev, s, R, ch):
    bp = bp_mod()
    wl, hl = 37, 23
    rng = np.random.default_rng(s * 10 + R)
    disp = rng.integers(0, 64, size=(hl, wl)).astype(np.int32)
    guide = rng.integers(0, 256, size=(hl * s, wl * s, 3) if ch == 3 else (hl * s, wl * s), dtype=np.uint8)
    g = bp.upsample(torch.from_numpy(disp).to(dev), torch.from_numpy(guide).to(dev), 8.0, 12.0, R)
    o = oracle.upsample(disp, guide, 8.0, 12.0, R)
    err = np.abs(g.cpu().numpy().astype(np.float64) - o).max()
    assert err <= 2e-3, err


@pytest.mark.parametrize("s,R,ch,sigma_r", [(4, 4, 3, 12.0), (3, 2, 1, 12.0), (2, 3, 3, 1.0)])
def test_upsample_far_colours(dev, s, R, ch, sigma_r):
    """Pixels whose guide colour is far from every tap in their window: every
    weight underflows relative to exponent 0 and the kernel re-evaluates them
    relative to their largest exponent; the sample pixels themselves take the
    ordinary path in the same launch."""
    bp = bp_mod()
    wl, hl = 29, 19
    rng = np.random.default_rng(100 + s * 10 + R)
    disp = rng.integers(0, 64, size=(hl, wl)).astype(np.int32)
    shape = (hl * s, wl * s) + ((3,) if ch == 3 else ())
    guide = rng.integers(200, 256, size=shape, dtype=np.uint8)
    guide[s // 2::s, s // 2::s] = rng.integers(0, 8, size=guide[s // 2::s, s // 2::s].shape, dtype=np.uint8)
    g = bp.upsample(torch.from_numpy(disp).to(dev), torch.from_numpy(guide).to(dev), 8.0, sigma_r, R)
    o = oracle.upsample(disp, guide, 8.0, sigma_r, R)
    gn = g.cpu().numpy().astype(np.float64)
    assert np.isfinite(gn).all()
    err = np.abs(gn - o).max()
    assert err <= 2e-3, err


# ---------------------------------------------------------------- full-size pair, bench configuration

@pytest.fixture(scope="module")
def aerial_full():
    w = workload("aerial2704x1520_s4_L64")
    l4, r4 = oracle.downsample(w["left"], 4), oracle.downsample(w["right"], 4)
    cost = oracle.cost_volume(l4, r4, 64, 20.0)
    o = oracle.run(cost, 5, 10, 10.0, 2.0, want_msgs=True)
    return w, cost, o


def test_aerial_full_pipeline_exact(dev, aerial_full):
    """The benchmarked pair end to end: cost, 5-level BP, readout, upsampling."""
    bp = bp_mod()
    w, cost, o = aerial_full
    left = torch.from_numpy(w["left"]).to(dev)
    right = torch.from_numpy(w["right"]).to(dev)
    c = bp.cost_volume(left, right, 64, 20.0, downsample=4)
    np.testing.assert_array_equal(c.cpu().numpy().astype(np.float64), cost)
    for pm_from in (0, 5):
        out = bp.run(c, bp.BPParams(levels=5, iters=10, lam=10.0, tau=2.0, pm_from=pm_from), want_msgs=True)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in out.items()}
        assert_exact(g, o, f"aerial full pm_from {pm_from}")
        del out, g
        # The same problem with the data term computed inside bp_run from the pair.
        out = bp.run(bp.Pair(left, right, 64, 20.0, downsample=4),
                     bp.BPParams(levels=5, iters=10, lam=10.0, tau=2.0, pm_from=pm_from), want_msgs=True)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in out.items()}
        assert_exact(g, o, f"aerial full from the pair, pm_from {pm_from}")
        del out, g
    out = bp.run(c, bp.BPParams(levels=5, iters=10, lam=10.0, tau=2.0), want_msgs=True)
    up = bp.upsample(out["disp"], left, 8.0, 12.0, -1)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    assert_exact(g, o, "aerial full")
    # Upsampling against the oracle on every 97th row of the 4.1 M-pixel frame.
    rows = np.arange(0, 1520, 97)
    ref = oracle.upsample(o["disp"], w["left"], 8.0, 12.0)
    err = np.abs(up.cpu().numpy()[rows].astype(np.float64) - ref[rows]).max()
    assert err <= 2e-3, err


# ---------------------------------------------------------------- triangulation (Eq. 3)

CAM = dict(baseline=0.5, focal=3.0e-3, du=1.5e-6, dv=1.6e-6, u0=1352.0, v0=760.0)


@pytest.mark.parametrize("s,R,ch", [(4, -1, 3), (2, 3, 1), (3, 0, 3)])
def test_upsample_points(dev, s, R, ch):
    """The fused epilogue: the disparity equals bp_upsample's bit for bit, the
    points equal the oracle's Eq. 3 applied to that disparity (FP32 rounding:
    a few ulps), and zero disparities give NaN."""
    bp = bp_mod()
    wl, hl = 61, 37
    rng = np.random.default_rng(s * 10 + ch)
    d_lo = rng.integers(0, 40, size=(hl, wl)).astype(np.int32)
    d_lo[:20, :20] = 0          # a region whose windows see only zero disparity
    shape = (hl * s, wl * s) + ((3,) if ch == 3 else ())
    guide_np = rng.integers(0, 256, size=shape, dtype=np.uint8)
    dl, guide = torch.from_numpy(d_lo).to(dev), torch.from_numpy(guide_np).to(dev)
    cam = bp.Camera(**CAM)
    up = bp.upsample(dl, guide, 8.0, 12.0, R)
    disp_hi, pts = bp.upsample_points(dl, guide, cam, 8.0, 12.0, R)
    _, pts2 = bp.upsample_points(dl, guide, cam, 8.0, 12.0, R, want_disp=False)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(disp_hi.cpu().numpy(), up.cpu().numpy())
    np.testing.assert_array_equal(pts2.cpu().numpy(), pts.cpu().numpy())
    g = pts.cpu().numpy().astype(np.float64)
    ref = oracle.triangulate(disp_hi.cpu().numpy().astype(np.float64), s, **CAM)
    np.testing.assert_allclose(g, ref, rtol=2e-6, atol=1e-9)
    zero = disp_hi.cpu().numpy() <= 0
    assert zero.any() and np.isnan(g[zero]).all() and np.isfinite(g[~zero]).all()


# ---------------------------------------------------------------- data term from the pair

@pytest.mark.parametrize("w,h,ch,s,mode,L,pm_from", [
    (160, 96, 3, 4, 0, 64, 0), (160, 96, 3, 4, 1, 64, 0), (101, 37, 1, 1, 0, 48, 0),
    (202, 74, 3, 2, 0, 100, 1), (151, 90, 3, 1, 1, 32, 3), (77, 45, 1, 3, 0, 256, 0),
    (9, 5, 3, 2, 0, 7, 0), (40, 24, 3, 8, 0, 32, 0), (33, 20, 1, 8, 0, 17, 0), (35, 21, 1, 4, 0, 100, 0),
])
def test_pair_input_exact(dev, w, h, ch, s, mode, L, pm_from):
    """bp_run from a pair (data term written straight into the finest level's
    layout) equals bp_run on bp_cost_volume's volume bit for bit, and the
    oracle on integer costs."""
    bp = bp_mod()
    rng = np.random.default_rng(w * h + L)
    shp = (h * s, w * s) + ((3,) if ch == 3 else ())
    left_np = rng.integers(0, 256, size=shp, dtype=np.uint8)
    right_np = np.roll(left_np, 3, axis=1) // 2 + rng.integers(0, 128, size=shp, dtype=np.uint8)
    left, right = torch.from_numpy(left_np).to(dev), torch.from_numpy(right_np).to(dev)
    p = bp.BPParams(levels=3, iters=5, lam=10.0, tau=2.0, pm_from=pm_from)
    c = bp.cost_volume(left, right, L, 20.0, downsample=s, rgb_mode=mode)
    a = bp.run(c, p, want_msgs=True)
    b = bp.run(bp.Pair(left, right, L, 20.0, downsample=s, rgb_mode=mode), p, want_msgs=True)
    torch.cuda.synchronize()
    ga = {k: v.cpu().numpy() for k, v in a.items()}
    gb = {k: v.cpu().numpy() for k, v in b.items()}
    np.testing.assert_array_equal(gb["disp"], ga["disp"])
    np.testing.assert_array_equal(gb["msgs"], ga["msgs"])
    if mode == 0:
        lo, ro = (oracle.downsample(left_np, s), oracle.downsample(right_np, s)) if s > 1 else (left_np, right_np)
        o = oracle_run(oracle.cost_volume(lo, ro, L, 20.0), 3, 5, 10.0, 2.0)
        assert_exact(gb, o, f"pair {w}x{h}x{L} s{s}")


@pytest.mark.parametrize("trunc,levels", [(600.0, 3), (2048.0, 2), (2049.0, 2), (7.0, 6), (20.5, 3)])
def test_pair_input_truncations(dev, trunc, levels):
    """The pair route with large, boundary and non-integral truncations and
    deep pyramids (pyramid sums up to 4^5 * 7): bit-exact for integral
    truncations, within tolerance otherwise."""
    bp = bp_mod()
    w, h, s, L = 70, 44, 2, 40
    rng = np.random.default_rng(int(trunc) + levels)
    left_np = rng.integers(0, 256, size=(h * s, w * s), dtype=np.uint8)
    right_np = np.roll(left_np, 4, axis=1)
    right_np = np.clip(right_np.astype(int) + rng.integers(-3, 4, size=right_np.shape), 0, 255).astype(np.uint8)
    left, right = torch.from_numpy(left_np).to(dev), torch.from_numpy(right_np).to(dev)
    p = bp.BPParams(levels=levels, iters=4, lam=10.0, tau=2.0)
    out = bp.run(bp.Pair(left, right, L, trunc, downsample=s), p, want_msgs=True)
    torch.cuda.synchronize()
    cost = oracle.cost_volume(oracle.downsample(left_np, s), oracle.downsample(right_np, s), L, trunc)
    o = oracle_run(cost, levels, 4, 10.0, 2.0)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    if trunc == int(trunc):
        assert_exact(g, o, f"pair trunc {trunc}")
    else:
        np.testing.assert_array_equal(g["disp"], o["disp"])
        assert np.abs(g["msgs"] - o["msgs"]).max() <= MSG_TOL_REL * 10.0 * 2.0


@pytest.mark.parametrize("trunc", [20.0, 20.5, 20.3, 300.0, 65504.0, 70000.0, 0.0])
@pytest.mark.parametrize("ch,mode,L", [(1, 0, 24), (3, 0, 24), (3, 1, 24), (3, 0, 96)])
def test_pair_cost_storage_invisible(dev, trunc, ch, mode, L):
    """On the pair route the finest level may keep its integer costs in bytes
    (an integral truncation of at most 255: 20, 0; four labels per lane), in
    FP16 (a truncation FP16 holds exactly: 20.5, 300, 65504, or 20 and 0 at 96
    labels, six per lane) or in FP32 (20.3, 70000, or the exact RGB mean);
    either way the messages, labels and soft-argmin disparities equal the
    volume route's, which is always FP32, bit for bit."""
    bp = bp_mod()
    w, h, s = 58, 34, 2
    rng = np.random.default_rng(int(trunc * 10) + 7 * ch + mode)
    shp = (h * s, w * s) + ((3,) if ch == 3 else ())
    left_np = rng.integers(0, 256, size=shp, dtype=np.uint8)
    right_np = np.roll(left_np, 3, axis=1) // 2 + rng.integers(0, 128, size=shp, dtype=np.uint8)
    left, right = torch.from_numpy(left_np).to(dev), torch.from_numpy(right_np).to(dev)
    for levels, K in ((3, 4), (2, 5)):
        p = bp.BPParams(levels=levels, iters=K, lam=3.5, tau=1.5)
        a = bp.run(bp.cost_volume(left, right, L, trunc, downsample=s, rgb_mode=mode), p, want_msgs=True,
                   want_soft=True)
        b = bp.run(bp.Pair(left, right, L, trunc, downsample=s, rgb_mode=mode), p, want_msgs=True, want_soft=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(b["disp"].cpu().numpy(), a["disp"].cpu().numpy())
        np.testing.assert_array_equal(b["soft"].cpu().numpy(), a["soft"].cpu().numpy())
        np.testing.assert_array_equal(b["msgs"].cpu().numpy(), a["msgs"].cpu().numpy())


def test_pair_input_unaligned_images(dev):
    """Images at an odd byte address take the byte-load downsampling path."""
    bp = bp_mod()
    w, h, s, L = 64, 36, 4, 48
    rng = np.random.default_rng(3)
    left_np = rng.integers(0, 256, size=(h * s, w * s, 3), dtype=np.uint8)
    right_np = np.roll(left_np, 5, axis=1)
    n = left_np.size
    buf = torch.empty(2 * n + 2, dtype=torch.uint8, device=dev)
    left = buf[1:1 + n].view(h * s, w * s, 3)
    right = buf[n + 2:].view(h * s, w * s, 3)
    left.copy_(torch.from_numpy(left_np))
    right.copy_(torch.from_numpy(right_np))
    assert left.data_ptr() % 4 != 0
    out = bp.run(bp.Pair(left, right, L, 20.0, downsample=s), bp.BPParams(levels=3, iters=5, lam=10.0, tau=2.0),
                 want_msgs=True)
    torch.cuda.synchronize()
    o = oracle_run(oracle.cost_volume(oracle.downsample(left_np, s), oracle.downsample(right_np, s), L, 20.0),
                   3, 5, 10.0, 2.0)
    assert_exact({k: v.cpu().numpy() for k, v in out.items()}, o, "unaligned pair")


def test_pair_and_volume_problems_batched(dev):
    """One batched call mixing pair-sourced problems and volumes."""
    bp = bp_mod()
    items, refs = [], []
    for i, (w, h, L) in enumerate([(60, 40, 32), (90, 50, 64), (33, 21, 96), (47, 29, 64)]):
        left_np, right_np, _ = aerial(2 * w, 2 * h, 2 * L, 40 + i, channels=3)
        lo, ro = oracle.downsample(left_np, 2), oracle.downsample(right_np, 2)
        cost = oracle.cost_volume(lo, ro, L, 20.0)
        refs.append(oracle_run(cost, 3, 6, 10.0, 2.0))
        if i % 2 == 0:
            items.append(bp.Pair(torch.from_numpy(left_np).to(dev), torch.from_numpy(right_np).to(dev), L, 20.0,
                                 downsample=2))
        else:
            items.append(torch.from_numpy(cost.astype(np.float32)).to(dev))
    outs = bp.run(items, bp.BPParams(levels=3, iters=6, lam=10.0, tau=2.0), want_msgs=True)
    torch.cuda.synchronize()
    for i, (og, o) in enumerate(zip(outs, refs)):
        assert_exact({k: v.cpu().numpy() for k, v in og.items()}, o, f"batched item {i}")


@pytest.mark.parametrize("truncs", [(20.0, 20.0, 20.0), (20.0, 300.0, 20.0), (20.0, 20.3, 20.0)])
def test_batched_pairs_cost_storage(dev, truncs):
    """A batched call of pair-sourced problems (fused pairs at every level)
    whose finest levels share the narrowest cost storage all of them allow:
    bytes (every truncation an integer <= 255, labels 32 / 64 / 128, four or
    eight per lane), FP16 (one truncation of 300) or FP32 (one of 20.3).  Each
    problem equals its own run on the FP32 volume route bit for bit, labels
    and messages, with an even and an odd number of pairs per level."""
    bp = bp_mod()
    shapes = [(60, 40, 32), (90, 50, 64), (47, 29, 128)]
    items, vols = [], []
    for i, ((w, h, L), t) in enumerate(zip(shapes, truncs)):
        left_np, right_np, _ = aerial(2 * w, 2 * h, 2 * L, 60 + i, channels=3)
        left, right = torch.from_numpy(left_np).to(dev), torch.from_numpy(right_np).to(dev)
        items.append(bp.Pair(left, right, L, t, downsample=2))
        vols.append(bp.cost_volume(left, right, L, t, downsample=2))
    for K in (4, 6):
        p = bp.BPParams(levels=3, iters=K, lam=10.0, tau=2.0)
        outs = bp.run(items, p, want_msgs=True)
        torch.cuda.synchronize()
        for i, v in enumerate(vols):
            ref = bp.run(v, p, want_msgs=True)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(outs[i]["disp"].cpu().numpy(), ref["disp"].cpu().numpy(),
                                          err_msg=f"problem {i} K {K}")
            np.testing.assert_array_equal(outs[i]["msgs"].cpu().numpy(), ref["msgs"].cpu().numpy(),
                                          err_msg=f"problem {i} K {K}")


# ---------------------------------------------------------------- batched form, kernel variants

BATCH_SHAPES = [(60, 40, 32), (90, 50, 64), (33, 21, 96), (120, 70, 128), (45, 35, 64), (17, 9, 16), (71, 45, 100)]


@pytest.mark.parametrize("fmt,mode", [("f32", oracle.STORE_F64), ("f16", oracle.STORE_F16)])
def test_batched_mixed_problems_exact(dev, fmt, mode):
    """Problems of uneven size and label count in one bp_run call (one launch
    per half-sweep and lane split) equal the oracle problem by problem."""
    bp = bp_mod()
    costs = [int_cost(w, h, L, w + h + L) for (w, h, L) in BATCH_SHAPES]
    vols = [torch.from_numpy(c.astype(np.float32)).to(dev) for c in costs]
    p = bp.BPParams(levels=3, iters=6, lam=10.0, tau=2.0, msg_dtype=fmt)
    outs = bp.run(vols, p, want_msgs=True)
    torch.cuda.synchronize()
    for c, o_gpu, shp in zip(costs, outs, BATCH_SHAPES):
        o = oracle_run(c, 3, 6, 10.0, 2.0, store_mode=mode)
        g = {k: v.cpu().numpy() for k, v in o_gpu.items()}
        assert_exact(g, o, f"batched {shp} {fmt}")


def test_batched_soft_readout(dev):
    """Batched problems with the soft-argmin readout (the last half-sweep
    then leaves the whole readout to the readout pass)."""
    bp = bp_mod()
    lam, tau, T = 7.3, 2.6, 0.5
    shapes = BATCH_SHAPES[:3]
    costs = [real_case(w, h, L, 11 + i) for i, (w, h, L) in enumerate(shapes)]
    vols = [torch.from_numpy(c.astype(np.float32)).to(dev) for c in costs]
    outs = bp.run(vols, bp.BPParams(levels=2, iters=5, lam=lam, tau=tau, temperature=T), want_soft=True)
    torch.cuda.synchronize()
    for c, og in zip(costs, outs):
        o = oracle_run(c, 2, 5, lam, tau, want_soft=True, temperature=T)
        assert np.abs(og["soft"].cpu().numpy() - o["soft"]).max() <= 2e-3
        assert (np.abs(og["disp"].cpu().numpy() - o["disp"]) > 1).mean() <= BAD_PIXEL_MAX


@pytest.mark.parametrize("K", [1, 2, 5])
def test_batched_iteration_counts(dev, K):
    bp = bp_mod()
    shapes = BATCH_SHAPES[:4]
    costs = [int_cost(w, h, L, 7 * w + L) for (w, h, L) in shapes]
    vols = [torch.from_numpy(c.astype(np.float32)).to(dev) for c in costs]
    outs = bp.run(vols, bp.BPParams(levels=2, iters=K, lam=10.0, tau=2.0), want_msgs=True)
    torch.cuda.synchronize()
    for c, o_gpu in zip(costs, outs):
        o = oracle_run(c, 2, K, 10.0, 2.0)
        assert_exact({k: v.cpu().numpy() for k, v in o_gpu.items()}, o, f"batched K{K}")


@pytest.mark.parametrize("L", [16, 17, 24, 32, 33, 48, 64, 96, 128])
@pytest.mark.parametrize("variant", [2, 3, 4, 5])
def test_pixel_major_variants_exact(dev, L, variant):
    cost = int_cost(53, 37, L, L + 1)
    o = oracle_run(cost, 3, 6, 10.0, 2.0)
    g = gpu_run(cost, dev, levels=3, iters=6, lam=10.0, tau=2.0, pm_from=0, variant=variant)
    assert_exact(g, o, f"L{L} pixel-major variant {variant}")


@pytest.mark.parametrize("variant", [3, 4, 5])
def test_batched_shuffled_sum_variants_exact(dev, variant):
    bp = bp_mod()
    costs = [int_cost(w, h, L, w + 3 * h + L) for (w, h, L) in BATCH_SHAPES]
    vols = [torch.from_numpy(c.astype(np.float32)).to(dev) for c in costs]
    outs = bp.run(vols, bp.BPParams(levels=3, iters=5, lam=10.0, tau=2.0, variant=variant, pm_from=0),
                  want_msgs=True)
    torch.cuda.synchronize()
    for c, o_gpu, shp in zip(costs, outs, BATCH_SHAPES):
        o = oracle_run(c, 3, 5, 10.0, 2.0)
        assert_exact({k: v.cpu().numpy() for k, v in o_gpu.items()}, o, f"batched {shp} variant {variant}")


def test_run_rejects_mismatched_outputs(dev):
    """Preallocated outputs are checked before anything is enqueued: shape,
    dtype, device and contiguity must match the problem."""
    bp = bp_mod()
    cost = torch.zeros((8, 5, 6), dtype=torch.float32, device=dev)
    p = bp.BPParams(levels=1, iters=2)
    bad = [
        {"disp": torch.empty((5, 7), dtype=torch.int32, device=dev)},
        {"disp": torch.empty((5, 6), dtype=torch.int64, device=dev)},
        {"soft": torch.empty((6, 5), dtype=torch.float32, device=dev).t()},
        {"msgs": torch.empty((4, 8, 5, 6), dtype=torch.float32)},
    ]
    for o in bad:
        with pytest.raises(ValueError):
            bp.run(cost, p, outputs=[o])
    with pytest.raises(ValueError):
        bp.run([cost, cost], p, outputs=[{"disp": torch.empty((5, 6), dtype=torch.int32, device=dev)}])
    good = {"disp": torch.empty((5, 6), dtype=torch.int32, device=dev), "soft": None, "msgs": None}
    bp.run(cost, p, outputs=[good])
    torch.cuda.synchronize()
    assert int(good["disp"].max()) == 0   # all-zero costs: label 0 everywhere
