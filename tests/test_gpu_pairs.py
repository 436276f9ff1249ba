"""The fused pair of half-sweeps (two checkerboard half-sweeps per launch,
colour-1 messages kept on chip between them) against one launch per
half-sweep.

The library runs pixel-major levels as fused pairs when the kernel choice is
left to it (variant 0); variant 1 is the one-half-sweep kernel with the same
per-message arithmetic (h summed in slot order).  On real-valued costs --
where any change of operation order would show -- both must give the same
labels, soft-argmin disparities and final finest-level messages bit for
bit, over tile edges and ragged grids (1x1 up to several tiles), every lane
split (2 to 256 labels), odd and even K (single half-sweeps before or after
the pairs), one to five levels, and the three storage formats (16-bit levels
under an FP32 coarsest level take the materialised parent copy).  On integer data the fused path
also equals the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1902_09733_amd as bp
    bp.stereo._abi.lib()
    return torch.device("cuda:0")


def both(bp, cost, levels, K, fmt, lam=7.3, tau=2.6):
    outs = []
    for variant in (0, 1):
        p = bp.BPParams(levels=levels, iters=K, lam=lam, tau=tau, msg_dtype=fmt, variant=variant, temperature=0.7)
        o = bp.run(cost, p, want_soft=True, want_msgs=True)
        torch.cuda.synchronize()
        outs.append(o)
    return outs


CASES = [
    # (L, H, W, levels, K, fmt)
    (64, 380 // 4, 676 // 4, 3, 10, "f32"),
    (64, 37, 53, 2, 7, "f32"),
    (64, 1, 1, 1, 4, "f32"),
    (64, 1, 2, 1, 3, "f32"),
    (64, 2, 1, 2, 2, "f32"),
    (64, 9, 17, 1, 5, "f32"),
    (64, 8, 16, 1, 6, "f32"),
    (2, 21, 34, 3, 8, "f32"),
    (5, 13, 40, 2, 9, "f32"),
    (16, 40, 33, 4, 6, "f32"),
    (17, 24, 19, 3, 4, "f32"),
    (32, 50, 70, 5, 10, "f32"),
    (33, 25, 31, 2, 5, "f32"),
    (65, 19, 23, 2, 4, "f32"),
    (96, 17, 40, 3, 6, "f32"),
    (128, 22, 35, 2, 8, "f32"),
    (200, 9, 20, 2, 3, "f32"),
    (256, 12, 17, 1, 2, "f32"),
    (64, 33, 47, 3, 10, "f16"),
    (64, 33, 47, 3, 9, "bf16"),
    (64, 30, 40, 2, 6, "f16"),
    (128, 20, 25, 4, 8, "f16"),
    (32, 31, 29, 3, 7, "bf16"),
]


@pytest.mark.parametrize("L,H,W,levels,K,fmt", CASES)
def test_pairs_equal_single_half_sweeps(dev, L, H, W, levels, K, fmt):
    import paper_1902_09733_amd as bp
    print(f"pairs vs single: L={L} {W}x{H} levels={levels} K={K} {fmt}", flush=True)
    rng = np.random.default_rng(L * 1000 + H * 10 + W + K)
    cost = torch.from_numpy(rng.uniform(0.0, 20.0, size=(L, H, W)).astype(np.float32)).to(dev)
    a, b = both(bp, cost, levels, K, fmt)
    assert torch.equal(a["disp"], b["disp"])
    assert torch.equal(a["msgs"], b["msgs"])
    # Soft-argmin: read out by the last fused pair (even K) or by the readout
    # pass, with the same arithmetic.
    assert torch.equal(a["soft"], b["soft"])


@pytest.mark.parametrize("L,H,W,levels,K", [(64, 47, 61, 3, 10), (32, 20, 29, 2, 7), (96, 13, 22, 2, 6)])
def test_pairs_equal_oracle_integer(dev, L, H, W, levels, K):
    import paper_1902_09733_amd as bp
    print(f"pairs vs oracle: L={L} {W}x{H} levels={levels} K={K}", flush=True)
    rng = np.random.default_rng(L + H + W)
    c = rng.integers(0, 21, size=(L, H, W)).astype(np.float64)
    o = oracle.run(c, levels, K, 10.0, 2.0, want_msgs=True)
    g = bp.run(torch.from_numpy(c.astype(np.float32)).to(dev), bp.BPParams(levels=levels, iters=K), want_msgs=True)
    torch.cuda.synchronize()
    assert np.array_equal(g["disp"].cpu().numpy(), o["disp"])
    assert np.array_equal(g["msgs"].cpu().numpy().astype(np.float64), o["msgs"])


@pytest.mark.parametrize("fmt,K,levels", [("f32", 6, 3), ("f32", 2, 2), ("f16", 8, 4), ("bf16", 4, 3),
                                          ("f32", 10, 5)])
def test_batched_pairs_equal_single_problems(dev, fmt, K, levels):
    """Batched fused pairs (one launch per level, pair and lane split over
    every problem) against each problem run alone with one launch per
    half-sweep: same labels and messages on real-valued costs, mixed sizes
    and label counts (several lane splits, tiles shrunk on small levels)."""
    import paper_1902_09733_amd as bp
    shapes = [(64, 37, 53), (32, 20, 29), (96, 17, 40), (17, 11, 60), (128, 12, 21), (64, 9, 9)]
    print(f"batched pairs: {fmt} K={K} levels={levels}", flush=True)
    rng = np.random.default_rng(K * 10 + levels)
    vols = [torch.from_numpy(rng.uniform(0.0, 20.0, size=sh).astype(np.float32)).to(dev) for sh in shapes]
    p0 = bp.BPParams(levels=levels, iters=K, lam=7.3, tau=2.6, msg_dtype=fmt)
    got = bp.run(vols, p0, want_msgs=True)
    torch.cuda.synchronize()
    p1 = bp.BPParams(levels=levels, iters=K, lam=7.3, tau=2.6, msg_dtype=fmt, variant=1)
    for v, g in zip(vols, got):
        ref = bp.run(v, p1, want_msgs=True)
        torch.cuda.synchronize()
        assert torch.equal(ref["disp"], g["disp"])
        assert torch.equal(ref["msgs"], g["msgs"])


@pytest.mark.parametrize("K,every", [(8, 2), (6, 2), (8, 4), (4, 4), (2, 2)])
def test_batched_pairs_checkpoints_equal_single_problems(dev, K, every):
    """Forward calls that save states for the adjoint run batched fused pairs
    over several problems.  The saved states (buffers zeroed beforehand, so
    every byte compares), the soft-argmin disparity and the adjoint's
    gradients equal those of each problem run on its own, bit for bit, on
    real-valued costs of mixed sizes and label counts."""
    import paper_1902_09733_amd as bp
    shapes = [(64, 37, 53), (32, 20, 29), (96, 17, 40), (64, 9, 9), (17, 11, 60)]
    print(f"batched pairs with checkpoints: K={K} every={every}", flush=True)
    rng = np.random.default_rng(K * 100 + every)
    vols = [torch.from_numpy(rng.uniform(0.0, 20.0, size=sh).astype(np.float32)).to(dev) for sh in shapes]
    gs = [torch.from_numpy(rng.standard_normal(size=sh[1:]).astype(np.float32)).to(dev) for sh in shapes]
    p = bp.BPParams(levels=1, iters=K, lam=7.3, tau=2.6, temperature=0.5, checkpoint_every=every)
    ck = torch.zeros(bp.checkpoint_bytes(vols, p), dtype=torch.uint8, device=dev)
    got = bp.run(vols, p, want_disp=False, want_soft=True, checkpoints=ck)
    gc, gl, gt = bp.backward(vols, p, ck, gs)
    torch.cuda.synchronize()
    off = 0
    gl_ref = gt_ref = 0.0
    for i, (v, g) in enumerate(zip(vols, gs)):
        n = bp.checkpoint_bytes(v, p)
        ck1 = torch.zeros(n, dtype=torch.uint8, device=dev)
        ref = bp.run(v, p, want_disp=False, want_soft=True, checkpoints=ck1)
        gc1, gl1, gt1 = bp.backward(v, p, ck1, g)
        torch.cuda.synchronize()
        assert torch.equal(ck[off:off + n], ck1), f"problem {i}: saved states differ"
        assert torch.equal(got[i]["soft"], ref["soft"]), f"problem {i}: soft disparity differs"
        assert torch.equal(gc[i], gc1), f"problem {i}: cost gradient differs"
        off += n
        gl_ref += float(gl1.item())
        gt_ref += float(gt1.item())
    assert off == ck.numel()
    # lambda and tau gradients sum over the batch (in another order here).
    assert abs(float(gl.item()) - gl_ref) <= 1e-5 * max(1.0, abs(gl_ref))
    assert abs(float(gt.item()) - gt_ref) <= 1e-5 * max(1.0, abs(gt_ref))


def test_batched_pairs_streaming_and_cache_groups(dev):
    """Problems whose finest level does not fit the batched form's cache
    budget run as groups of their own there and share launches at coarser
    levels, small ones share cache groups: labels and messages equal each
    problem run alone with one launch per half-sweep, on real-valued
    costs."""
    import paper_1902_09733_amd as bp
    shapes = [(64, 500, 900), (64, 37, 53), (96, 400, 640), (64, 300, 1000), (17, 11, 60)]
    rng = np.random.default_rng(7)
    vols = [torch.from_numpy(rng.uniform(0.0, 20.0, size=sh).astype(np.float32)).to(dev) for sh in shapes]
    p0 = bp.BPParams(levels=3, iters=4, lam=7.3, tau=2.6)
    got = bp.run(vols, p0, want_msgs=True)
    torch.cuda.synchronize()
    p1 = bp.BPParams(levels=3, iters=4, lam=7.3, tau=2.6, variant=1)
    for i, (v, g) in enumerate(zip(vols, got)):
        ref = bp.run(v, p1, want_msgs=True)
        torch.cuda.synchronize()
        assert torch.equal(ref["disp"], g["disp"]), f"problem {i}: labels differ"
        assert torch.equal(ref["msgs"], g["msgs"]), f"problem {i}: messages differ"
