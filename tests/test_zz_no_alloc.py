"""bp_run_noalloc (the entry point for callers that cannot allocate device
memory) against bp_run, through the C ABI.

Two calls in a row on the fixed per-GPU scratch array, the second with a
smaller input than the first (the array keeps the first call's contents),
then a batched call: every output equals bp_run's on the same inputs bit for
bit (integer-valued data, every BP quantity an exact integer in FP32), and
the first call's labels also equal the FP64 oracle's.  Problems that need
more than the array are rejected before anything is enqueued, and a call with
preallocated outputs leaves the device's free memory unchanged.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1902_09733_amd as bp
    bp.stereo._abi.lib()
    return torch.device("cuda:0")


def both(bp, problem, params, dev, want_msgs=True):
    """bp_run and bp_run_noalloc on the same problem(s); returns the outputs."""
    ref = bp.run(problem, params, want_msgs=want_msgs)
    torch.cuda.synchronize()
    got = bp.run_noalloc(problem, params, want_msgs=want_msgs)
    torch.cuda.synchronize()
    return ref, got


def assert_same(ref, got):
    ref = ref if isinstance(ref, list) else [ref]
    got = got if isinstance(got, list) else [got]
    assert len(ref) == len(got)
    for r, g in zip(ref, got):
        assert r.keys() == g.keys()
        for k in r:
            assert torch.equal(r[k], g[k]), k


def test_noalloc_matches_bp_run_twice_then_smaller(dev):
    import paper_1902_09733_amd as bp
    # First call: the benchmarked 676x380x64 five-level problem from the pair.
    w = workload("aerial2704x1520_s4_L64")
    print("noalloc call 1: aerial 2704x1520 -> 676x380x64, 5 levels x 10", flush=True)
    left = torch.from_numpy(w["left"]).to(dev)
    right = torch.from_numpy(w["right"]).to(dev)
    pair = bp.Pair(left, right, 64, 20.0, downsample=4)
    p5 = bp.BPParams(levels=5, iters=10, lam=10.0, tau=2.0)
    ref, got = both(bp, pair, p5, dev)
    assert_same(ref, got)
    cost = oracle.cost_volume(oracle.downsample(w["left"], 4), oracle.downsample(w["right"], 4), 64, 20.0)
    o = oracle.run(cost, 5, 10, 10.0, 2.0)
    assert np.array_equal(got["disp"].cpu().numpy(), o["disp"])

    # Second call: a smaller problem (fewer levels, labels and pixels) on the
    # array that still holds the first call's state.
    s = workload("planes160x120_L32")
    print("noalloc call 2: planes 160x120x32, 2 levels x 10", flush=True)
    c = bp.cost_volume(torch.from_numpy(s["left"]).to(dev), torch.from_numpy(s["right"]).to(dev), 32, 20.0)
    p2 = bp.BPParams(levels=2, iters=10, lam=10.0, tau=2.0)
    ref, got = both(bp, c, p2, dev)
    assert_same(ref, got)
    o = oracle.run(oracle.cost_volume(s["left"], s["right"], 32, 20.0), 2, 10, 10.0, 2.0)
    assert np.array_equal(got["disp"].cpu().numpy(), o["disp"])


def test_noalloc_batched_and_soft(dev):
    """The batched form (mixed sizes and label counts, FP16 messages) and the
    soft readout run on the array too."""
    import paper_1902_09733_amd as bp
    rng = np.random.default_rng(7)
    shapes = [(32, 40, 64), (64, 23, 37), (17, 50, 31)]
    vols = [torch.from_numpy(rng.integers(0, 21, size=sh).astype(np.float32)).to(dev) for sh in shapes]
    print("noalloc call 3: batch of 3 mixed problems, FP16 messages", flush=True)
    p = bp.BPParams(levels=3, iters=6, lam=10.0, tau=2.0, msg_dtype="f16")
    ref, got = both(bp, vols, p, dev, want_msgs=False)
    assert_same(ref, got)
    print("noalloc call 4: soft readout", flush=True)
    ref = bp.run(vols[1], bp.BPParams(levels=2, iters=5), want_soft=True)
    got = bp.run_noalloc(vols[1], bp.BPParams(levels=2, iters=5), want_soft=True)
    torch.cuda.synchronize()
    assert_same(ref, got)


def test_noalloc_rejects_oversized_and_allocates_nothing(dev):
    import paper_1902_09733_amd as bp
    from paper_1902_09733_amd import _abi
    # 1352x760x128 at six levels needs about 3.3 GB of workspace.
    big = bp.Pair(torch.zeros((760, 1352, 3), dtype=torch.uint8, device=dev),
                  torch.zeros((760, 1352, 3), dtype=torch.uint8, device=dev), 128, 20.0)
    p6 = bp.BPParams(levels=6, iters=12)
    assert bp.workspace_bytes([big], p6) > _abi.BP_NOALLOC_SCRATCH_BYTES
    with pytest.raises(_abi.BPError) as e:
        bp.run_noalloc(big, p6)
    assert e.value.status == _abi.BP_ERR_WORKSPACE_TOO_SMALL
    # With outputs passed in, a call leaves torch's allocator and the
    # device's free memory where they were.
    vol = torch.full((32, 30, 41), 4.0, dtype=torch.float32, device=dev)
    vol[:, ::2, ::3] = 0.0
    outs = [{"disp": torch.empty((30, 41), dtype=torch.int32, device=dev)}]
    p = bp.BPParams(levels=3, iters=4)
    bp.run_noalloc([vol], p, outputs=outs)
    torch.cuda.synchronize()
    a0, f0 = torch.cuda.memory_allocated(), torch.cuda.mem_get_info()[0]
    bp.run_noalloc([vol], p, outputs=outs)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == a0
    assert torch.cuda.mem_get_info()[0] == f0
    ref = bp.run(vol, p)
    assert torch.equal(ref["disp"], outs[0]["disp"])
