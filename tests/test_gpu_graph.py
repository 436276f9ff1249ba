"""Parity of the launch sequences the benchmark times, as replayed HIP graphs.

bench.py times graph replays: the single-pair step (pair -> data term,
pyramid, BP, readout -> joint bilateral upsampling) and the 48-pair batched
form.  These tests capture the same sequences with the same workspaces,
replay each graph several times with eager work and synchronisations in
between (outputs overwritten, another problem run eagerly on the same
stream), and check every replay against the FP64 oracle: labels of Eq. 1's
readout bit for bit (integer-valued data, every BP quantity an exact integer
in FP32), and the Eq. 2 upsampling within 2e-3 labels on every row of the
2704x1520 frame.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import workload

pytestmark = pytest.mark.gpu

JBU_TOL = 2e-3


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1902_09733_amd as bp
    bp.stereo._abi.lib()
    return torch.device("cuda:0")


def capture(fn):
    """fn once eagerly on a side stream, then captured in a graph (as bench.py does)."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


def perturb(bp, dev, outs):
    """Eager work between replays: overwrite the graph's outputs and run an
    unrelated problem through the library on the current stream."""
    for t in outs:
        if t.dtype == torch.int32:
            t.fill_(-7)
        else:
            t.fill_(float("nan"))
    other = torch.full((16, 24, 40), 3.0, dtype=torch.float32, device=dev)
    other[:, :, ::3] = 0.0
    bp.run(other, bp.BPParams(levels=2, iters=3))
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def aerial_ref():
    w = workload("aerial2704x1520_s4_L64")
    cost = oracle.cost_volume(oracle.downsample(w["left"], 4), oracle.downsample(w["right"], 4), 64, 20.0)
    o = oracle.run(cost, 5, 10, 10.0, 2.0, want_msgs=True)
    up = oracle.upsample(o["disp"], w["left"], 8.0, 12.0)
    return w, o, up


def test_bench_step_graph_replays_exact(dev, aerial_ref):
    """The benchmarked step exactly as bench.py captures it."""
    import paper_1902_09733_amd as bp
    w, o, up_ref = aerial_ref
    left = torch.from_numpy(w["left"]).to(dev)
    right = torch.from_numpy(w["right"]).to(dev)
    disp = torch.empty((380, 676), dtype=torch.int32, device=dev)
    up = torch.empty((1520, 2704), dtype=torch.float32, device=dev)
    params = bp.BPParams(levels=5, iters=10, lam=10.0, tau=2.0)
    ws = bp.Workspace()
    outs = [{"disp": disp, "soft": None, "msgs": None}]
    pair = bp.Pair(left, right, 64, 20.0, downsample=4)

    def step():
        bp.run(pair, params, workspace=ws, outputs=outs)
        bp.upsample(disp, left, 8.0, 12.0, -1, out=up)

    g = capture(step)
    for rep in range(3):
        perturb(bp, dev, [disp, up])
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(disp.cpu().numpy(), o["disp"], err_msg=f"labels, replay {rep}")
        err = np.abs(up.cpu().numpy().astype(np.float64) - up_ref).max()
        assert err <= JBU_TOL, f"replay {rep}: upsampling error {err}"


def test_bench_step_graph_messages_exact(dev, aerial_ref):
    """The same captured sequence with the final level-0 messages exported:
    every message of every replay equals the oracle's."""
    import paper_1902_09733_amd as bp
    w, o, _ = aerial_ref
    left = torch.from_numpy(w["left"]).to(dev)
    right = torch.from_numpy(w["right"]).to(dev)
    disp = torch.empty((380, 676), dtype=torch.int32, device=dev)
    msgs = torch.empty((4, 64, 380, 676), dtype=torch.float32, device=dev)
    params = bp.BPParams(levels=5, iters=10, lam=10.0, tau=2.0)
    ws = bp.Workspace()
    outs = [{"disp": disp, "soft": None, "msgs": msgs}]
    pair = bp.Pair(left, right, 64, 20.0, downsample=4)
    g = capture(lambda: bp.run(pair, params, workspace=ws, outputs=outs))
    for rep in range(2):
        perturb(bp, dev, [disp, msgs])
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(disp.cpu().numpy(), o["disp"], err_msg=f"labels, replay {rep}")
        np.testing.assert_array_equal(msgs.cpu().numpy().astype(np.float64), o["msgs"],
                                      err_msg=f"messages, replay {rep}")


@pytest.fixture(scope="module")
def batch48():
    return workload("batch48_mixed")


def smallest_per_label_count(pairs):
    best = {}
    for i, p in enumerate(pairs):
        L = p["num_labels"]
        if L not in best or p["width"] * p["height"] < pairs[best[L]]["width"] * pairs[best[L]]["height"]:
            best[L] = i
    return [best[L] for L in sorted(best)]


@pytest.mark.parametrize("fmt,mode", [("f32", oracle.STORE_F64), ("f16", oracle.STORE_F16)])
def test_batched_graph_replays_exact(dev, batch48, fmt, mode):
    """The 48-pair batched form as bench.py captures it (all pairs from their
    images, 5 levels x 8 half-sweeps, FP32 and FP16 messages): the smallest
    pair of each label count (32, 64, 96, 128) against the oracle on every
    replay, and every pair's labels identical across replays."""
    import paper_1902_09733_amd as bp
    wl = batch48
    pairs = wl["pairs"]
    lefts = [torch.from_numpy(p["left"]).to(dev) for p in pairs]
    rights = [torch.from_numpy(p["right"]).to(dev) for p in pairs]
    srcs = [bp.Pair(l, r, p["num_labels"], wl["data_trunc"]) for l, r, p in zip(lefts, rights, pairs)]
    outs = [{"disp": torch.empty((p["height"], p["width"]), dtype=torch.int32, device=dev), "soft": None,
             "msgs": None} for p in pairs]
    pp = bp.BPParams(levels=wl["levels"], iters=wl["iters"], lam=wl["lam"], tau=wl["tau"], msg_dtype=fmt)
    ws = bp.Workspace()
    g = capture(lambda: bp.run(srcs, pp, workspace=ws, outputs=outs))
    check = smallest_per_label_count(pairs)
    refs = {}
    for i in check:
        p = pairs[i]
        cost = oracle.cost_volume(p["left"], p["right"], p["num_labels"], wl["data_trunc"])
        refs[i] = oracle.run(cost, wl["levels"], wl["iters"], wl["lam"], wl["tau"], store_mode=mode)["disp"]
    first = None
    for rep in range(2):
        perturb(bp, dev, [o["disp"] for o in outs])
        g.replay()
        torch.cuda.synchronize()
        got = [o["disp"].cpu().numpy() for o in outs]
        for i in check:
            np.testing.assert_array_equal(got[i], refs[i], err_msg=f"pair {i} {fmt}, replay {rep}")
        if first is None:
            first = got
        else:
            for i, (a, b) in enumerate(zip(first, got)):
                np.testing.assert_array_equal(a, b, err_msg=f"pair {i} {fmt} differs between replays")
