"""GPU parity of the differentiation form (hand-written adjoint) against the
FP64 oracle adjoint (element-wise, small grids) and against FP64 central
finite differences of the oracle's forward pass (the 8 x 320x240 x 64-label
batch, K = 8, checkpoints every 2 half-sweeps).

FP32 forward values can pick a different winner than FP64 at near-ties of
the piecewise-linear transform, which moves single gradient entries; the
element-wise bar is therefore on the fraction of entries within tolerance,
and directional derivatives must agree within 1e-3 relative."""
import numpy as np
import pytest
import torch

import oracle
from synth import workload

pytestmark = pytest.mark.gpu

DIR_TOL = 1e-3


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch.device("cuda:0")


def jittered(shape, seed):
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 20, size=shape) + rng.uniform(0.0, 0.5, size=shape)).astype(np.float32).astype(np.float64)


def gpu_grad(costs, g, K, lam, tau, T, every, dev):
    import paper_1902_09733_amd as bp
    p = bp.BPParams(levels=1, iters=K, lam=lam, tau=tau, temperature=T, checkpoint_every=every)
    vols = [torch.from_numpy(c.astype(np.float32)).to(dev) for c in costs]
    ck = torch.empty(bp.checkpoint_bytes(vols, p), dtype=torch.uint8, device=dev)
    outs = bp.run(vols, p, want_disp=False, want_soft=True, checkpoints=ck)
    gs = [torch.from_numpy(x.astype(np.float32)).to(dev) for x in g]
    gc, gl, gt = bp.backward(vols, p, ck, gs)
    torch.cuda.synchronize()
    return ([o["soft"].cpu().numpy() for o in outs], [x.cpu().numpy().astype(np.float64) for x in gc],
            float(gl.item()), float(gt.item()))


@pytest.mark.parametrize("shape,K,every", [((16, 12, 20), 1, 1), ((32, 12, 20), 5, 2), ((64, 9, 14), 8, 2),
                                           ((32, 7, 11), 6, 3), ((20, 10, 13), 4, 4), ((64, 1, 33), 7, 2)])
def test_adjoint_matches_oracle_adjoint(dev, shape, K, every):
    L, H, W = shape
    rng = np.random.default_rng(L + H + K)
    costs = [jittered(shape, 11 + i) for i in range(2)]
    g = [rng.normal(size=(H, W)) for _ in costs]
    lam, tau, T = 3.0, 2.5, 0.5
    soft, gc, gl, gt = gpu_grad(costs, g, K, lam, tau, T, every, dev)
    ol = ot = 0.0
    for i, c in enumerate(costs):
        s_o, gc_o, gl_o, gt_o = oracle.backward(c, K, lam, tau, T, g[i])
        ol += gl_o
        ot += gt_o
        assert np.abs(soft[i] - s_o).max() <= 1e-3
        scale = np.abs(gc_o).max()
        close = np.abs(gc[i] - gc_o) <= 1e-3 * scale + 1e-5
        assert close.mean() >= 0.999, close.mean()
        V = np.random.default_rng(i).normal(size=shape)
        a, b = (gc[i] * V).sum(), (gc_o * V).sum()
        assert abs(a - b) <= DIR_TOL * max(abs(b), np.abs(gc_o).sum() * 1e-3), (a, b)
    assert abs(gl - ol) <= DIR_TOL * max(1.0, abs(ol)), (gl, ol)
    assert abs(gt - ot) <= DIR_TOL * max(1.0, abs(ot)), (gt, ot)


def test_autograd_batch_matches_finite_differences(dev):
    """The 8 x 320x240 x 64 batch: directional derivatives of a random
    projection of the loss against FP64 central differences (eps = 1e-4)."""
    from paper_1902_09733_amd import soft_argmin_bp
    w = workload("planes320x240_L64_x8")
    K, lam, tau, T = w["iters"], 10.0, w["tau"], w["temperature"]
    costs = []
    for pr in w["pairs"]:
        c = oracle.cost_volume(pr["left"], pr["right"], 64, 20.0) + pr["jitter"]
        costs.append(c.astype(np.float32).astype(np.float64))
    C = np.stack(costs)
    rng = np.random.default_rng(5)
    G = rng.normal(size=(8, 240, 320))
    ct = torch.from_numpy(C.astype(np.float32)).to(dev).requires_grad_(True)
    lt = torch.tensor(lam, device=dev, requires_grad=True)
    tt = torch.tensor(tau, device=dev, requires_grad=True)
    soft = soft_argmin_bp(ct, lt, tt, iters=K, temperature=T, checkpoint_every=w["checkpoint_every"])
    loss = (soft * torch.from_numpy(G.astype(np.float32)).to(dev)).sum()
    loss.backward()
    gC = ct.grad.double().cpu().numpy()

    def ell(Cx, l=lam, t=tau):
        return sum(float((G[i] * oracle.run(Cx[i], 1, K, l, t, want_soft=True, temperature=T)["soft"]).sum())
                   for i in range(8))
    eps = 1e-4
    for d in range(3):
        V = np.random.default_rng(100 + d).normal(size=C.shape)
        fd = (ell(C + eps * V) - ell(C - eps * V)) / (2 * eps)
        an = float((gC * V).sum())
        print(f"direction {d}: fd {fd:.6f} adjoint {an:.6f}", flush=True)
        assert abs(fd - an) <= DIR_TOL * abs(fd), (fd, an)
    fdl = (ell(C, lam + eps) - ell(C, lam - eps)) / (2 * eps)
    fdt = (ell(C, lam, tau + eps) - ell(C, lam, tau - eps)) / (2 * eps)
    print(f"lambda: fd {fdl:.6f} adjoint {lt.grad.item():.6f}; tau: fd {fdt:.6f} adjoint {tt.grad.item():.6f}")
    assert abs(fdl - lt.grad.item()) <= DIR_TOL * abs(fdl)
    assert abs(fdt - tt.grad.item()) <= DIR_TOL * abs(fdt)
