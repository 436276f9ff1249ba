"""Pins of the oracle's reverse-mode derivative (differentiation form) by
central finite differences of its own forward pass, in FP64.

Costs carry a U(0, 0.5) jitter so that ties in the piecewise-linear transform
have measure zero; tau is non-integer (the tau-derivative is one-sided at
integer tau)."""
import numpy as np
import pytest


def loss(orc, cost, g, K, lam, tau, T):
    return float((g * orc.run(cost, 1, K, lam, tau, want_soft=True, temperature=T)["soft"]).sum())


@pytest.mark.parametrize("shape,K", [((8, 5, 6), 6), ((12, 7, 9), 8), ((5, 1, 11), 7), ((6, 9, 1), 5)])
def test_adjoint_matches_finite_differences(orc, shape, K):
    rng = np.random.default_rng(sum(shape) + K)
    L, H, W = shape
    cost = rng.integers(0, 20, size=shape) + rng.uniform(0.0, 0.5, size=shape)
    g = rng.normal(size=(H, W))
    lam, tau, T = 3.0, 2.5, 0.5
    soft, gc, gl, gt = orc.backward(cost, K, lam, tau, T, g)
    ref = orc.run(cost, 1, K, lam, tau, want_soft=True, temperature=T)["soft"]
    np.testing.assert_array_equal(soft, ref)
    eps = 1e-6
    for _ in range(3):
        V = rng.normal(size=shape)
        fd = (loss(orc, cost + eps * V, g, K, lam, tau, T) - loss(orc, cost - eps * V, g, K, lam, tau, T)) / (2 * eps)
        an = float((gc * V).sum())
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
    fdl = (loss(orc, cost, g, K, lam + eps, tau, T) - loss(orc, cost, g, K, lam - eps, tau, T)) / (2 * eps)
    fdt = (loss(orc, cost, g, K, lam, tau + eps, T) - loss(orc, cost, g, K, lam, tau - eps, T)) / (2 * eps)
    assert abs(fdl - gl) <= 1e-6 * max(1.0, abs(gl)), (fdl, gl)
    assert abs(fdt - gt) <= 1e-6 * max(1.0, abs(gt)), (fdt, gt)


def test_adjoint_elementwise_finite_differences(orc):
    """Every element of grad_cost on a tiny grid against its own central difference."""
    rng = np.random.default_rng(3)
    L, H, W, K = 5, 3, 4, 5
    cost = rng.integers(0, 15, size=(L, H, W)) + rng.uniform(0.0, 0.5, size=(L, H, W))
    g = rng.normal(size=(H, W))
    lam, tau, T = 2.0, 1.5, 0.7
    _, gc, _, _ = orc.backward(cost, K, lam, tau, T, g)
    eps = 1e-6
    for idx in np.ndindex(cost.shape):
        e = np.zeros_like(cost)
        e[idx] = eps
        fd = (loss(orc, cost + e, g, K, lam, tau, T) - loss(orc, cost - e, g, K, lam, tau, T)) / (2 * eps)
        assert abs(fd - gc[idx]) <= 1e-6 * max(1.0, abs(gc[idx])), (idx, fd, gc[idx])


def test_adjoint_zero_iterations_is_softmax_derivative(orc):
    """K = 0: d = sum f softmax(-C/T); dd/dC_f = -(1/T) p_f (f - d) (closed form)."""
    rng = np.random.default_rng(4)
    L, H, W = 7, 2, 3
    cost = rng.uniform(0, 5, size=(L, H, W))
    g = rng.normal(size=(H, W))
    T = 0.8
    soft, gc, gl, gt = orc.backward(cost, 0, 3.0, 2.5, T, g)
    p = np.exp(-(cost - cost.min(axis=0)) / T)
    p /= p.sum(axis=0)
    d = (np.arange(L)[:, None, None] * p).sum(axis=0)
    np.testing.assert_allclose(soft, d, rtol=1e-14)
    ref = -g[None] / T * p * (np.arange(L)[:, None, None] - d[None])
    np.testing.assert_allclose(gc, ref, rtol=1e-12, atol=1e-15)
    assert gl == 0.0 and gt == 0.0


@pytest.mark.parametrize("shape,K,lam,tau", [((6, 4, 5), 5, 3.0, 2.5), ((8, 5, 6), 6, 2.0, 2.0),
                                             ((5, 1, 9), 4, 4.0, 1.5)])
def test_adjoint_elementwise_autograd_with_ties(orc, shape, K, lam, tau):
    """Integer costs make ties in the transform's comparisons common.  The
    oracle's adjoint must equal, entry by entry, torch autograd through an
    FP64 re-implementation of the forward pass that takes the same branch on
    every tie (tests/_pins.py), for grad_cost, grad_lambda and grad_tau."""
    torch = pytest.importorskip("torch")
    import _pins
    rng = np.random.default_rng(sum(shape) * 7 + K)
    L, H, W = shape
    cost = rng.integers(0, 12, size=shape).astype(float)
    g = rng.normal(size=(H, W))
    T = 0.5
    soft, gc, gl, gt = orc.backward(cost, K, lam, tau, T, g)
    c = torch.tensor(cost, dtype=torch.float64, requires_grad=True)
    lt = torch.tensor(lam, dtype=torch.float64, requires_grad=True)
    tt = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    d = _pins.autograd_soft_bp(c, lt, tt, K, T)
    np.testing.assert_allclose(d.detach().numpy(), soft, rtol=0, atol=1e-12)
    (d * torch.tensor(g)).sum().backward()
    np.testing.assert_allclose(gc, c.grad.numpy(), rtol=1e-10, atol=1e-12)
    assert abs(gl - lt.grad.item()) <= 1e-10 * max(1.0, abs(gl))
    assert abs(gt - tt.grad.item()) <= 1e-10 * max(1.0, abs(gt))
    # The case exercises ties: pixels with two labels of equal cost.
    assert (np.diff(np.sort(cost, axis=0), axis=0) == 0).any(axis=0).sum() > 0
