"""Pins of the oracle's hierarchical checkerboard BP (Eq. 1 energy and argmin).

Loopy BP has no closed form, so the pins are: exactness on chains and trees
(textbook dynamic programming and enumeration), equality with an independent
synchronous-schedule implementation (the bipartite argument), symmetries,
invariants, pyramid plumbing against single-level runs, and recovery of known
disparities on a synthetic scene.
"""
import numpy as np
import pytest

import _pins


def beliefs(cost, msgs):
    return cost + msgs.sum(axis=0)


def norm(a):
    return a - a.min(axis=0, keepdims=True)


@pytest.mark.parametrize("orient", ["row", "col"])
@pytest.mark.parametrize("N,L,lam,tau", [(9, 5, 3.0, 2.0), (16, 8, 2.0, 3.0), (7, 4, 5.0, 0.5)])
def test_chain_exact_min_marginals(orc, orient, N, L, lam, tau):
    rng = np.random.default_rng(N * 31 + L)
    unary = rng.integers(0, 20, size=(N, L)).astype(float)
    cost = unary.T[:, None, :] if orient == "row" else unary.T[:, :, None]
    cost = np.ascontiguousarray(cost)
    res = orc.run(cost, 1, 2 * N + 2, lam, tau, want_msgs=True)
    b = beliefs(cost, res["msgs"]).reshape(L, N)
    mm = _pins.chain_min_marginals(unary, _pins.vpair(lam, tau, L)).T
    np.testing.assert_array_equal(norm(b), norm(mm))
    # Argmin: lowest label attaining the min-marginal minimum.
    np.testing.assert_array_equal(res["disp"].reshape(N), np.argmin(mm, axis=0))


def test_chain_enumeration(orc):
    rng = np.random.default_rng(5)
    for N, L in ((5, 3), (6, 2), (4, 4)):
        unary = rng.integers(0, 12, size=(N, L)).astype(float)
        cost = np.ascontiguousarray(unary.T[:, None, :])
        V = _pins.vpair(4.0, 2.0, L)
        mm, _, _ = _pins.enumerate_min_marginals(cost, _pins.edges_of(N, 1), V)
        res = orc.run(cost, 1, 2 * N + 2, 4.0, 2.0, want_msgs=True)
        np.testing.assert_array_equal(norm(beliefs(cost, res["msgs"])), norm(mm))


def comb_mask(W, H):
    """Spanning comb tree: the whole top row plus every column."""
    m = np.zeros((H, W), np.uint8)
    m[0, :-1] |= 1
    m[:-1, :] |= 2
    return m


def test_tree_enumeration_3x3(orc):
    rng = np.random.default_rng(11)
    W = H = 3
    L = 3
    cost = rng.integers(0, 10, size=(L, H, W)).astype(float)
    mask = comb_mask(W, H)
    V = _pins.vpair(3.0, 2.0, L)
    mm, best_e, best_lab = _pins.enumerate_min_marginals(cost, _pins.edges_of(W, H, mask), V)
    res = orc.run(cost, 1, 20, 3.0, 2.0, edges=mask, want_msgs=True)
    np.testing.assert_array_equal(norm(beliefs(cost, res["msgs"])), norm(mm))


@pytest.mark.parametrize("shape", [(5, 4), (6, 7)])
def test_tree_dp(orc, shape):
    W, H = shape
    L = 6
    rng = np.random.default_rng(W * H)
    cost = rng.integers(0, 30, size=(L, H, W)).astype(float)
    mask = comb_mask(W, H)
    V = _pins.vpair(7.0, 2.5, L)
    mm = _pins.tree_min_marginals(cost, _pins.edges_of(W, H, mask), V)
    res = orc.run(cost, 1, 2 * (W + H) + 4, 7.0, 2.5, edges=mask, want_msgs=True)
    np.testing.assert_array_equal(norm(beliefs(cost, res["msgs"])), norm(mm))


def row_comb_mask(W, H):
    """Spanning comb tree: the whole left column plus every row."""
    m = np.zeros((H, W), np.uint8)
    m[:, :-1] |= 1
    m[:-1, 0] |= 2
    return m


def test_tree_dp_row_comb(orc):
    W, H, L = 6, 5, 5
    rng = np.random.default_rng(2)
    cost = rng.integers(0, 30, size=(L, H, W)).astype(float)
    mask = row_comb_mask(W, H)
    V = _pins.vpair(6.0, 2.0, L)
    mm = _pins.tree_min_marginals(cost, _pins.edges_of(W, H, mask), V)
    res = orc.run(cost, 1, 2 * (W + H) + 4, 6.0, 2.0, edges=mask, want_msgs=True)
    np.testing.assert_array_equal(norm(beliefs(cost, res["msgs"])), norm(mm))


@pytest.mark.parametrize("W,H,T", [(7, 5, 1), (7, 5, 2), (6, 5, 5), (9, 8, 8)])
def test_checkerboard_equals_synchronous(orc, W, H, T):
    """After T half-sweeps, the slots of colour T%2 hold synchronous messages
    of iteration T and the slots of the other colour those of iteration T-1."""
    rng = np.random.default_rng(W * 100 + H * 10 + T)
    L = 6
    lam, tau = 4.0, 2.0
    cost = rng.integers(0, 25, size=(L, H, W)).astype(float)
    res = orc.run(cost, 1, T, lam, tau, want_msgs=True)
    M = _pins.synchronous_bp(cost, lam, tau, T)
    yy, xx = np.mgrid[0:H, 0:W]
    colour = (xx + yy) % 2
    got = res["msgs"]
    for c, s in ((T % 2, T), ((T - 1) % 2, T - 1)):
        sel = colour == c
        np.testing.assert_array_equal(got[:, :, sel], M[s][:, :, sel])


def test_message_invariants_on_scene(orc):
    from synth import workload
    w = workload("planes160x120_L32")
    cost = orc.cost_volume(w["left"], w["right"], 32, 20.0)
    lam, tau = 10.0, 2.0
    res = orc.run(cost, 1, 7, lam, tau, want_msgs=True)
    m = res["msgs"]
    assert m.min() == 0.0 and m.max() <= lam * tau
    # Every in-grid slot is normalised to minimum zero.
    mins = m.min(axis=1)
    assert (mins == 0).all()
    # Integer inputs keep every message an integer.
    assert np.array_equal(m, np.rint(m))


def test_lambda_zero_is_winner_take_all(orc):
    rng = np.random.default_rng(9)
    cost = rng.uniform(0, 20, size=(12, 9, 11))
    res = orc.run(cost, 3, 6, 0.0, 2.0)
    np.testing.assert_array_equal(res["disp"], np.argmin(cost, axis=0))


def test_per_pixel_shift_invariance(orc):
    rng = np.random.default_rng(4)
    cost = rng.integers(0, 20, size=(8, 10, 13)).astype(float)
    shift = rng.integers(0, 50, size=(1, 10, 13)).astype(float)
    a = orc.run(cost, 2, 6, 5.0, 2.0, want_msgs=True)
    b = orc.run(cost + shift, 2, 6, 5.0, 2.0, want_msgs=True)
    np.testing.assert_array_equal(a["disp"], b["disp"])
    np.testing.assert_array_equal(a["msgs"], b["msgs"])


def test_mirror_and_transpose_symmetry(orc):
    """Mirroring the grid (odd sizes keep the checkerboard phase) swaps the
    left/right (or up/down) slots; transposing swaps left<->up, right<->down."""
    rng = np.random.default_rng(8)
    L, H, W = 7, 9, 11
    cost = rng.integers(0, 25, size=(L, H, W)).astype(float)
    base = orc.run(cost, 1, 9, 5.0, 2.0, want_msgs=True)
    mx = orc.run(np.ascontiguousarray(cost[:, :, ::-1]), 1, 9, 5.0, 2.0, want_msgs=True)
    np.testing.assert_array_equal(mx["disp"], base["disp"][:, ::-1])
    np.testing.assert_array_equal(mx["msgs"][[1, 0, 2, 3]][..., ::-1], base["msgs"])
    my = orc.run(np.ascontiguousarray(cost[:, ::-1, :]), 1, 9, 5.0, 2.0, want_msgs=True)
    np.testing.assert_array_equal(my["msgs"][[0, 1, 3, 2]][:, :, ::-1, :], base["msgs"])
    tr = orc.run(np.ascontiguousarray(cost.transpose(0, 2, 1)), 1, 9, 5.0, 2.0, want_msgs=True)
    np.testing.assert_array_equal(tr["disp"].T, base["disp"])
    np.testing.assert_array_equal(tr["msgs"][[2, 3, 0, 1]].transpose(0, 1, 3, 2), base["msgs"])


def test_brute_mode_matches_dt_mode(orc):
    rng = np.random.default_rng(12)
    cost = rng.uniform(0, 20, size=(9, 8, 10))
    a = orc.run(cost, 2, 5, 3.3, 2.6, want_msgs=True)
    b = orc.run(cost, 2, 5, 3.3, 2.6, want_msgs=True, brute=True)
    np.testing.assert_allclose(a["msgs"], b["msgs"], rtol=0, atol=1e-12)


def test_pyramid_closed_form(orc):
    L, H, W = 3, 7, 9
    cost = np.full((L, H, W), 2.0)
    for lev in range(4):
        p = orc.pyramid(cost, lev)
        w, h = W, H
        for _ in range(lev):
            w, h = (w + 1) // 2, (h + 1) // 2
        assert p.shape == (L, h, w)
        # Interior blocks hold 4^lev children of value 2; the count per pixel is
        # the product of per-axis child counts, computed independently.
        def counts(n, lev):
            c = np.ones(n, int)
            for _ in range(lev):
                c = np.add.reduceat(c, np.arange(0, len(c), 2))
            return c
        cnt = counts(H, lev)[:, None] * counts(W, lev)[None, :]
        np.testing.assert_array_equal(p[0], 2.0 * cnt)


def test_pyramid_sum_random(orc):
    rng = np.random.default_rng(1)
    cost = rng.integers(0, 9, size=(4, 5, 7)).astype(float)
    p1 = orc.pyramid(cost, 1)
    pad = np.zeros((4, 6, 8))
    pad[:, :5, :7] = cost
    ref = pad.reshape(4, 3, 2, 4, 2).sum(axis=(2, 4))
    np.testing.assert_array_equal(p1, ref)


@pytest.mark.parametrize("W,H", [(13, 9), (12, 10)])
def test_two_level_plumbing(orc, W, H):
    """levels=2 equals: BP on the summed coarse cost, each fine pixel starting
    from its parent's final messages, then BP at the fine level."""
    rng = np.random.default_rng(W + H)
    L, K = 6, 5
    cost = rng.integers(0, 20, size=(L, H, W)).astype(float)
    two = orc.run(cost, 2, K, 4.0, 2.0, want_msgs=True)
    pad = np.zeros((L, H + H % 2, W + W % 2))
    pad[:, :H, :W] = cost
    coarse = pad.reshape(L, (H + 1) // 2, 2, (W + 1) // 2, 2).sum(axis=(2, 4))
    c_res = orc.run(coarse, 1, K, 4.0, 2.0, want_msgs=True)
    init = c_res["msgs"][:, :, np.arange(H)[:, None] // 2, np.arange(W)[None, :] // 2]
    fine = orc.run(cost, 1, K, 4.0, 2.0, msgs_init=init, want_msgs=True)
    np.testing.assert_array_equal(two["msgs"], fine["msgs"])
    np.testing.assert_array_equal(two["disp"], fine["disp"])


def test_levels_one_is_plain(orc):
    rng = np.random.default_rng(6)
    cost = rng.integers(0, 20, size=(5, 6, 8)).astype(float)
    a = orc.run(cost, 1, 4, 3.0, 2.0, want_msgs=True)
    b = orc.run(cost, 1, 4, 3.0, 2.0, want_msgs=True, msgs_init=np.zeros((4, 5, 6, 8)))
    np.testing.assert_array_equal(a["msgs"], b["msgs"])


def test_zero_iterations_reads_cost(orc):
    rng = np.random.default_rng(10)
    cost = rng.integers(0, 20, size=(5, 6, 8)).astype(float)
    res = orc.run(cost, 1, 0, 3.0, 2.0, want_msgs=True)
    assert (res["msgs"] == 0).all()
    np.testing.assert_array_equal(res["disp"], np.argmin(cost, axis=0))


def test_loopy_energy_not_below_map(orc):
    rng = np.random.default_rng(13)
    L, H, W = 3, 3, 3
    cost = rng.integers(0, 10, size=(L, H, W)).astype(float)
    V = _pins.vpair(3.0, 2.0, L)
    edges = _pins.edges_of(W, H)
    _, best_e, best_lab = _pins.enumerate_min_marginals(cost, edges, V)
    res = orc.run(cost, 1, 30, 3.0, 2.0)
    assert _pins.energy(res["disp"], cost, edges, V) >= best_e


def test_soft_argmin_closed_forms(orc):
    # Two labels on one pixel: weight of label 1 is 1 / (1 + exp((b1 - b0) / T)).
    cost = np.array([[[0.0]], [[0.7]]])
    res = orc.run(cost, 1, 0, 1.0, 2.0, want_soft=True, temperature=0.5)
    assert abs(res["soft"][0, 0] - 1.0 / (1.0 + np.exp(0.7 / 0.5))) < 1e-15
    # Constant beliefs: the mean label.
    cost = np.full((9, 3, 4), 5.0)
    res = orc.run(cost, 1, 3, 1.0, 2.0, want_soft=True, temperature=0.5)
    np.testing.assert_allclose(res["soft"], 4.0, rtol=0, atol=1e-14)
    # Temperature to zero: the argmin.
    rng = np.random.default_rng(1)
    cost = rng.integers(0, 30, size=(7, 4, 5)).astype(float)
    res = orc.run(cost, 1, 3, 2.0, 2.0, want_soft=True, temperature=1e-3)
    np.testing.assert_allclose(res["soft"], res["disp"], rtol=0, atol=1e-12)


def test_recovery_slanted_planes(orc):
    """Sanity bound, not parity: the oracle recovers the planes' disparities."""
    from synth import workload
    w = workload("planes160x120_L32")
    cost = orc.cost_volume(w["left"], w["right"], 32, 20.0)
    res = orc.run(cost, 1, 10, 10.0, 2.0)
    m = ~w["edge"]
    m[:, :31] = False
    good = np.abs(res["disp"] - w["gt"]) <= 1.0
    assert good[m].mean() >= 0.90
