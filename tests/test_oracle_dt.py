"""Pins of the oracle's message update (Eq. 1 messages, truncated-linear smoothness)."""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_dt_worked_examples(orc):
    cases = json.load(open(os.path.join(GOLD, "dt_worked.json")))["cases"]
    for c in cases:
        for brute in (False, True):
            got = orc.dt(np.array(c["h"], float), c["lambda"], c["tau"], brute=brute)
            np.testing.assert_array_equal(got, np.array(c["expected"], float), err_msg=str(c))


@pytest.mark.parametrize("L", [1, 2, 3, 7, 32, 64, 96, 128])
@pytest.mark.parametrize("tau", [0.5, 1.0, 2.0, 2.6, 200.0])
def test_dt_equals_bruteforce_integers(orc, L, tau):
    rng = np.random.default_rng(L * 1000 + int(tau * 10))
    lam = 10.0 if tau != 2.6 else 5.0
    for _ in range(20):
        h = rng.integers(0, 200, size=L).astype(float)
        a = orc.dt(h, lam, tau)
        b = orc.dt(h, lam, tau, brute=True)
        np.testing.assert_array_equal(a, b)
        # Normalised: min 0 and bounded by lambda * tau.
        assert a.min() == 0.0
        assert a.max() <= lam * tau


@pytest.mark.parametrize("L", [2, 5, 33, 128])
def test_dt_equals_bruteforce_reals(orc, L):
    rng = np.random.default_rng(7 + L)
    for tau in (0.3, 1.7, 2.6, 9.9):
        for lam in (0.0, 0.7, 7.3):
            h = rng.uniform(-50, 50, size=L)
            a = orc.dt(h, lam, tau)
            b = orc.dt(h, lam, tau, brute=True)
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * max(1.0, np.abs(h).max()))


def test_dt_numpy_definition_random(orc):
    """Min over g of h(g) + lam*min(|f-g|, tau) by broadcasting, minus the minimum."""
    rng = np.random.default_rng(3)
    for L in (4, 16, 64):
        h = rng.integers(0, 60, size=L).astype(float)
        f = np.arange(L)
        V = 10.0 * np.minimum(np.abs(f[:, None] - f[None, :]), 2.0)
        ref = np.min(h[None, :] + V, axis=1)
        ref -= ref.min()
        np.testing.assert_array_equal(orc.dt(h, 10.0, 2.0), ref)


def test_dt_zero_lambda_is_flat(orc):
    h = np.array([5.0, 1.0, 9.0, 3.0])
    np.testing.assert_array_equal(orc.dt(h, 0.0, 2.0), np.zeros(4))
