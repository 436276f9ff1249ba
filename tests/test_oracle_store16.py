"""Pins of where the oracle rounds 16-bit message storage (precision form).

Reading of the precision form (Eq. 1 messages stored in FP16 or BF16, with
FP32-or-better arithmetic): every sent message and every parent copy into a
16-bit level is rounded to nearest-even in the storage format, after
normalisation; the coarsest level keeps full precision.  An independent numpy
checkerboard BP (O(L^2) min-plus messages, tests/_pins.py) rounds at those
points with numpy's binary16 and torch's bfloat16 conversions, and the oracle
must reproduce it bit for bit on real-valued costs, where rounding is visible.
"""
import numpy as np
import pytest

import _pins

LAM, TAU = 7.3, 2.6


def _cost(seed, L, H, W):
    return np.random.default_rng(seed).uniform(0.0, 20.0, size=(L, H, W))


def test_round_helpers_round_once():
    """The reference's rounding goes from FP64 straight to the format (no
    double rounding through float32)."""
    x = 1.0 + 2.0 ** -8 + 2.0 ** -30          # just above a bfloat16 midpoint
    assert _pins.round_bf16(np.array([x]))[0] == 1.0 + 2.0 ** -7
    y = 1.0 + 2.0 ** -11 + 2.0 ** -40         # just above a binary16 midpoint
    assert _pins.round_f16(np.array([y]))[0] == 1.0 + 2.0 ** -10
    z = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8])   # exact midpoints: ties to even
    np.testing.assert_array_equal(_pins.round_bf16(z), [1.0, 1.0 + 2.0 ** -6])


def _representable(a, rnd):
    return np.array_equal(rnd(a), a)


@pytest.mark.parametrize("mode", [1, 2])
def test_coarsest_level_keeps_full_precision(orc, mode):
    """With one level, the only level is the coarsest: 16-bit modes must equal
    the FP64 run, whose messages are not 16-bit values."""
    cost = _cost(1, 9, 8, 11)
    full = orc.run(cost, 1, 5, LAM, TAU, want_msgs=True)
    s16 = orc.run(cost, 1, 5, LAM, TAU, store_mode=mode, want_msgs=True)
    np.testing.assert_array_equal(s16["msgs"], full["msgs"])
    ref = _pins.hierarchical_bp(cost, 1, 5, LAM, TAU)
    np.testing.assert_allclose(full["msgs"], ref, rtol=0, atol=1e-12)
    rnd = _pins.round_f16 if mode == 1 else _pins.round_bf16
    assert not _representable(full["msgs"], rnd)


@pytest.mark.parametrize("mode,levels,iters,shape", [
    (1, 2, 1, (9, 10, 13)),    # K = 1: half the finest slots keep the rounded parent copy
    (1, 2, 4, (9, 10, 13)),
    (1, 3, 3, (7, 13, 11)),
    (2, 2, 1, (9, 10, 13)),
    (2, 2, 4, (9, 10, 13)),
    (2, 3, 3, (7, 13, 11)),
])
def test_rounding_points_match_reference(orc, mode, levels, iters, shape):
    L, H, W = shape
    cost = _cost(10 * levels + iters + mode, L, H, W)
    rnd = _pins.round_f16 if mode == 1 else _pins.round_bf16
    got = orc.run(cost, levels, iters, LAM, TAU, store_mode=mode, want_msgs=True)
    ref = _pins.hierarchical_bp(cost, levels, iters, LAM, TAU, rnd=rnd)
    np.testing.assert_array_equal(got["msgs"], ref)
    # Every finest-level message is a 16-bit value, and rounding changed them.
    assert _representable(got["msgs"], rnd)
    full = orc.run(cost, levels, iters, LAM, TAU, want_msgs=True)
    assert not np.array_equal(got["msgs"], full["msgs"])
    b = cost + ref.sum(axis=0)
    np.testing.assert_array_equal(got["disp"], np.argmin(b, axis=0))


def test_reference_without_rounding_matches_fp64(orc):
    """The same reference with no rounding is the FP64 oracle (up to the
    order of FP64 operations), at two and three levels."""
    for levels, iters in ((2, 3), (3, 2)):
        cost = _cost(40 + levels, 6, 9, 12)
        got = orc.run(cost, levels, iters, LAM, TAU, want_msgs=True)
        ref = _pins.hierarchical_bp(cost, levels, iters, LAM, TAU)
        np.testing.assert_allclose(got["msgs"], ref, rtol=0, atol=1e-12)
