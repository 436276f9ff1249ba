"""Pins of the oracle's radial-only undistortion with bilinear sampling
(Sec. 2.1: undistort-and-remap of every frame with the calibrated radial
model).  Checked against what the model and bilinear interpolation fix on
their own: zero distortion is the identity, a hand-worked pixel, and an
intensity ramp sampled at the model's source points computed independently
in FP64 with an independent bilinear interpolation.
"""
import numpy as np
import pytest

import oracle


def source_points(w, h, fx, fy, cx, cy, k1, k2, k3):
    """FP64 source position of every output pixel: the pinhole projection of
    the radially scaled normalised point, fx * xn * g + cx."""
    u, v = np.meshgrid(np.arange(w, dtype=np.float64), np.arange(h, dtype=np.float64))
    xn, yn = (u - cx) / fx, (v - cy) / fy
    r2 = xn * xn + yn * yn
    g = 1.0 + k1 * r2 + k2 * r2 ** 2 + k3 * r2 ** 3
    return fx * xn * g + cx, fy * yn * g + cy


@pytest.mark.parametrize("C", [1, 3])
def test_zero_distortion_is_identity(C):
    rng = np.random.default_rng(C)
    img = rng.integers(0, 256, size=(41, 67) + ((3,) if C == 3 else ()), dtype=np.uint8)
    out = oracle.undistort(img, 50.0, 55.0, 33.5, 20.0)
    np.testing.assert_array_equal(out, img)


def test_worked_pixel():
    # fx = fy = 100, principal point at the origin, k1 = 0.1: output (50, 0)
    # has xn = 0.5, r2 = 0.25, g = 1.025 and samples (51.25, 0), a quarter of
    # the way from 100 to 200.
    img = np.zeros((4, 60), dtype=np.uint8)
    img[0, 51], img[0, 52] = 100, 200
    out = oracle.undistort(img, 100.0, 100.0, 0.0, 0.0, k1=0.1)
    assert out[0, 50] == 125


@pytest.mark.parametrize("k", [(-0.2, 0.05, 0.0), (0.15, -0.02, 0.003), (-0.35, 0.12, -0.01)])
def test_ramp_at_model_points(k):
    w, h = 200, 150
    fx, fy, cx, cy = 180.0, 170.0, 99.5, 74.5
    u, v = np.meshgrid(np.arange(w), np.arange(h))
    ramp = (u + 0.25 * v + 5).astype(np.uint8)                 # exact: at most 241
    out = oracle.undistort(ramp, fx, fy, cx, cy, *k).astype(np.float64)
    us, vs = source_points(w, h, fx, fy, cx, cy, *k)
    inside = (us >= 0) & (vs >= 0) & (us <= w - 1) & (vs <= h - 1)
    # A float-rounding hair from the border can flip inside/outside; skip that rim.
    rim = (np.abs(us) < 1e-3) | (np.abs(vs) < 1e-3) | (np.abs(us - (w - 1)) < 1e-3) | (np.abs(vs - (h - 1)) < 1e-3)
    # The u8 ramp truncates 0.25 v, so the reference is the FP64 bilinear
    # value of that integer image at the FP64 model points (FP32 rounding
    # may move a value across a .5 boundary: at most one level, rarely).
    expect = np.floor(bilinear(ramp.astype(np.float64), us, vs) + 0.5)
    m = inside & ~rim
    assert np.abs(out[m] - expect[m]).max() <= 1.0
    assert (out[m] == expect[m]).mean() >= 0.999
    assert (out[~inside & ~rim] == 0).all()
    # The distortion is visible: far from the centre the samples move by pixels.
    assert np.abs(us - u).max() > 5


def bilinear(img, us, vs):
    h, w = img.shape
    x0 = np.clip(np.floor(us).astype(int), 0, w - 1)
    y0 = np.clip(np.floor(vs).astype(int), 0, h - 1)
    x1, y1 = np.minimum(x0 + 1, w - 1), np.minimum(y0 + 1, h - 1)
    ax, ay = us - x0, vs - y0
    top = img[y0, x0] * (1 - ax) + img[y0, x1] * ax
    bot = img[y1, x0] * (1 - ax) + img[y1, x1] * ax
    return top * (1 - ay) + bot * ay
