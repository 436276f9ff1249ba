"""Pins of the oracle's triangulation (Eq. 3) by the projection it inverts.

Eq. 3's first line maps a camera-frame point (x, y, z) to its pixel (u, v)
and disparity d; the oracle inverts it.  The checks: a hand-worked pixel,
the round trip through the first line (which fixes the reading of the
garbled last entry of the second line: with f B / du there, depth would come
out B times too large), a plane of constant depth, the disparity scale, and
non-positive disparities.
"""
import numpy as np
import pytest

import oracle

CAM = dict(baseline=0.5, focal=3.0e-3, du=1.5e-6, dv=1.6e-6, u0=1352.0, v0=760.0)


def project(p, cam):
    """Eq. 3, first line: [u, v, d] = (1/z)[f x/du, f y/dv, f B/du] + [u0, v0, 0]."""
    x, y, z = p[..., 0], p[..., 1], p[..., 2]
    f, B = cam["focal"], cam["baseline"]
    return (f * x / (cam["du"] * z) + cam["u0"], f * y / (cam["dv"] * z) + cam["v0"], f * B / (cam["du"] * z))


def test_worked_pixel():
    # f / du = 2000 px.  d = 20 px at (u, v) = (1500, 900), square pixels:
    # z = 0.5 * 2000 / 20 = 50, x = (0.5 / 20) * 148 = 3.7, y = (0.5 / 20) * 140 = 3.5.
    cam = dict(CAM, dv=1.5e-6)
    disp = np.zeros((901, 1501))
    disp[900, 1500] = 20.0
    p = oracle.triangulate(disp, 1.0, **cam)
    np.testing.assert_allclose(p[900, 1500], [3.7, 3.5, 50.0], rtol=1e-12)


def test_round_trip_through_the_projection():
    rng = np.random.default_rng(4)
    h, w, scale = 37, 53, 4.0
    disp = rng.uniform(0.25, 64.0, size=(h, w))
    p = oracle.triangulate(disp, scale, **CAM)
    u, v, d = project(p, CAM)
    uu, vv = np.meshgrid(np.arange(w, dtype=np.float64), np.arange(h, dtype=np.float64))
    np.testing.assert_allclose(u, uu, rtol=0, atol=1e-9)
    np.testing.assert_allclose(v, vv, rtol=0, atol=1e-9)
    np.testing.assert_allclose(d, scale * disp, rtol=1e-12)


def test_plane_of_constant_depth():
    h, w, z0, scale = 20, 30, 80.0, 2.0
    d = CAM["focal"] * CAM["baseline"] / (z0 * CAM["du"])        # pixels
    p = oracle.triangulate(np.full((h, w), d / scale), scale, **CAM)
    np.testing.assert_allclose(p[..., 2], z0, rtol=1e-12)
    u = np.arange(w, dtype=np.float64)
    np.testing.assert_allclose(p[5, :, 0], (u - CAM["u0"]) * z0 * CAM["du"] / CAM["focal"], rtol=1e-12)


def test_disparity_scale():
    disp = np.full((3, 4), 7.0)
    a = oracle.triangulate(disp, 1.0, **CAM)
    b = oracle.triangulate(disp, 2.0, **CAM)
    np.testing.assert_allclose(b, a / 2.0, rtol=1e-12)


@pytest.mark.parametrize("val", [0.0, -3.0])
def test_no_finite_depth_is_nan(val):
    disp = np.full((2, 2), 5.0)
    disp[1, 0] = val
    p = oracle.triangulate(disp, 1.0, **CAM)
    assert np.isnan(p[1, 0]).all()
    assert np.isfinite(p[0, 0]).all() and np.isfinite(p[1, 1]).all()
