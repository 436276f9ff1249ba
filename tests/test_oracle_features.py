"""Pins of the oracle's Harris response (Eq. 4-5), per-cell corner selection
and ZSSD matching (Sec. 2.3) by what the mathematics fixes: closed forms on
images whose derivatives are known (a ramp: det M = 0; the saddle x*y, where
the binomial window's unit variance enters), exact symmetries and scalings,
corner positions of a bright square, brute force of the selection rule on
small inputs, and shift recovery by ZSSD with an intensity offset.
"""
import numpy as np
import pytest

import oracle


def test_ramp_closed_form():
    # I = 3x + 2y: A = 6, B = 4 everywhere, window weights sum to 256, so
    # M = 256 [[36, 24], [24, 16]], det M = 0 and 25 R = -(256 * 52)^2.
    x, y = np.meshgrid(np.arange(40), np.arange(30))
    r = oracle.harris_response((3 * x + 2 * y).astype(np.uint8))
    np.testing.assert_array_equal(r[3:-3, 3:-3], -(256 * 52) ** 2)
    assert (r[:3] == 0).all() and (r[:, -3:] == 0).all()


def test_saddle_closed_form():
    # I = x y: A = 2y, B = 2x; with the binomial window (weights 1 4 6 4 1,
    # mean offset 0, variance 1 per axis): M = 1024 [[y^2+1, xy], [xy, x^2+1]],
    # det M = 1024^2 (x^2 + y^2 + 1), tr M = 1024 (x^2 + y^2 + 2).
    n = 16
    x, y = np.meshgrid(np.arange(n, dtype=np.int64), np.arange(n, dtype=np.int64))
    r = oracle.harris_response((x * y).astype(np.uint8))
    det = 1024 ** 2 * (x * x + y * y + 1)
    tr = 1024 * (x * x + y * y + 2)
    np.testing.assert_array_equal(r[3:-3, 3:-3], (25 * det - tr * tr)[3:-3, 3:-3])


def test_symmetries_and_scaling():
    rng = np.random.default_rng(1)
    img = rng.integers(0, 128, size=(37, 45), dtype=np.uint8)
    r = oracle.harris_response(img)
    np.testing.assert_array_equal(oracle.harris_response(np.ascontiguousarray(img.T)), r.T)
    np.testing.assert_array_equal(oracle.harris_response(np.ascontiguousarray(img[::-1, ::-1])), r[::-1, ::-1])
    np.testing.assert_array_equal(oracle.harris_response(img + 100), r)          # offset invariance
    np.testing.assert_array_equal(oracle.harris_response(img * 2), 16 * r)       # degree 4 in I
    assert (oracle.harris_response(np.full((20, 20), 77, np.uint8)) == 0).all()


def test_bright_square_corners():
    img = np.zeros((60, 80), dtype=np.uint8)
    img[20:40, 25:55] = 200
    r = oracle.harris_response(img)
    c = oracle.harris_cells(r, grid=2, threshold=0)
    got = sorted((int(a), int(b)) for a, b, _ in c if a >= 0)
    want = [(24, 19), (24, 40), (55, 19), (55, 40)]      # just outside/inside each corner
    for (gx, gy), (wx, wy) in zip(got, sorted(want)):
        assert abs(gx - wx) <= 1 and abs(gy - wy) <= 1, (got, want)
    # Straight edges away from the corners respond negatively.
    assert r[30, 25] < 0 and r[20, 40] < 0


def brute_cells(r, g, thr):
    h, w = r.shape
    out = []
    for ci in range(g):
        for cj in range(g):
            best = None
            for yy in range(ci * h // g, (ci + 1) * h // g):
                for xx in range(cj * w // g, (cj + 1) * w // g):
                    v = r[yy, xx]
                    nb = r[max(yy - 1, 0):yy + 2, max(xx - 1, 0):xx + 2]
                    if v > thr and v >= nb.max() and (best is None or v > best[2]):
                        best = (xx, yy, v)
            out.append(best if best else (-1, -1, 0))
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("seed,g,thr", [(0, 3, 0), (1, 4, 5), (2, 5, -3)])
def test_cell_selection_brute_force(seed, g, thr):
    rng = np.random.default_rng(seed)
    r = rng.integers(-10, 10, size=(23, 31)).astype(np.int64)      # many ties and plateaus
    np.testing.assert_array_equal(oracle.harris_cells(r, g, thr), brute_cells(r, g, thr))


def test_zssd_recovers_shift_with_offset():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 200, size=(64, 80), dtype=np.uint8)
    dy, dx = 3, -5
    b = np.roll(a, (dy, dx), axis=(0, 1)).astype(np.int64) + 40
    b = np.clip(b, 0, 255).astype(np.uint8)
    corners = np.array([[30, 30, 0], [40, 25, 0], [20, 44, 0], [2, 30, 0]], dtype=np.int64)
    m = oracle.zssd_match(a, b, corners, patch_radius=4, search_radius=7)
    for k in range(3):
        assert (m[k, 0], m[k, 1], m[k, 2]) == (corners[k, 0] + dx, corners[k, 1] + dy, 0)
    assert m[3, 0] == -1                      # the corner's own patch leaves the frame


def test_zssd_brute_force():
    rng = np.random.default_rng(4)
    a = rng.integers(0, 256, size=(30, 34), dtype=np.uint8)
    b = rng.integers(0, 256, size=(30, 34), dtype=np.uint8)
    pr, sr = 2, 3
    corners = np.array([[10, 12, 0], [20, 15, 0], [5, 5, 0]], dtype=np.int64)
    m = oracle.zssd_match(a, b, corners, pr, sr)
    n = (2 * pr + 1) ** 2
    for k, (cx, cy, _) in enumerate(corners):
        pa = a[cy - pr:cy + pr + 1, cx - pr:cx + pr + 1].astype(np.float64)
        best = None
        for dy in range(-sr, sr + 1):
            for dx in range(-sr, sr + 1):
                qx, qy = cx + dx, cy + dy
                if qx < pr or qy < pr or qx + pr >= 34 or qy + pr >= 30:
                    continue
                pb = b[qy - pr:qy + pr + 1, qx - pr:qx + pr + 1].astype(np.float64)
                z = ((pa - pa.mean()) - (pb - pb.mean())) ** 2
                cost = round(n * z.sum())
                if best is None or cost < best[2]:
                    best = (qx, qy, cost)
        assert tuple(m[k]) == best
