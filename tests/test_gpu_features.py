"""GPU parity of the Harris response, per-cell corner selection and ZSSD
matching (Sec. 2.3, Eq. 4-5) against the integer oracle: bit for bit, since
every quantity is an exact integer on both sides."""
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
    return torch.device("cuda:0")


def grey(rgb):
    return ((rgb[..., 0].astype(np.int32) * 77 + rgb[..., 1].astype(np.int32) * 150 +
             rgb[..., 2].astype(np.int32) * 29) >> 8).astype(np.uint8)


def corners_np(out):
    return np.stack([out["x"].cpu().numpy(), out["y"].cpu().numpy(), out["corner_response"].cpu().numpy()],
                    axis=1).astype(np.int64)


@pytest.mark.parametrize("w,h,g,thr", [(67, 45, 5, 0), (130, 97, 30, 10 ** 9), (33, 20, 40, -5), (16, 16, 1, 0)])
def test_harris_exact(dev, w, h, g, thr):
    import paper_1902_09733_amd as bp
    rng = np.random.default_rng(w + h)
    img = rng.integers(0, 256, size=(h, w), dtype=np.uint8)
    img[h // 3:2 * h // 3, w // 4:w // 2] = 230
    out = bp.harris(torch.from_numpy(img).to(dev), grid=g, threshold=thr)
    torch.cuda.synchronize()
    r = oracle.harris_response(img)
    np.testing.assert_array_equal(out["response"].cpu().numpy(), r)
    np.testing.assert_array_equal(corners_np(out), oracle.harris_cells(r, g, thr))


def test_harris_and_zssd_full_frame(dev):
    """The benchmarked pair's left frame (grey, 2704x1520), a 30 x 30 grid,
    and ZSSD matches of its corners in the right frame."""
    import paper_1902_09733_amd as bp
    w = workload("aerial2704x1520_s4_L64")
    a, b = grey(w["left"]), grey(w["right"])
    thr = 2 * 10 ** 7                             # about the 97th percentile of 25 R on this frame
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    out = bp.harris(ta, grid=30, threshold=thr)
    m = bp.zssd_match(ta, tb, out["raw"], patch_radius=5, search_radius=16)
    torch.cuda.synchronize()
    r = oracle.harris_response(a)
    np.testing.assert_array_equal(out["response"].cpu().numpy(), r)
    c = oracle.harris_cells(r, 30, thr)
    np.testing.assert_array_equal(corners_np(out), c)
    assert (c[:, 0] >= 0).sum() > 800           # the scene is textured: nearly every cell has a corner
    om = oracle.zssd_match(a, b, c, 5, 16)
    gm = np.stack([m["x"].cpu().numpy(), m["y"].cpu().numpy(), m["cost"].cpu().numpy()], axis=1)
    np.testing.assert_array_equal(gm, om)


@pytest.mark.parametrize("pr,sr", [(0, 0), (2, 5), (7, 32), (15, 3)])
def test_zssd_edges(dev, pr, sr):
    import paper_1902_09733_amd as bp
    rng = np.random.default_rng(pr * 100 + sr)
    h, w = 70, 90
    a = rng.integers(0, 256, size=(h, w), dtype=np.uint8)
    b = np.roll(a, (2, -3), axis=(0, 1))
    pts = np.array([[45, 35], [1, 1], [w - 2, h - 2], [20, 60], [-1, -1], [pr, pr], [w - 1 - pr, h - 1 - pr]])
    raw = np.zeros((len(pts), 2), dtype=np.int64)
    raw[:, 0] = (pts[:, 0] & 0xffffffff) | (pts[:, 1].astype(np.int64) << 32)
    corners = np.concatenate([pts, np.zeros((len(pts), 1), dtype=np.int64)], axis=1)
    m = bp.zssd_match(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), torch.from_numpy(raw).to(dev),
                      patch_radius=pr, search_radius=sr)
    torch.cuda.synchronize()
    om = oracle.zssd_match(a, b, corners, pr, sr)
    gm = np.stack([m["x"].cpu().numpy(), m["y"].cpu().numpy(), m["cost"].cpu().numpy()], axis=1)
    np.testing.assert_array_equal(gm, om)
