"""GPU parity of the radial-only undistortion (Sec. 2.1) against the oracle.

The u8 output is decided in FP32 by the same sequence of operations on both
sides (no fused multiply-adds), so the comparison is bit for bit: zero
distortion, barrel and pincushion coefficients, grey and RGB, ragged sizes
and the full 2704x1520 RGB frame of the benchmarked pair.
"""
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


@pytest.mark.parametrize("w,h,C,K", [
    (67, 41, 1, (50.0, 55.0, 33.5, 20.0, 0.0, 0.0, 0.0)),
    (200, 150, 3, (180.0, 170.0, 99.5, 74.5, -0.2, 0.05, 0.0)),
    (201, 97, 3, (150.0, 150.0, 100.0, 48.0, 0.15, -0.02, 0.003)),
    (129, 257, 1, (120.0, 110.0, 64.25, 128.75, -0.35, 0.12, -0.01)),
    (5, 3, 3, (2.0, 2.0, 2.0, 1.0, 0.3, 0.0, 0.0)),
])
def test_undistort_exact(dev, w, h, C, K):
    import paper_1902_09733_amd as bp
    rng = np.random.default_rng(w * h + C)
    img = rng.integers(0, 256, size=(h, w) + ((3,) if C == 3 else ()), dtype=np.uint8)
    out = bp.undistort(torch.from_numpy(img).to(dev), bp.Intrinsics(*K))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), oracle.undistort(img, *K))


def test_undistort_full_frame_exact(dev):
    import paper_1902_09733_amd as bp
    w = workload("aerial2704x1520_s4_L64")
    K = (1600.0, 1600.0, 1351.5, 759.5, -0.12, 0.02, -0.001)
    out = bp.undistort(torch.from_numpy(w["left"]).to(dev), bp.Intrinsics(*K))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), oracle.undistort(w["left"], *K))


def test_undistort_unaligned_input(dev):
    """An input at an odd address takes the byte-load path; same result."""
    import paper_1902_09733_amd as bp
    rng = np.random.default_rng(7)
    h, w = 61, 90
    img = rng.integers(0, 256, size=(h, w, 3), dtype=np.uint8)
    K = (80.0, 85.0, 44.5, 30.0, -0.25, 0.04, 0.0)
    buf = torch.empty(img.size + 1, dtype=torch.uint8, device=dev)
    src = buf[1:].view(h, w, 3)
    src.copy_(torch.from_numpy(img))
    assert src.data_ptr() % 4 != 0
    out = bp.undistort(src, bp.Intrinsics(*K))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), oracle.undistort(img, *K))
