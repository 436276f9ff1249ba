"""Pins of the oracle's data term, downsampling, upsampling (Eq. 2) and storage rounding."""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_cost_worked_example(orc):
    g = json.load(open(os.path.join(GOLD, "cost_worked.json")))
    gr = g["grey"]
    c = orc.cost_volume(np.array(gr["left"], np.uint8), np.array(gr["right"], np.uint8),
                        gr["labels"], gr["trunc"])
    np.testing.assert_array_equal(c, np.array(gr["expected"], float))
    rgb = g["rgb"]
    l, r = np.array(rgb["left"], np.uint8), np.array(rgb["right"], np.uint8)
    np.testing.assert_array_equal(orc.cost_volume(l, r, 1, 20.0, rgb_mode=0),
                                  np.array(rgb["expected_rounded"], float))
    np.testing.assert_allclose(orc.cost_volume(l, r, 1, 20.0, rgb_mode=1),
                               np.array(rgb["expected_mean"], float), rtol=1e-15)


def test_cost_shifted_copy_is_zero_at_true_disparity(orc):
    rng = np.random.default_rng(0)
    right = rng.integers(0, 256, size=(6, 40), dtype=np.uint8)
    d0 = 5
    left = np.zeros_like(right)
    left[:, d0:] = right[:, :-d0]
    c = orc.cost_volume(left, right, 8, 20.0)
    assert (c[d0][:, d0:] == 0).all()
    assert (c[:, :, :1][1:] == 20).all()          # x - d < 0 -> truncation value
    assert c.max() <= 20 and c.min() >= 0


def test_downsample_worked_and_constant(orc):
    g = json.load(open(os.path.join(GOLD, "downsample_worked.json")))
    out = orc.downsample(np.array(g["input"], np.uint8), g["s"])
    np.testing.assert_array_equal(out, np.array(g["expected"]))
    img = np.full((8, 12, 3), 77, np.uint8)
    np.testing.assert_array_equal(orc.downsample(img, 4), np.full((2, 3, 3), 77))


def jbu_literal(disp, guide, s, sigma_s, sigma_r, R):
    """Eq. 2 written directly with unshifted Gaussian weights (small inputs)."""
    hl, wl = disp.shape
    hh, wh = guide.shape[:2]
    g = guide.astype(float).reshape(hh, wh, -1)
    out = np.zeros((hh, wh))
    for py in range(hh):
        for px in range(wh):
            pl = np.array([(px + 0.5) / s - 0.5, (py + 0.5) / s - 0.5])
            num = den = 0.0
            for qy in range(py // s - R, py // s + R + 1):
                for qx in range(px // s - R, px // s + R + 1):
                    if not (0 <= qx < wl and 0 <= qy < hl):
                        continue
                    sp = np.exp(-np.sum((s * (pl - [qx, qy])) ** 2) / (2 * sigma_s ** 2))
                    iq = g[s * qy + s // 2, s * qx + s // 2]
                    rg = np.exp(-np.sum((g[py, px] - iq) ** 2) / (2 * sigma_r ** 2))
                    num += disp[qy, qx] * sp * rg
                    den += sp * rg
            out[py, px] = num / den
    return out


def test_jbu_literal_small(orc):
    rng = np.random.default_rng(2)
    disp = rng.integers(0, 30, size=(4, 5)).astype(np.int32)
    guide = rng.integers(0, 256, size=(16, 20, 3), dtype=np.uint8)
    got = orc.upsample(disp, guide, sigma_s=6.0, sigma_r=40.0, radius=2)
    ref = jbu_literal(disp, guide, 4, 6.0, 40.0, 2)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_jbu_constant_disparity(orc):
    rng = np.random.default_rng(3)
    disp = np.full((6, 7), 13, np.int32)
    guide = rng.integers(0, 256, size=(24, 28, 3), dtype=np.uint8)
    np.testing.assert_allclose(orc.upsample(disp, guide, 8.0, 12.0), 13.0, rtol=0, atol=1e-12)


def test_jbu_range_to_infinity_is_spatial_gaussian(orc):
    """sigma_r -> infinity: the weights are the separable spatial Gaussian."""
    rng = np.random.default_rng(4)
    s, R, sig = 2, 2, 3.0
    disp = rng.integers(0, 20, size=(5, 6)).astype(np.int32)
    guide = rng.integers(0, 256, size=(10, 12), dtype=np.uint8)
    got = orc.upsample(disp, guide, sig, 1e12, R)
    hl, wl = disp.shape

    def axis_w(p, n):
        c = p // s
        q = np.arange(n)
        w = np.exp(-((p + 0.5 - s * q - s / 2) ** 2) / (2 * sig ** 2))
        w[(q < c - R) | (q > c + R)] = 0.0
        return w
    for py in range(10):
        for px in range(12):
            wy, wx = axis_w(py, hl), axis_w(px, wl)
            W2 = wy[:, None] * wx[None, :]
            assert abs(got[py, px] - (W2 * disp).sum() / W2.sum()) < 1e-9


def test_jbu_identity_at_unit_scale(orc):
    rng = np.random.default_rng(5)
    disp = rng.integers(0, 40, size=(9, 11)).astype(np.int32)
    guide = rng.integers(0, 256, size=(9, 11, 3), dtype=np.uint8)
    np.testing.assert_allclose(orc.upsample(disp, guide, 0.05, 12.0, 1), disp, rtol=0, atol=1e-9)


def test_jbu_no_underflow_at_strong_edges(orc):
    disp = np.array([[0, 50]], np.int32)
    guide = np.zeros((4, 8, 3), np.uint8)
    guide[:, 4:] = 255
    guide[0, 0] = 255   # isolated bright pixel far (in range) from both samples it sees
    out = orc.upsample(disp, guide, 8.0, 1.0, 1)
    assert np.isfinite(out).all()


def test_round_f16_matches_numpy(orc):
    rng = np.random.default_rng(6)
    xs = np.concatenate([rng.uniform(0, 100, 2000), rng.uniform(0, 1e-5, 500),
                         np.arange(0, 2048, 0.125)[:3000], [2049.0, 2051.0, 65504.0, 6e-8, 3e-8]])
    for x in xs:
        assert orc.round_f16(x) == float(np.float16(x)), x


def test_round_bf16_matches_torch(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    xs = np.concatenate([rng.uniform(0, 300, 3000), rng.uniform(0, 1e-3, 300)]).astype(np.float32)
    ref = torch.from_numpy(xs).to(torch.bfloat16).to(torch.float64).numpy()
    for x, r in zip(xs, ref):
        assert orc.round_bf16(float(x)) == r, x


def test_generator_deterministic():
    from synth import workload
    a = workload("planes160x120_L32")
    b = workload("planes160x120_L32")
    assert np.array_equal(a["left"], b["left"]) and np.array_equal(a["right"], b["right"])
    c = workload("planes160x120_L32", seed=99)
    assert not np.array_equal(a["left"], c["left"])
