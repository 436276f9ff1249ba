"""Seeded synthetic rectified stereo pairs.

This module only draws inputs: textures, scene geometry, ground-truth
disparities and the warped right view.  It contains none of the stereo
method's arithmetic (no cost volume, no message passing, no upsampling), so
both the FP64 oracle's tests and the GPU path's tests and benchmark may use
it as their common input source.

Two scene families stand in for the paper's UAV footage (the author's flight
data is not available): slanted planes over value-noise texture, and a nadir
view of a terrain heightfield with box-shaped buildings.  The full-resolution
frame size 2704x1520 is the GoPro 2.7K format of Sec. 2.2; the low-resolution
matching grid and label counts follow the stereo workloads this library is
benchmarked on.  Left is the reference view; a left pixel (x, y) with
disparity d is seen at (x - d, y) in the right view.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "value_noise",
    "slanted_planes",
    "aerial",
    "batch_specs",
    "jitter",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def value_noise(width: int, height: int, rng: np.random.Generator, octaves: int = 5,
                base_period: float = 32.0, persistence: float = 0.5) -> np.ndarray:
    """Octave sum of bilinearly interpolated random lattices, rescaled to [0, 1]."""
    out = np.zeros((height, width), dtype=np.float64)
    amp = 1.0
    period = float(base_period)
    ys = np.arange(height, dtype=np.float64)
    xs = np.arange(width, dtype=np.float64)
    for _ in range(octaves):
        gw = int(np.ceil(width / period)) + 2
        gh = int(np.ceil(height / period)) + 2
        lattice = rng.random((gh, gw))
        fx = xs / period
        fy = ys / period
        x0 = np.floor(fx).astype(np.int64)
        y0 = np.floor(fy).astype(np.int64)
        tx = (fx - x0)[None, :]
        ty = (fy - y0)[:, None]
        a = lattice[y0[:, None], x0[None, :]]
        b = lattice[y0[:, None], x0[None, :] + 1]
        c = lattice[y0[:, None] + 1, x0[None, :]]
        d = lattice[y0[:, None] + 1, x0[None, :] + 1]
        out += amp * ((a * (1 - tx) + b * tx) * (1 - ty) + (c * (1 - tx) + d * tx) * ty)
        amp *= persistence
        period = max(period / 2.0, 1.0)
    lo, hi = out.min(), out.max()
    return (out - lo) / max(hi - lo, 1e-12)


def _sample_x(img: np.ndarray, xs: np.ndarray) -> np.ndarray:
    """Linear interpolation of ``img`` along x at positions ``xs`` [H][W]."""
    h, w = xs.shape
    xs = np.clip(xs, 0.0, w - 1.0)
    x0 = np.floor(xs).astype(np.int64)
    x1 = np.minimum(x0 + 1, w - 1)
    t = xs - x0
    rows = np.arange(h)[:, None]
    if img.ndim == 3:
        t = t[..., None]
    return img[rows, x0] * (1 - t) + img[rows, x1] * t


def _warp_right(left: np.ndarray, disp: np.ndarray, rng: np.random.Generator,
                noise_sigma: float) -> np.ndarray:
    """Right view of a left view with disparity ``disp`` (left coordinates).

    A right pixel x' shows the left pixel x with x - d(x) = x'.  The right-view
    disparity d_R(x') = d(x' + d_R(x')) is found by fixed-point iteration, then
    Right(x', y) = Left(x' + d_R(x', y), y), linear in x, plus Gaussian noise.
    ``left`` is float [H][W] or [H][W][C] in 0..255, ``disp`` is [H][W].
    """
    h, w = disp.shape
    base = np.arange(w, dtype=np.float64)[None, :]
    d_r = disp.copy()
    for _ in range(12):
        d_r = _sample_x(disp, base + d_r)
    right = _sample_x(left, base + d_r)
    right = right + rng.normal(0.0, noise_sigma, size=right.shape)
    return np.clip(np.rint(right), 0, 255).astype(np.uint8)


def slanted_planes(width: int, height: int, num_labels: int, seed: int,
                   n_planes: int = 4, noise_sigma: float = 2.0):
    """Grey pair over ``n_planes`` slanted planes on a seeded Voronoi partition.

    Returns ``(left u8 [H][W], right u8 [H][W], gt float64 [H][W], edge bool
    [H][W])``; ``edge`` marks a 2-pixel band around plane boundaries, where the
    backward warp is not a faithful view.
    """
    rng = _rng(seed)
    tex = value_noise(width, height, rng, octaves=5, base_period=32.0, persistence=0.5)
    left_f = tex * 255.0
    sites = rng.random((n_planes, 2)) * np.array([width, height])
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float64)
    dist = (xx[None] - sites[:, 0, None, None]) ** 2 + (yy[None] - sites[:, 1, None, None]) ** 2
    region = np.argmin(dist, axis=0)
    dmax = float(num_labels - 1)
    gt = np.zeros((height, width))
    for k in range(n_planes):
        a = rng.uniform(-0.06, 0.06) * 160.0 / width
        b = rng.uniform(-0.06, 0.06) * 120.0 / height
        c = rng.uniform(0.15, 0.85) * dmax
        cx, cy = sites[k]
        plane = c + a * (xx - cx) + b * (yy - cy)
        gt = np.where(region == k, plane, gt)
    gt = np.clip(gt, 0.0, dmax)
    left = np.clip(np.rint(left_f), 0, 255).astype(np.uint8)
    right = _warp_right(left.astype(np.float64), gt, rng, noise_sigma)
    edge = np.zeros_like(region, dtype=bool)
    diff_x = region[:, 1:] != region[:, :-1]
    diff_y = region[1:, :] != region[:-1, :]
    edge[:, 1:] |= diff_x
    edge[:, :-1] |= diff_x
    edge[1:, :] |= diff_y
    edge[:-1, :] |= diff_y
    for _ in range(1):
        grown = edge.copy()
        grown[:, 1:] |= edge[:, :-1]
        grown[:, :-1] |= edge[:, 1:]
        grown[1:, :] |= edge[:-1, :]
        grown[:-1, :] |= edge[1:, :]
        edge = grown
    return left, right, gt, edge


def aerial(width: int, height: int, num_labels: int, seed: int, channels: int = 3,
           n_boxes: int = 12, disparity_scale: float = 1.0, noise_sigma: float = 2.0):
    """Nadir view over an fBm heightfield with ``n_boxes`` box buildings.

    Disparity is an affine function of 1/depth, scaled so that it spans
    ``[0, (num_labels - 1) * disparity_scale]`` at this resolution (a frame
    rendered at 4x the matching grid passes ``disparity_scale=4``).  The albedo
    is value noise per channel shaded by the heightfield normal.  Returns
    ``(left u8 [H][W][C] or [H][W], right (same), gt float64 [H][W])``.
    """
    rng = _rng(seed)
    period = max(width, height) / 4.0
    terrain = value_noise(width, height, rng, octaves=6, base_period=period, persistence=0.5)
    height_m = 25.0 * terrain
    scale = max(width, height) / 2704.0
    for _ in range(n_boxes):
        bw = int(rng.integers(40, 251) * scale) + 2
        bh = int(rng.integers(40, 251) * scale) + 2
        x0 = int(rng.integers(0, max(width - bw, 1)))
        y0 = int(rng.integers(0, max(height - bh, 1)))
        roof = float(rng.uniform(8.0, 30.0))
        base = height_m[y0:y0 + bh, x0:x0 + bw].max()
        height_m[y0:y0 + bh, x0:x0 + bw] = base + roof
    altitude = 100.0
    depth = altitude - height_m
    inv = 1.0 / depth
    lo, hi = inv.min(), inv.max()
    gt = (inv - lo) / max(hi - lo, 1e-12) * (num_labels - 1) * disparity_scale
    gy, gx = np.gradient(height_m)
    nz = 1.0 / np.sqrt(gx * gx + gy * gy + 1.0)
    light = np.array([0.4, -0.3, 0.87])
    light = light / np.linalg.norm(light)
    shade = np.clip((-gx * light[0] - gy * light[1] + light[2]) * nz, 0.25, 1.0)
    if channels == 3:
        albedo = np.stack([value_noise(width, height, rng, octaves=6,
                                       base_period=max(8.0, 48.0 * scale)) for _ in range(3)], axis=-1)
        tint = rng.uniform(0.5, 1.0, size=3)
        left_f = 255.0 * np.clip(0.15 + 0.85 * albedo * tint[None, None, :], 0, 1) * shade[..., None]
    else:
        albedo = value_noise(width, height, rng, octaves=6, base_period=max(8.0, 48.0 * scale))
        left_f = 255.0 * np.clip(0.15 + 0.85 * albedo, 0, 1) * shade
    left = np.clip(np.rint(left_f), 0, 255).astype(np.uint8)
    right = _warp_right(left.astype(np.float64), gt, rng, noise_sigma)
    return left, right, gt


def jitter(shape, seed: int, high: float = 0.5) -> np.ndarray:
    """Seeded U(0, high) float64 array, used to break ties in real-valued costs."""
    return _rng(seed).uniform(0.0, high, size=shape)


def batch_specs(count: int = 48, seed: int = 3):
    """Sizes and label counts of a mixed serving-style batch.

    W ~ U{320..1352}, H = floor(9W/16) (320x180 .. 1352x760), L ~ U{32,64,96,128}.
    Returns a list of ``(width, height, num_labels, pair_seed)``.
    """
    rng = _rng(seed)
    out = []
    for i in range(count):
        w = int(rng.integers(320, 1353))
        h = (9 * w) // 16
        lab = int(rng.choice([32, 64, 96, 128]))
        out.append((w, h, lab, seed * 1000 + i))
    return out
