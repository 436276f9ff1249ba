"""Named stereo workloads: seeded inputs plus the method's parameters.

Each workload is named for what it is.  Inputs are u8 images (grey [H][W] or
RGB [H][W][3]); ``downsample`` is the integer factor the path applies before
matching (the paper matches on a downsampled copy of the 2.7K frames and
upsamples the result with the full-resolution colour image, Sec. 2.2).
Smoothness weight, truncation and data-cost truncation default to 10, 2 and 20.
"""
from __future__ import annotations

from .scenes import aerial, batch_specs, jitter, slanted_planes

__all__ = ["workload", "WORKLOADS"]

WORKLOADS = (
    "planes160x120_L32",
    "aerial2704x1520_s4_L64",
    "batch48_mixed",
    "aerial1352x760_L128",
    "planes320x240_L64_x8",
)


def _base(**kw):
    p = dict(data_trunc=20.0, lam=10.0, tau=2.0, levels=1, iters=10, downsample=1,
             sigma_s=8.0, sigma_r=12.0)
    p.update(kw)
    return p


def workload(name: str, seed: int | None = None, **overrides):
    """Build a named workload; returns a dict with inputs and parameters."""
    if name == "planes160x120_L32":
        s = 1 if seed is None else seed
        left, right, gt, edge = slanted_planes(160, 120, 32, s)
        w = _base(name=name, left=left, right=right, gt=gt, edge=edge, width=160, height=120,
                  channels=1, num_labels=32, levels=1, iters=10)
    elif name == "aerial2704x1520_s4_L64":
        s = 2 if seed is None else seed
        left, right, gt = aerial(2704, 1520, 64, s, channels=3, disparity_scale=4.0)
        w = _base(name=name, left=left, right=right, gt=gt / 4.0, width=2704, height=1520,
                  channels=3, num_labels=64, levels=5, iters=10, downsample=4,
                  sigma_s=8.0, sigma_r=12.0)
    elif name == "batch48_mixed":
        s = 3 if seed is None else seed
        pairs = []
        for (wd, ht, lab, ps) in batch_specs(48, s):
            left, right, gt = aerial(wd, ht, lab, ps, channels=3)
            pairs.append(dict(left=left, right=right, gt=gt, width=wd, height=ht, channels=3,
                              num_labels=lab))
        w = _base(name=name, pairs=pairs, levels=5, iters=8)
    elif name == "aerial1352x760_L128":
        s = 4 if seed is None else seed
        left, right, gt = aerial(1352, 760, 128, s, channels=3)
        w = _base(name=name, left=left, right=right, gt=gt, width=1352, height=760, channels=3,
                  num_labels=128, levels=6, iters=12)
    elif name == "planes320x240_L64_x8":
        base = 500 if seed is None else seed
        pairs = []
        for i in range(8):
            left, right, gt, edge = slanted_planes(320, 240, 64, base + i)
            pairs.append(dict(left=left, right=right, gt=gt, edge=edge, width=320, height=240,
                              channels=1, num_labels=64, jitter=jitter((64, 240, 320), base + 100 + i)))
        w = _base(name=name, pairs=pairs, levels=1, iters=8, tau=2.5, temperature=0.5,
                  checkpoint_every=2)
    else:
        raise KeyError(f"unknown workload {name!r}; known: {WORKLOADS}")
    w.update(overrides)
    return w
