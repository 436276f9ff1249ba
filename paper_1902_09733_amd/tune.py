"""Launch-shape autotuner for the half-sweep kernels.

For each problem shape (width, height, labels, message format, levels,
half-sweeps per level) it times every candidate (first pixel-major level x
kernel variant) with bp_run_profiled, which records HIP events on the launch
stream around the half-sweep launches of each level, and writes the fastest
to a text table:

    # width height labels fmt levels pm_from variant us
    676 380 64 0 5 0 0 655.2

libbpstereo reads the table named by the environment variable BP_TUNE_TABLE
once, at its first bp_run / bp_workspace_size call, and uses the entry with
the same label count, format and level count whose pixel count is nearest
(in log scale) whenever bp_params.pm_from == -1 and bp_params.variant == 0.
Every candidate computes the same result; only speed differs.

Usage:  python -m paper_1902_09733_amd.tune --out tune_table.txt 676x380x64 1352x760x128 ...
"""
from __future__ import annotations

import argparse
import ctypes
import math

import numpy as np
import torch

from . import _abi, stereo


def time_candidate(cost, params: stereo.BPParams, reps: int = 3) -> float:
    lib = _abi.lib()
    L, H, W = cost.shape
    probs = (_abi.BpProblem * 1)()
    probs[0].width, probs[0].height, probs[0].num_labels = W, H, L
    probs[0].cost = cost.data_ptr()
    cp = params.c()
    nb = lib.bp_workspace_size(probs, 1, ctypes.byref(cp))
    if nb == 0:
        raise ValueError("rejected")
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=cost.device)
    wp = ws.data_ptr() + ((-ws.data_ptr()) % 256)
    recs = (_abi.BpLaunchRecord * 1024)()
    n = ctypes.c_int32()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    totals = []
    for r in range(reps + 1):
        st = lib.bp_run_profiled(probs, 1, ctypes.byref(cp), ctypes.c_void_p(wp), nb, stream, 1, recs, 1024,
                                 ctypes.byref(n))
        _abi.check("bp_run_profiled", st)
        if r:
            totals.append(sum(recs[i].ms for i in range(n.value)))
    return float(np.median(totals)) * 1e3


def candidates(L: int, levels: int):
    """(first pixel-major level, variant) pairs; variant 0 is the library's
    own kernel choice (fused pairs of half-sweeps on pixel-major levels)."""
    lib = _abi.lib()
    nv = max(lib.bp_variant_count(L), 2)
    for pm_from in range(levels + 1):
        for variant in range(0, nv + 1):
            yield pm_from, variant


def table_lines(shapes, fmt: str = "f32", levels: int = 5, iters: int = 10, device=None):
    """Tune every (W, H, L) shape; returns the table's lines (header first)
    and the picks as (W, H, L, levels, pm_from, variant, us)."""
    lines = ["# width height labels fmt levels pm_from variant us"]
    picks = []
    for (W, H, L) in shapes:
        lv = max(1, min(levels, int(math.log2(max(2, min(W, H))))))
        best, _ = tune_shape(W, H, L, fmt, lv, iters, device)
        if best is None:
            continue
        lines.append(f"{W} {H} {L} {stereo.MSG_DTYPES[fmt]} {lv} {best[0]} {best[1]} {best[2]:.1f}")
        picks.append((W, H, L, lv, best[0], best[1], round(best[2], 1)))
    return lines, picks


def tune_shape(W: int, H: int, L: int, fmt: str = "f32", levels: int = 5, iters: int = 10, device=None):
    device = device or torch.device("cuda:0")
    rng = np.random.default_rng(0)
    cost = torch.from_numpy(rng.integers(0, 21, size=(L, H, W)).astype(np.float32)).to(device)
    best = None
    results = []
    for pm_from, variant in candidates(L, levels):
        p = stereo.BPParams(levels=levels, iters=iters, lam=10.0, tau=2.0, msg_dtype=fmt, pm_from=pm_from,
                            variant=variant)
        try:
            us = time_candidate(cost, p)
        except Exception:
            continue
        results.append((pm_from, variant, us))
        if best is None or us < best[2]:
            best = (pm_from, variant, us)
    return best, results


def parse_shape(s: str):
    parts = [int(v) for v in s.lower().split("x")]
    if len(parts) != 3:
        raise argparse.ArgumentTypeError("shape must be WIDTHxHEIGHTxLABELS")
    return parts


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("shapes", nargs="+", type=parse_shape)
    ap.add_argument("--out", required=True)
    ap.add_argument("--fmt", default="f32", choices=list(stereo.MSG_DTYPES))
    ap.add_argument("--levels", type=int, default=5)
    ap.add_argument("--iters", type=int, default=10)
    a = ap.parse_args()
    lines, _ = table_lines(a.shapes, a.fmt, a.levels, a.iters)
    print("\n".join(lines[1:]), flush=True)
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
