#!/usr/bin/env python3
"""Benchmark of the stereo hot path on one MI355X.

One step = the whole path for one synthetic aerial pair at 2.7K:
  2704x1520 RGB u8 pair (resident in HBM) -> 4x block-mean downsampling fused
  with the truncated absolute-difference cost volume [64][380][676] ->
  5-level pyramid, 10 checkerboard half-sweeps per level, argmin readout ->
  joint bilateral upsampling to 2704x1520 (sigma_s 8 px, sigma_r 12).
The timed steps replay one HIP graph of that launch sequence.

Prints ONE JSON line.  `value` is BP updates (pixel*label*iteration) per
second of whole-step time; the line also carries pairs/s, the BP-only rate,
the roofline of the dominant kernel (the half-sweep, measured with HIP events
on its launch stream) and the FP64 CPU oracle's rate on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BP updates/s (pixel·label·iter), pairs/s at 676x380x64; HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = {"f32": 18.0, "f16": 10.0, "bf16": 10.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--msg-dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def level_dims(w, h, n):
    out = []
    for _ in range(n):
        out.append((w, h))
        w, h = (w + 1) // 2, (h + 1) // 2
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1902_09733_amd as bp
    from paper_1902_09733_amd import _abi
    from synth import workload

    wl = workload("aerial2704x1520_s4_L64")
    W0, H0, S, L = wl["width"], wl["height"], wl["downsample"], wl["num_labels"]
    levels, K = wl["levels"], wl["iters"]
    w, h = W0 // S, H0 // S
    dims = level_dims(w, h, levels)
    updates = float(sum(a * b for a, b in dims) * L * K)

    dev = torch.device("cuda:0")
    left = torch.from_numpy(wl["left"]).to(dev)
    right = torch.from_numpy(wl["right"]).to(dev)
    cost = torch.empty((L, h, w), dtype=torch.float32, device=dev)
    disp = torch.empty((h, w), dtype=torch.int32, device=dev)
    up = torch.empty((H0, W0), dtype=torch.float32, device=dev)
    params = bp.BPParams(levels=levels, iters=K, lam=wl["lam"], tau=wl["tau"], msg_dtype=args.msg_dtype)
    ws = bp.Workspace()
    outs = [{"disp": disp, "soft": None, "msgs": None}]

    def step():
        bp.cost_volume(left, right, L, wl["data_trunc"], downsample=S, out=cost)
        bp.run(cost, params, workspace=ws, outputs=outs)
        bp.upsample(disp, left, wl["sigma_s"], wl["sigma_r"], -1, out=up)

    step()
    torch.cuda.synchronize()
    replay = step
    if not args.no_graph:
        stream = torch.cuda.Stream()
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            step()
        torch.cuda.current_stream().wait_stream(stream)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        replay = graph.replay
    for _ in range(args.warmup):
        replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        replay()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed * 1e3 / args.steps

    # BP-only time (events around bp_run on the current stream).
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        bp.run(cost, params, workspace=ws, outputs=outs)
    e1.record()
    torch.cuda.synchronize()
    bp_ms = e0.elapsed_time(e1) / reps

    # Dominant kernel: the half-sweep, timed per launch with HIP events
    # recorded on the stream it is launched on.
    import ctypes
    lib = _abi.lib()
    probs = (_abi.BpProblem * 1)()
    probs[0].width, probs[0].height, probs[0].num_labels = w, h, L
    probs[0].cost = cost.data_ptr()
    probs[0].disparity = disp.data_ptr()
    cp = params.c()
    nbytes = lib.bp_workspace_size(probs, 1, ctypes.byref(cp))
    wsb = ws.get(nbytes, dev)
    recs = (_abi.BpLaunchRecord * 256)()
    nrec = ctypes.c_int32(0)
    stream_h = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    per = {}
    for _ in range(5):
        st = lib.bp_run_profiled(probs, 1, ctypes.byref(cp), ctypes.c_void_p(wsb.data_ptr()), nbytes, stream_h,
                                 recs, 256, ctypes.byref(nrec))
        _abi.check("bp_run_profiled", st)
        for i in range(nrec.value):
            r = recs[i]
            if r.readout_fused:
                continue       # a different kernel instance (it also writes labels)
            per.setdefault("ms", []).append(r.ms)
            # Algorithmic bytes: the active half of the pixels reads the cost
            # (4 B) and 4 incoming messages and writes 4 outgoing ones.
            per.setdefault("bytes", []).append(r.units * (4.0 + 8.0 * r.msg_bytes) / 2.0)
            per.setdefault("lvl0", []).append(r.level == 0)
    ms = np.array(per["ms"])
    byt = np.array(per["bytes"])
    lvl0 = np.array(per["lvl0"])
    avg_ms = float(ms.mean())
    achieved = float(byt.mean() / (avg_ms * 1e-3) / 1e9)
    lvl0_gbs = float(byt[lvl0].mean() / (ms[lvl0].mean() * 1e-3) / 1e9)

    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
        "kernel": "k_iter (checkerboard half-sweep), all levels",
        "avg_launch_us": round(avg_ms * 1e3, 2), "launches": int(len(ms)) // 5,
        "level0_GBps": round(lvl0_gbs, 1), "level0_avg_launch_us": round(float(ms[lvl0].mean()) * 1e3, 2),
        "bytes_per_update": BYTES_PER_UPDATE[args.msg_dtype],
    }

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, updates, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": round(updates / (ms_step * 1e-3), 1),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.msg_dtype == "f32" else f"f32 arithmetic, {args.msg_dtype} messages",
        "data": "synthetic",
        "config": {
            "workload": "aerial2704x1520_s4_L64",
            "pair": f"{W0}x{H0} RGB u8, downsampled {S}x to {w}x{h}",
            "labels": L, "levels": levels, "iters_per_level": K, "lambda": wl["lam"], "tau": wl["tau"],
            "data_trunc": wl["data_trunc"], "jbu_sigma_s": wl["sigma_s"], "jbu_sigma_r": wl["sigma_r"],
            "graph": not args.no_graph,
        },
        "pairs_per_s": round(1e3 / ms_step, 2),
        "updates_per_step": updates,
        "bp_only_ms": round(bp_ms, 4),
        "bp_only_updates_per_s": round(updates / (bp_ms * 1e-3), 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def cpu_baseline(wl, updates, budget_s):
    """The FP64 oracle (as it stands) on the host cores: cost + 5-level BP of
    the same pair, repeated for about `budget_s` seconds."""
    import oracle
    S, L = wl["downsample"], wl["num_labels"]
    l4 = oracle.downsample(wl["left"], S)
    r4 = oracle.downsample(wl["right"], S)
    reps, t0 = 0, time.perf_counter()
    while True:
        c = oracle.cost_volume(l4, r4, L, wl["data_trunc"])
        oracle.run(c, wl["levels"], wl["iters"], wl["lam"], wl["tau"])
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 50:
            break
    return {
        "value": round(reps * updates / el, 1), "unit": "updates/s", "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": f"{reps} x (downsampled-pair cost volume + 5-level BP, {updates/1e6:.2f} M updates) of the "
                  f"benchmarked pair, {el:.1f} s",
    }


if __name__ == "__main__":
    main()
