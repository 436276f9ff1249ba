#!/usr/bin/env python3
"""Benchmark of the stereo hot path on one MI355X.

One step = the whole path for one synthetic aerial pair at 2.7K:
  2704x1520 RGB u8 pair (resident in HBM) -> 4x block-mean downsampling ->
  truncated absolute-difference data term for 64 labels at 676x380, written
  by bp_run straight into the finest level's colour-split layout (with
  --volume: bp_cost_volume's planar [64][380][676] volume, then bp_run) ->
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--msg-dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--volume", action="store_true",
                    help="materialise the planar cost volume with bp_cost_volume inside the step")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--form", default="pair", choices=["pair", "batch", "precision", "adjoint", "points", "undistort", "ceiling",
                                                  "features", "icp", "counters"],
                    help="pair: the benchmarked single-pair path (default); batch, precision, adjoint "
                         "measure the other forms; points the JBU with fused triangulation; counters "
                         "runs the pair path eagerly plus a plain copy of known size, for rocprofv3 "
                         "--pmc passes")
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
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if args.form != "pair":
        print(json.dumps(run_form(args.form, args)))
        return
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

    pair = bp.Pair(left, right, L, wl["data_trunc"], downsample=S)
    # The planar volume for the BP-only and per-level timings below.
    bp.cost_volume(left, right, L, wl["data_trunc"], downsample=S, out=cost)

    def step():
        if args.volume:
            bp.cost_volume(left, right, L, wl["data_trunc"], downsample=S, out=cost)
            bp.run(cost, params, workspace=ws, outputs=outs)
        else:
            bp.run(pair, params, workspace=ws, outputs=outs)
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

    # bp_run alone as the step runs it (data term, pyramid, BP, readout;
    # events around it on the current stream).
    src = cost if args.volume else pair
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        bp.run(src, params, workspace=ws, outputs=outs)
    e1.record()
    torch.cuda.synchronize()
    bp_ms = e0.elapsed_time(e1) / reps
    # The same bp_run captured once in a HIP graph and replayed (how the step
    # runs it): launch gaps between its ~60 kernels shrink.
    g_bp = _graph(lambda: bp.run(src, params, workspace=ws, outputs=outs))
    g_bp.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        g_bp.replay()
    e1.record()
    torch.cuda.synchronize()
    bp_graph_ms = e0.elapsed_time(e1) / reps

    # Dominant kernel: the level-0 half-sweep (k_iter_pm), timed with a HIP
    # event pair recorded on its launch stream around the level's K
    # back-to-back launches (per-level records keep the events' own cost out).
    import ctypes
    lib = _abi.lib()
    probs = bp.stereo._problems([src], [disp], [None], [None])
    cp = params.c()
    nbytes = lib.bp_workspace_size(probs, 1, ctypes.byref(cp))
    wsb = ws.get(nbytes, dev)
    recs = (_abi.BpLaunchRecord * 64)()
    nrec = ctypes.c_int32(0)
    stream_h = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    lv_ms, lv_bytes, lv_units, lv_n = {}, {}, {}, {}
    for _ in range(6):
        st = lib.bp_run_profiled(probs, 1, ctypes.byref(cp), ctypes.c_void_p(wsb.data_ptr()), nbytes, stream_h, 1,
                                 recs, 64, ctypes.byref(nrec))
        _abi.check("bp_run_profiled", st)
        for i in range(nrec.value):
            r = recs[i]
            # Algorithmic bytes of the level's launches as the library reports
            # them: a single half-sweep's active half reads its cost and four
            # incoming rows and writes four outgoing ones (18 B per pixel and
            # label in FP32); a fused pair reads both colours' costs (4 B per
            # pixel and label; 2 B or 1 B where the finest level keeps its
            # integer costs in FP16 or bytes) and colour 0's rows and writes
            # colour 0's rows (10, 9 or 8.5 B per pixel, label and half-sweep
            # in FP32), colour 1's rows also at the level's end.
            lv_ms.setdefault(r.level, []).append(r.ms / r.launches)
            lv_bytes[r.level] = r.bytes / r.launches
            lv_units[r.level] = r.units / r.launches
            lv_n[r.level] = r.launches
    per_level = {l: float(np.median(v[1:])) for l, v in lv_ms.items()}     # first run is a warm-up
    l0_ms = per_level[0]
    achieved = lv_bytes[0] / (l0_ms * 1e-3) / 1e9
    all_ms = sum(per_level[l] * lv_n[l] for l in per_level)
    all_bytes = sum(lv_bytes[l] * lv_n[l] for l in per_level)
    fused = lv_units[0] > w * h * L
    # The same updates at the single-half-sweep schedule's 18 B (FP32): what a
    # one-half-sweep kernel would have to stream to match this time.
    equiv = lv_units[0] * (4.0 + 8.0 * (4 if args.msg_dtype == "f32" else 2)) / 2.0 / (l0_ms * 1e-3) / 1e9

    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": stored_traffic("k_iter_pm2") if fused and args.msg_dtype == "f32" else None,
        "kernel": (f"k_iter_pm2 level-0 fused pair of checkerboard half-sweeps ({w}x{h}x{L}, {args.msg_dtype} "
                   "messages)") if fused else
                  f"k_iter_pm level-0 checkerboard half-sweep ({w}x{h}x{L}, {args.msg_dtype} messages)",
        "avg_launch_us": round(l0_ms * 1e3, 2), "launches_per_step": lv_n[0],
        "half_sweeps_per_launch": round(lv_units[0] / (w * h * L)),
        "bytes_per_launch": lv_bytes[0], "bytes_per_update": lv_bytes[0] / lv_units[0],
        "single_half_sweep_equivalent_GBps": round(equiv, 1),
        "per_level_avg_launch_us": {str(l): round(per_level[l] * 1e3, 2) for l in sorted(per_level)},
        "all_levels_GBps": round(all_bytes / (all_ms * 1e-3) / 1e9, 1),
    }

    cpu = cpu1 = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, updates, args.cpu_seconds)
        # The same oracle on one core: one repetition (about 10 s).
        cpu1 = cpu_baseline(wl, updates, 0.0, threads=1)

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
            "cost_source": "planar volume (bp_cost_volume)" if args.volume else "pair, fused into bp_run",
        },
        "pairs_per_s": round(1e3 / ms_step, 2),
        "updates_per_step": updates,
        "bp_run_ms": round(bp_ms, 4),
        "bp_run_updates_per_s": round(updates / (bp_ms * 1e-3), 1),
        "bp_run_graph_ms": round(bp_graph_ms, 4),
        "bp_run_graph_updates_per_s": round(updates / (bp_graph_ms * 1e-3), 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_baseline_1core": cpu1,
    }
    print(json.dumps(out))


def cpu_baseline(wl, updates, budget_s, threads=0):
    """The FP64 oracle (as it stands) on the host cores (all of them, or
    `threads`): the benchmarked step's three stages on the same pair --
    downsample + cost volume, 5-level BP, joint bilateral upsampling to the
    full frame -- repeated for about `budget_s` seconds (at least once); the
    median time of each stage over the repetitions, and updates/s over the
    whole step as the GPU's value counts them."""
    import statistics

    import oracle
    S, L = wl["downsample"], wl["num_labels"]
    n = threads or oracle.max_threads()
    times = {"cost": [], "bp": [], "jbu": []}
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        l4 = oracle.downsample(wl["left"], S)
        r4 = oracle.downsample(wl["right"], S)
        c = oracle.cost_volume(l4, r4, L, wl["data_trunc"])
        t1 = time.perf_counter()
        o = oracle.run(c, wl["levels"], wl["iters"], wl["lam"], wl["tau"], nthreads=n)
        t2 = time.perf_counter()
        oracle.upsample(o["disp"], wl["left"], wl["sigma_s"], wl["sigma_r"], nthreads=n)
        t3 = time.perf_counter()
        times["cost"].append(t1 - t0)
        times["bp"].append(t2 - t1)
        times["jbu"].append(t3 - t2)
        if time.perf_counter() - t_start >= budget_s or len(times["bp"]) >= 50:
            break
    med = {k: statistics.median(v) for k, v in times.items()}
    step = sum(med.values())
    reps = len(times["bp"])
    return {
        "value": round(updates / step, 1), "unit": "updates/s", "cores": n,
        "kind": "oracle",
        "sample": f"{reps} x the benchmarked pair's step (downsample + cost volume, 5-level BP of "
                  f"{updates/1e6:.2f} M updates, JBU to {wl['width']}x{wl['height']}), median per stage",
        "stage_s": {k: round(v, 4) for k, v in med.items()},
        "pairs_per_s": round(1.0 / step, 3),
        "bp_updates_per_s": round(updates / med["bp"], 1),
        "build": oracle.BUILD_FLAGS,
    }


# ---------------------------------------------------------------------------
# Forms: batched, 16-bit messages, differentiation (python bench.py --form ...)
# ---------------------------------------------------------------------------

def _graph(fn):
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def level_units(w, h, L, levels, K):
    u = 0
    for _ in range(levels):
        u += w * h
        w, h = (w + 1) // 2, (h + 1) // 2
    return u * L * K


def form_batch(args):
    """48 pairs, 320x180 .. 1352x760, labels in {32, 64, 96, 128}, 5 levels x 8
    half-sweeps.  Plain form: one bp_run per pair, FP32, eager launches (and
    the same replayed as a graph).  Batched form: one bp_run over all 48
    pairs, replayed as a HIP graph, in FP32 and with FP16 message storage.
    Every problem comes from its pair (bp_run computes the data term), so a
    step is data term + pyramid + BP + readout for all 48 pairs."""
    import torch

    import paper_1902_09733_amd as bp
    from synth import workload
    dev = torch.device("cuda:0")
    wl = workload("batch48_mixed")
    pairs = wl["pairs"]
    lefts = [torch.from_numpy(p["left"]).to(dev) for p in pairs]
    rights = [torch.from_numpy(p["right"]).to(dev) for p in pairs]
    srcs = [bp.Pair(l, r, p["num_labels"], wl["data_trunc"]) for l, r, p in zip(lefts, rights, pairs)]
    updates = float(sum(level_units(p["width"], p["height"], p["num_labels"], wl["levels"], wl["iters"]) for p in pairs))

    def make_outs():
        return [{"disp": torch.empty((p["height"], p["width"]), dtype=torch.int32, device=dev), "soft": None,
                 "msgs": None} for p in pairs]

    res = {}
    plain_outs = make_outs()
    p32 = bp.BPParams(levels=wl["levels"], iters=wl["iters"], lam=wl["lam"], tau=wl["tau"])
    ws_plain = bp.Workspace()

    def plain():
        for c, o in zip(srcs, plain_outs):
            bp.run(c, p32, workspace=ws_plain, outputs=[o])
    t_plain = _time(plain, 3)
    res["plain_f32_pairs_per_s"] = round(48 / t_plain, 2)
    t_plain_g = _time(_graph(plain).replay, 3)
    res["plain_f32_graph_pairs_per_s"] = round(48 / t_plain_g, 2)
    disp_plain = [o["disp"].clone() for o in plain_outs]

    for fmt in ("f32", "f16"):
        outs = make_outs()
        pp = bp.BPParams(levels=wl["levels"], iters=wl["iters"], lam=wl["lam"], tau=wl["tau"], msg_dtype=fmt)
        ws = bp.Workspace()

        def batched():
            bp.run(srcs, pp, workspace=ws, outputs=outs)
        batched()
        torch.cuda.synchronize()
        g = _graph(batched)
        t = _time(g.replay, 5)
        res[f"batched_{fmt}_pairs_per_s"] = round(48 / t, 2)
        res[f"batched_{fmt}_updates_per_s"] = round(updates / t, 1)
        bad = sum(int((torch.abs(o["disp"] - d) > 1).sum()) for o, d in zip(outs, disp_plain))
        npx = sum(int(d.numel()) for d in disp_plain)
        res[f"batched_{fmt}_bad_pixel_vs_plain_f32"] = bad / npx
    res["speedup_batched_f16_vs_plain_f32"] = round(res["batched_f16_pairs_per_s"] / res["plain_f32_pairs_per_s"], 3)
    res["speedup_batched_f32_vs_plain_f32"] = round(res["batched_f32_pairs_per_s"] / res["plain_f32_pairs_per_s"], 3)

    # The autotuner over the batch's shapes: for each label count the
    # smallest, median and largest pair, both storage formats; the table is
    # loaded into the library and the batched form timed again with it.
    import tempfile

    from paper_1902_09733_amd import _abi, tune
    by_L = {}
    for p in pairs:
        by_L.setdefault(p["num_labels"], []).append((p["width"] * p["height"], p["width"], p["height"]))
    reps = []
    for L in sorted(by_L):
        sizes = sorted(by_L[L])
        for q in sorted({0, len(sizes) // 2, len(sizes) - 1}):
            reps.append((sizes[q][1], sizes[q][2], L))
    lines, picks = ["# width height labels fmt levels pm_from variant us"], {}
    for fmt in ("f32", "f16"):
        ln, pk = tune.table_lines(reps, fmt, wl["levels"], wl["iters"], dev)
        lines += ln[1:]
        picks[fmt] = [list(x) for x in pk]
    with tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False) as fh:
        fh.write("\n".join(lines) + "\n")
        table = fh.name
    lib = _abi.lib()
    _abi.check("bp_load_tune_table", lib.bp_load_tune_table(table.encode()))
    try:
        for fmt in ("f32", "f16"):
            outs = make_outs()
            pp = bp.BPParams(levels=wl["levels"], iters=wl["iters"], lam=wl["lam"], tau=wl["tau"], msg_dtype=fmt)
            ws = bp.Workspace()

            def tuned():
                bp.run(srcs, pp, workspace=ws, outputs=outs)
            tuned()
            torch.cuda.synchronize()
            t = _time(_graph(tuned).replay, 5)
            res[f"tuned_batched_{fmt}_pairs_per_s"] = round(48 / t, 2)
    finally:
        lib.bp_load_tune_table(None)
        os.unlink(table)
    res["tune_shapes"] = [list(r) for r in reps]
    res["tune_picks"] = picks   # (W, H, L, levels, pm_from, variant (0 = fused pairs), us)
    return {"form": "batched", "workload": "batch48_mixed", "updates_per_batch": updates, **res}


def form_precision(args):
    """1352x760 RGB pair, 128 labels, 6 levels x 12 half-sweeps, data term from
    the pair inside bp_run: FP32 / FP16 / BF16 message storage, times and
    deviation from the FP32 GPU result, on an
    integer-valued parameter set (16-bit storage is exact there) and a
    real-valued one (unrounded channel mean, lambda 7.3, tau 2.6).  The
    comparison with the FP64 oracle is made by the GPU test suite."""
    import torch

    import paper_1902_09733_amd as bp
    from synth import workload
    dev = torch.device("cuda:0")
    wl = workload("aerial1352x760_L128")
    L, levels, K = wl["num_labels"], wl["levels"], wl["iters"]
    left = torch.from_numpy(wl["left"]).to(dev)
    right = torch.from_numpy(wl["right"]).to(dev)
    units = level_units(1352, 760, L, levels, K)
    out = {"form": "precision", "workload": "aerial1352x760_L128", "updates_per_pair": units}
    for pset, rgb_mode, lam, tau in (("int", 0, 10.0, 2.0), ("real", 1, 7.3, 2.6)):
        # The pair route: bp_run computes the data term itself (the values
        # bp_cost_volume gives) straight into its layout.
        pair = bp.Pair(left, right, L, 20.0, rgb_mode=rgb_mode)
        ref = None
        for fmt in ("f32", "f16", "bf16"):
            p = bp.BPParams(levels=levels, iters=K, lam=lam, tau=tau, msg_dtype=fmt)
            r = bp.run(pair, p, want_msgs=True)
            ws = bp.Workspace()
            outs = [{"disp": torch.empty_like(r["disp"]), "soft": None, "msgs": None}]
            t = _time(lambda: bp.run(pair, p, workspace=ws, outputs=outs), 10)
            rec = {"bp_ms": round(t * 1e3, 3), "updates_per_s": round(units / t, 1)}
            if ref is None:
                ref = r
            else:
                rec["bad_pixel_vs_gpu_f32"] = float((torch.abs(r["disp"] - ref["disp"]) > 1).float().mean())
                d = ((r["msgs"] - ref["msgs"]).abs() / (lam * tau)).flatten()
                rec["max_msg_diff_vs_gpu_f32_over_lambda_tau"] = float(d.max())
                # Where the maximum comes from: a near-tie of the message's
                # minimiser resolved differently moves whole messages, so the
                # distribution matters more than its maximum.
                k = max(1, int(d.numel() * 1e-3))
                rec["msg_diff_p99_9_over_lambda_tau"] = float(torch.topk(d, k).values[-1])
                rec["msg_entries_off_by_over_1pct_lambda_tau"] = float((d > 1e-2).float().mean())
                rec["msg_entries_off_by_over_half_lambda_tau"] = float((d > 0.5).float().mean())
            out[f"{pset}_{fmt}"] = rec
        del ref
    return out


def form_adjoint(args):
    """8 x 320x240 grey pairs, 64 labels, 8 half-sweeps, soft-argmin (T 0.5),
    checkpoints every 2: forward (with checkpoints) and backward times."""
    import torch

    import paper_1902_09733_amd as bp
    from synth import workload
    from paper_1902_09733_amd import soft_argmin_bp
    dev = torch.device("cuda:0")
    wl = workload("planes320x240_L64_x8")
    vols = [bp.cost_volume(torch.from_numpy(p["left"]).to(dev), torch.from_numpy(p["right"]).to(dev), 64, 20.0)
            + torch.from_numpy(p["jitter"].astype(np.float32)).to(dev) for p in wl["pairs"]]
    ct = torch.stack(vols).detach().requires_grad_(True)
    lt = torch.tensor(10.0, device=dev, requires_grad=True)
    tt = torch.tensor(wl["tau"], device=dev, requires_grad=True)
    G = torch.randn(8, 240, 320, device=dev)

    def fwd():
        return soft_argmin_bp(ct, lt, tt, iters=wl["iters"], temperature=wl["temperature"],
                              checkpoint_every=wl["checkpoint_every"])

    def fwd_bwd():
        ct.grad = None
        (fwd() * G).sum().backward()
    t_f = _time(lambda: fwd(), 5)
    t_fb = _time(fwd_bwd, 5)
    units = 8 * 320 * 240 * 64 * wl["iters"]
    return {"form": "differentiation", "workload": "planes320x240_L64_x8", "forward_ms": round(t_f * 1e3, 3),
            "forward_backward_ms": round(t_fb * 1e3, 3), "backward_ms": round((t_fb - t_f) * 1e3, 3),
            "forward_updates_per_s": round(units / t_f, 1)}


COPY_BYTES = 256 << 20
# Counter-measured HBM traffic of the dominant level-0 kernel, per kernel:
# the committed file and the sources whose digest it was taken with.
TRAFFIC = {
    "k_iter_pm2": ("traffic_k_iter_pm2_aerial676x380_L64_f32.txt",
                   ["paper_1902_09733_amd/csrc/bp_iter_pm2_impl.h", "paper_1902_09733_amd/csrc/bp_iter_pm2_f32.hip",
                    "paper_1902_09733_amd/csrc/bp_pm_core.h", "paper_1902_09733_amd/csrc/bp_device.h",
                    "paper_1902_09733_amd/csrc/bp_internal.h"]),
}


def sources_digest(kernel="k_iter_pm2"):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC[kernel][1]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(kernel="k_iter_pm2"):
    """HBM bytes per level-0 launch of `kernel` from the committed counter
    passes (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter's reading
    for a plain copy of known size), or None when the kernel sources changed
    since the counters were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", TRAFFIC[kernel][0])) as fh:
            kv = dict(line.split(None, 1) for line in fh if line.strip() and not line.startswith("#"))
    except OSError:
        return None
    if kv.get("sources_sha256", "").strip() != sources_digest(kernel):
        return None
    return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])


def form_points(args):
    """JBU of the benchmarked pair's disparity to 2704x1520, alone and with
    the fused Eq. 3 triangulation (float32 [1520][2704][3], 49.3 MB), timed
    with HIP events on the current stream."""
    import torch

    import paper_1902_09733_amd as bp
    from synth import workload
    wl = workload("aerial2704x1520_s4_L64")
    dev = torch.device("cuda:0")
    left = torch.from_numpy(wl["left"]).to(dev)
    right = torch.from_numpy(wl["right"]).to(dev)
    S, L = wl["downsample"], wl["num_labels"]
    params = bp.BPParams(levels=wl["levels"], iters=wl["iters"], lam=wl["lam"], tau=wl["tau"])
    disp = bp.run(bp.Pair(left, right, L, wl["data_trunc"], downsample=S), params)["disp"]
    W0, H0 = wl["width"], wl["height"]
    cam = bp.Camera(baseline=0.5, focal=2.77e-3, du=1.55e-6, dv=1.55e-6, u0=W0 / 2.0, v0=H0 / 2.0)
    up = torch.empty((H0, W0), dtype=torch.float32, device=dev)
    pts = torch.empty((H0, W0, 3), dtype=torch.float32, device=dev)

    def ev_time(fn, reps=20):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    t_jbu = ev_time(lambda: bp.upsample(disp, left, wl["sigma_s"], wl["sigma_r"], -1, out=up))
    t_pts = ev_time(lambda: bp.upsample_points(disp, left, cam, wl["sigma_s"], wl["sigma_r"], -1, out=(up, pts)))
    return {"form": "points", "workload": "aerial2704x1520_s4_L64", "jbu_ms": round(t_jbu, 4),
            "jbu_points_ms": round(t_pts, 4), "points_bytes": int(pts.numel() * 4),
            "epilogue_us": round((t_pts - t_jbu) * 1e3, 2)}


def form_undistort(args):
    """Radial-only undistortion of both 2704x1520 RGB frames of the benchmarked
    pair (HIP events on the current stream; 2 x 12.3 MB read, 2 x 12.3 MB written)."""
    import torch

    import paper_1902_09733_amd as bp
    from synth import workload
    wl = workload("aerial2704x1520_s4_L64")
    dev = torch.device("cuda:0")
    left = torch.from_numpy(wl["left"]).to(dev)
    right = torch.from_numpy(wl["right"]).to(dev)
    K = bp.Intrinsics(1600.0, 1600.0, 1351.5, 759.5, -0.12, 0.02, -0.001)
    lo, ro = torch.empty_like(left), torch.empty_like(right)

    def step():
        bp.undistort(left, K, out=lo)
        bp.undistort(right, K, out=ro)
    step()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 50
    e0.record()
    for _ in range(reps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 4 * left.numel()
    return {"form": "undistort", "workload": "aerial2704x1520 RGB pair", "pair_ms": round(ms, 4),
            "per_frame_us": round(ms * 500, 2), "GBps_algorithmic": round(nbytes / (ms * 1e-3) / 1e9, 1)}


def form_features(args):
    """Harris response + 30 x 30 cell corners of the benchmarked pair's left
    frame (grey 2704x1520), then ZSSD matches (11 x 11 patches, +-16 px) of
    those corners in the right frame; HIP events on the current stream."""
    import torch

    import paper_1902_09733_amd as bp
    from synth import workload
    wl = workload("aerial2704x1520_s4_L64")
    dev = torch.device("cuda:0")

    def grey(rgb):
        return ((rgb[..., 0].astype(np.int32) * 77 + rgb[..., 1].astype(np.int32) * 150 +
                 rgb[..., 2].astype(np.int32) * 29) >> 8).astype(np.uint8)
    a = torch.from_numpy(grey(wl["left"])).to(dev)
    b = torch.from_numpy(grey(wl["right"])).to(dev)
    thr = 2 * 10 ** 7

    def ev_time(fn, reps=20):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    out = bp.harris(a, 30, thr)
    t_h = ev_time(lambda: bp.harris(a, 30, thr))
    t_m = ev_time(lambda: bp.zssd_match(a, b, out["raw"], 5, 16))
    found = int((out["x"] >= 0).sum().item())
    return {"form": "features", "workload": "aerial2704x1520 grey pair, 30x30 cells", "harris_ms": round(t_h, 4),
            "zssd_ms": round(t_m, 4), "corners": found, "zssd_shifts_per_corner": 33 * 33, "patch": "11x11"}


def form_icp(args):
    """Point-to-point ICP of a 676x380-point terrain cloud (the size of a cloud
    from the benchmarked pair's disparity) onto a copy moved by a small rigid
    motion (the residual left by the estimated poses) with 2 cm noise, 30
    iterations, correspondences within 1 m; HIP events on the current stream."""
    import torch

    import paper_1902_09733_amd as bp
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(11)
    n = 676 * 380
    xy = rng.uniform(-100.0, 100.0, size=(n, 2))
    z = 8.0 * np.sin(0.05 * xy[:, 0]) * np.cos(0.04 * xy[:, 1]) + 0.002 * xy[:, 0] ** 2
    src = np.column_stack([xy, z])
    a, b, c = 0.002, -0.003, 0.004
    Rx = np.array([[1, 0, 0], [0, np.cos(a), -np.sin(a)], [0, np.sin(a), np.cos(a)]])
    Ry = np.array([[np.cos(b), 0, np.sin(b)], [0, 1, 0], [-np.sin(b), 0, np.cos(b)]])
    Rz = np.array([[np.cos(c), -np.sin(c), 0], [np.sin(c), np.cos(c), 0], [0, 0, 1]])
    R_true, T_true = Rz @ Ry @ Rx, np.array([0.5, -0.4, 0.2])
    dst = src @ R_true.T + T_true + 0.02 * rng.normal(size=src.shape)
    s_t = torch.from_numpy(src.astype(np.float32)).to(dev)
    d_t = torch.from_numpy(dst.astype(np.float32)).to(dev)
    pose = torch.tensor([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], dtype=torch.float64, device=dev)
    ws = bp.Workspace()
    iters = 30
    out = bp.icp(s_t, d_t, pose, iters, 1.0, workspace=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        bp.icp(s_t, d_t, pose, iters, 1.0, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    est = out["pose"].cpu().numpy()
    return {"form": "icp", "workload": f"terrain cloud {n} points onto a moved noisy copy", "iters": iters,
            "icp_ms": round(ms, 3), "per_iteration_us": round(ms * 1e3 / iters, 1),
            "final_rms_m": round(float(out["rms"][-1].item()), 5), "final_pairs": int(out["pairs"][-1].item()),
            "rotation_error": float(np.abs(est[:9].reshape(3, 3) - R_true).max()),
            "translation_error_m": float(np.abs(est[9:] - T_true).max())}


def form_counters(args):
    """The pair path three times without a graph (every dispatch visible to a
    counter pass) with the library's kernel choice, three times with one
    half-sweep per launch (variant 1, the same per-message arithmetic), then
    three plain device-to-device copies of 256 MiB."""
    import torch

    import paper_1902_09733_amd as bp
    from synth import workload
    wl = workload("aerial2704x1520_s4_L64")
    W0, H0, S, L = wl["width"], wl["height"], wl["downsample"], wl["num_labels"]
    dev = torch.device("cuda:0")
    left = torch.from_numpy(wl["left"]).to(dev)
    right = torch.from_numpy(wl["right"]).to(dev)
    params = bp.BPParams(levels=wl["levels"], iters=wl["iters"], lam=wl["lam"], tau=wl["tau"])
    pair = bp.Pair(left, right, L, wl["data_trunc"], downsample=S)
    for _ in range(3):
        bp.run(pair, params)
    single = bp.BPParams(levels=wl["levels"], iters=wl["iters"], lam=wl["lam"], tau=wl["tau"], variant=1)
    for _ in range(3):
        bp.run(pair, single)
    src = torch.empty(COPY_BYTES, dtype=torch.uint8, device=dev).fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"form": "counters", "copy_bytes": COPY_BYTES, "pair_runs": 3, "single_half_sweep_runs": 3, "copies": 3,
            "sources_sha256": {k: sources_digest(k) for k in TRAFFIC}}


def form_ceiling(args):
    """Practical bandwidth ceiling for the level-0 launches' read/write mixes:
    bp_stream_probe moves the same bytes in 16-byte accesses (no BP work),
    timed with HIP events on its stream around 20 back-to-back launches (as
    the BP launches run), median of 5 such batches.  Mixes at the
    benchmarked 676x380x64 level 0: a single half-sweep (reads 164.4 MB,
    writes 131.5 MB), a fused pair (reads both costs and colour 0's rows,
    197.3 MB, writes colour 0's rows, 131.5 MB), the fused pair with the
    finest level's cost in FP16 (reads 164.4 MB, writes 131.5 MB: the same
    volumes as the single half-sweep), and a plain 1:1 copy."""
    import ctypes

    import torch

    from paper_1902_09733_amd import _abi
    lib = _abi.lib()
    nl = 676 * 380 * 64
    mixes = {
        "single_half_sweep": (nl * (4 + 16) // 2, nl * 16 // 2),
        "fused_pair": (nl * (4 + 8), nl * 8),
        "fused_pair_cost16": (nl * (2 + 8), nl * 8),
        "copy_256MiB": (256 << 20, 256 << 20),
    }
    dev = torch.device("cuda:0")
    big = max(max(r, w) for r, w in mixes.values())
    src = torch.ones(big // 4 + 64, dtype=torch.float32, device=dev)
    dst = torch.empty(big // 4 + 64, dtype=torch.float32, device=dev)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = {"form": "ceiling", "peak_GBps": HBM_PEAK_GBS}
    for name, (rb, wb) in mixes.items():
        rb, wb = rb // 16 * 16, wb // 16 * 16

        def once():
            _abi.check("bp_stream_probe", lib.bp_stream_probe(ctypes.c_void_p(src.data_ptr()), rb,
                                                              ctypes.c_void_p(dst.data_ptr()), wb, st))
        for _ in range(3):
            once()
        times = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                once()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 20)
        ms = float(np.median(times))
        out[name] = {"read_bytes": rb, "write_bytes": wb, "us": round(ms * 1e3, 2),
                     "GBps": round((rb + wb) / (ms * 1e-3) / 1e9, 1),
                     "frac_of_peak": round((rb + wb) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def run_form(form, args):
    return {"batch": form_batch, "precision": form_precision, "adjoint": form_adjoint, "points": form_points,
            "undistort": form_undistort, "features": form_features, "icp": form_icp,
            "counters": form_counters, "ceiling": form_ceiling}[form](args)


if __name__ == "__main__":
    main()
