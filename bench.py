#!/usr/bin/env python3
"""Benchmark: iterated 2D Jacobi Box-2D49P sweep on one MI355X.

Workload (the headline configuration): a 7x7 box stencil (radius 3) with 49 weights drawn
uniform[0,1) from seed 1 and normalised to sum 1 (FP32), on a 16384 x 16384 FP32 grid with a zero
Dirichlet halo, interior uniform[0,1), 1000 Jacobi steps.  One benchmark "step" is one full
1000-step run through ``stencil_run`` (the C ABI), with input and output resident in HBM.

Metric: GStencil/s = T * Nx * Ny / (t * 1e9)  (paper Sec. VI-A, Eq. 1), t = pure kernel time
measured with HIP events on the stream the kernels run on.

The JSON line also carries
  roofline      the sweep kernel's achieved FLOP/s against the published FP32 vector peak
                (157.3 TFLOP/s; the vector ALU is the binding roof for this stencil: 97 FLOP and
                8/tb bytes per update), beside the fraction of the non-packed FMA issue rate
                (78.6 TFLOP/s) these kernels can reach, and the HBM traffic measured by rocprofv3
                when the committed counters match the current kernel source;
  cpu_baseline  the CPU oracle (FP32-canonical mode, all host cores) timed on a bounded sample;
  extras        the other workloads (heat 512^2, batched 256 grids, 16-bit storage, surrogate) at a
                glance -- their parity lives in the test suite.
"""
from __future__ import annotations

import argparse
import functools
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402

VALU_FP32_PEAK = 256 * 4 * 16 * 2 * 2.4e9   # 78.6 TFLOP/s: FP32 FMA issued one lane-op per cycle (no packed math)
VALU_FP32_PEAK_PACKED = 157.3e12             # published FP32 vector peak (needs packed FP32, not used here)
HBM_PEAK = 8.0e12


def flop_per_update(taps: int) -> float:
    """FLOP of one cell update with `taps` footprint taps: the centre product, then one fused
    multiply-add (2 FLOP) per other tap -- 9 for the 5-point star, as counted in Sec. VI-E."""
    return 2.0 * taps - 1.0


def gstencil_s(steps: int, rows: int, cols: int, seconds: float) -> float:
    """Cell updates per second in units of 10^9 (Sec. VI-A)."""
    return steps * rows * cols / (seconds * 1e9)


KERNEL_NAMES = {0: "sweep_tiled", 1: "sweep_stream", 2: "sweep_march", 3: "sweep_march", 4: "sweep_march",
                5: "sweep_resident", 6: "sweep_mfma"}
VARIANT_NAMES = {0: "tiled", 1: "stream", 2: "march", 3: "march8", 4: "march1", 5: "resident", 6: "mfma"}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("sweep.hip", "sweep_body.h", "storage.h", "internal.h", "march.hip", "march_body.h", "march_kern.h",
              "march_layout.h", "march_f32_box.hip"):
        with open(os.path.join(ROOT, "paper_2605_07954_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(tb: int, tile, variant: int) -> float | None:
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source with the same blocking; else None."""
    path = os.path.join(ROOT, "profiles", "box49_16384_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if (d.get("kernel_hash") != kernel_source_hash() or d.get("tb") != tb or list(d.get("tile", [])) != list(tile)
            or d.get("variant") != variant):
        return None
    return d.get("hbm_bytes_per_launch")


def time_each(fn, reps: int, stream) -> list:
    """Seconds of each of `reps` back-to-back calls of `fn`, from HIP events recorded on `stream`
    (the stream the library launches on) between the calls; the host does not wait in between."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(reps):
        fn()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    return [ev[k].elapsed_time(ev[k + 1]) / 1e3 for k in range(reps)]


def time_median(fn, reps: int, stream) -> float:
    """Median over `reps` (at least 10) timed calls, in seconds."""
    return float(np.median(time_each(fn, max(reps, 10), stream)))


def cpu_baseline(p) -> dict:
    import oracle
    rows = cols = 1024
    steps = int(os.environ.get("BENCH_CPU_STEPS", "3000"))
    u0 = np.ascontiguousarray(p.u0[:rows, :cols])
    t0 = time.perf_counter()
    oracle.stencil_f32(u0, p.weights, 0.0, steps)
    dt = time.perf_counter() - t0
    return {"value": gstencil_s(steps, rows, cols, dt), "unit": "GStencil/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"box2d49p FP32-canonical oracle on the 1024x1024 top-left crop, {steps} steps ({dt:.1f} s)"}


def cpu_oracle_timings() -> dict:
    """The oracle as written, timed on this host for every configuration (all threads, and one
    thread for the small ones): a reported CPU baseline, never the target."""
    import oracle
    nthreads = oracle.num_threads()

    def timed(fn, *a):
        t0 = time.perf_counter()
        fn(*a)
        return time.perf_counter() - t0

    out = {"threads": nthreads}
    p = wl.heat2d()
    for mode, fn in (("f64", oracle.stencil_f64), ("f32", oracle.stencil_f32)):
        dt = timed(fn, p.u0, p.weights, 0.0, p.steps)
        oracle.set_threads(1)
        dt1 = timed(fn, p.u0, p.weights, 0.0, p.steps)
        oracle.set_threads(nthreads)
        upd = p.steps * p.rows * p.cols
        out[f"heat2d_512_100_{mode}"] = {"s": dt, "gstencil_s": upd / dt / 1e9, "s_1thread": dt1,
                                         "gstencil_s_1thread": upd / dt1 / 1e9}
    p = wl.box49(rows=1024, cols=1024, steps=200)
    for mode, fn in (("f64", oracle.stencil_f64), ("f32", oracle.stencil_f32)):
        dt = timed(fn, p.u0, p.weights, 0.0, p.steps)
        out[f"box49_1024crop_200_{mode}"] = {"s": dt, "gstencil_s": p.steps * p.rows * p.cols / dt / 1e9}
    probs = wl.batch_problems(n_grids=256, steps=200)
    t0 = time.perf_counter()
    for q in probs:
        oracle.stencil_f32(q.u0, q.weights, 0.0, q.steps)
    dt = time.perf_counter() - t0
    upd = sum(q.steps * q.rows * q.cols for q in probs)
    out["batched_256_200_f32"] = {"s": dt, "gstencil_s": upd / dt / 1e9}
    p = wl.star9_precision()
    dt = timed(oracle.stencil_f64, p.u0, p.weights, 0.0, p.steps)
    out["star9_8192_500_f64"] = {"s": dt, "gstencil_s": p.steps * p.rows * p.cols / dt / 1e9}
    bits = oracle.to_bits(p.u0[:2048, :2048], "bf16")
    dt = timed(oracle.stencil_lowp, bits, p.weights, 0.0, 100, "bf16")
    out["star9_2048crop_100_bf16_emulated"] = {"s": dt, "gstencil_s": 100 * 2048 * 2048 / dt / 1e9}
    u0, kappa = wl.varcoef_problem()[:2]
    for mode, fn in (("f64", oracle.varcoef_f64), ("f32", oracle.varcoef_f32)):
        dt = timed(fn, u0, kappa, 0.0, 16)
        out[f"varcoef_1024_16_{mode}"] = {"s": dt, "gstencil_s": 16 * u0.size / dt / 1e9}
    return out


def main_line(args, torch, lib, stream):
    p = wl.box49(rows=args.size, cols=args.size, steps=args.jacobi_steps)
    rows, cols = p.rows, p.cols
    x = torch.from_numpy(p.u0).to("cuda")
    out = torch.empty_like(x)
    # the whole 1000-step run is one captured hipGraph (the autotuner times direct launches)
    plan = lib.stencil_plan(rows, cols, p.radius, p.weights, 0.0, "f32", lib.ST_FLAG_GRAPH)
    t0 = time.perf_counter()
    tune_steps = 24
    ws = torch.empty_like(x)
    if args.tb:
        lib.stencil_set_blocking(plan, 1, *(args.tile or (0, 0)))
        lib.stencil_set_variant(plan, args.variant)
        lib.stencil_set_blocking(plan, args.tb)
        tb, tx, ty = lib.stencil_get_blocking(plan)
    else:
        tb, tx, ty = lib.stencil_autotune(plan, x, out, ws, tune_steps, stream)
    variant = lib.stencil_get_variant(plan)
    tune_s = time.perf_counter() - t0
    T = p.steps
    run = lambda: lib.stencil_run(plan, x, out, T, ws, stream)  # noqa: E731
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    each = time_each(run, args.steps, stream)  # the K timed steps, synchronised before and after
    t = float(sum(each))
    ms = t / args.steps * 1e3
    value = gstencil_s(T * args.steps, rows, cols, t)
    launches = math.ceil(T / tb) * args.steps
    fpu = flop_per_update(49)  # 97: 1 multiply + 48 FMA
    flops = fpu * T * rows * cols * args.steps
    achieved = flops / t
    traffic = measured_traffic(tb, (tx, ty), variant)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_FP32_PEAK_PACKED / 1e12, "unit": "TFLOP/s",
            "frac": achieved / VALU_FP32_PEAK_PACKED, "traffic": traffic,
            "issue_rate_peak": VALU_FP32_PEAK / 1e12, "frac_of_issue_rate": achieved / VALU_FP32_PEAK,
            "ms_per_step_median": float(np.median(each)) * 1e3,
            "ms_per_step_min": min(each) * 1e3, "ms_per_step_max": max(each) * 1e3,
            "kernel": KERNEL_NAMES[variant] + f"<f32, r=3, box{', 8 columns per lane' if variant == 3 else ''}, tb={tb}>",
            "launches": launches,
            "avg_launch_us": t / launches * 1e6,
            "alg_flop_per_launch": fpu * rows * cols * tb, "alg_bytes_per_update": 8.0 / tb,
            "hbm_roof_gstencil": HBM_PEAK / (8.0 / tb) / 1e9,
            "alu_roof_gstencil": VALU_FP32_PEAK / fpu / 1e9,
            "alg_hbm_gbps": 8.0 / tb * T * rows * cols * args.steps / t / 1e9}
    lib.stencil_destroy(plan)
    del x, out, ws
    torch.cuda.empty_cache()
    return p, value, ms, roof, (tb, tx, ty, variant), tune_s


def tune_batch_plans(lib, probs, plans, ins, outs, wss, stream=None) -> list:
    """Blocking of a batch's plans: ``stencil_autotune`` on every grid, so that the per-grid baseline
    runs each grid with its own best single-grid kernel (the batch itself keeps each plan's depth)."""
    return [lib.stencil_autotune(pl, i, o, w, 20, stream) + (lib.stencil_get_variant(pl),)
            for pl, i, o, w in zip(plans, ins, outs, wss)]


def _roofs(flop: float, bytes_per_update: float, gst: float) -> dict:
    hbm = HBM_PEAK / bytes_per_update / 1e9
    alu = VALU_FP32_PEAK / flop / 1e9
    return {"alg_bytes_per_update": bytes_per_update, "hbm_roof_gstencil": hbm, "alu_roof_gstencil": alu,
            "bound": "hbm" if hbm < alu else "alu", "frac_of_roof": gst / min(hbm, alu)}


def extra_heat2d(torch, lib, stream) -> dict:
    """Heat 512^2, 100 steps: L2-resident and launch-bound, so no roofline (the grid never leaves L2)."""
    p = wl.heat2d()
    x = torch.from_numpy(p.u0).to("cuda")
    out = torch.empty_like(x)
    ws = torch.empty_like(x)
    plan = lib.stencil_plan(p.rows, p.cols, 1, p.weights, 0.0, "f32", lib.ST_FLAG_GRAPH)
    tb, _, _ = lib.stencil_autotune(plan, x, out, ws, p.steps, stream)  # the whole run: a few ms
    var = lib.stencil_get_variant(plan)
    seg = lib.stencil_get_march_segment(plan)
    run = lambda: lib.stencil_run(plan, x, out, p.steps, ws, stream)  # noqa: E731
    run()
    t = time_median(run, 20, stream)
    lib.stencil_destroy(plan)
    return {"gstencil_s": gstencil_s(p.steps, p.rows, p.cols, t), "us": t * 1e6, "tb": tb,
            "variant": VARIANT_NAMES[var], "march_seg_min": seg, "launches": math.ceil(p.steps / tb)}


def extra_box49_tb1(torch, lib, stream) -> dict:
    """Box-2D49P 16384^2 x 1000 with one level per pass (8 bytes per update, read and write once):
    the HBM-bound form, against the HBM roof (8 TB/s / 8 B = 1000 GStencil/s) and against the rate a
    device copy reaches.  The best of the marching kernels with four and eight columns per lane."""
    p = wl.box49(rows=16384, cols=16384, steps=1000)
    x = torch.from_numpy(p.u0).to("cuda")
    out = torch.empty_like(x)
    ws = torch.empty_like(x)
    res = {}
    for var in (lib.ST_VARIANT_MARCH8, lib.ST_VARIANT_MARCH):
        plan = lib.stencil_plan(p.rows, p.cols, 3, p.weights, 0.0, "f32", lib.ST_FLAG_GRAPH)
        lib.stencil_set_blocking(plan, 1)
        lib.stencil_set_variant(plan, var)
        run = lambda: lib.stencil_run(plan, x, out, p.steps, ws, stream)  # noqa: E731
        run()
        t = time_median(run, 10, stream)
        lib.stencil_destroy(plan)
        res[VARIANT_NAMES[var]] = gstencil_s(p.steps, p.rows, p.cols, t)
    y = torch.empty_like(x)
    cp = lambda: y.copy_(x)  # noqa: E731
    cp()
    tc = time_median(cp, 10, stream)
    copy_gbs = 2.0 * x.numel() * 4 / tc / 1e9
    best = max(res.values())
    del x, out, ws, y
    torch.cuda.empty_cache()
    return {"gstencil_s": best, "by_variant": res, "alg_bytes_per_update": 8.0,
            "hbm_roof_gstencil": HBM_PEAK / 8.0 / 1e9, "frac_of_hbm_roof": best / (HBM_PEAK / 8.0 / 1e9),
            "alg_hbm_gbps": best * 8.0, "device_copy_gbps": copy_gbs,
            "frac_of_device_copy": best * 8.0 / copy_gbs}


def extra_star9(torch, lib, stream) -> dict:
    """Star-2D9P 8192^2, 500 steps, FP32 / BF16 / FP16 storage (17 FLOP per update)."""
    p = wl.star9_precision(rows=8192, cols=8192, steps=500)
    res = {}
    for st in ("f32", "bf16", "f16"):
        xh = torch.from_numpy(p.u0).to("cuda")
        if st != "f32":
            xh = xh.to(torch.bfloat16 if st == "bf16" else torch.float16).view(torch.int16)
        o = torch.empty_like(xh)
        w2 = torch.empty_like(xh)
        plan = lib.stencil_plan(p.rows, p.cols, 2, p.weights, 0.0, st, 0)
        # 120 sample steps: a whole number of passes at every depth up to 6 and at 8, so that no
        # candidate is timed with a shallower last pass than the real run has
        tb, _, _ = lib.stencil_autotune(plan, xh, o, w2, 120, stream)
        var = lib.stencil_get_variant(plan)
        seg = lib.stencil_get_march_segment(plan)
        run = lambda: lib.stencil_run(plan, xh, o, p.steps, w2, stream)  # noqa: E731
        run()
        t = time_median(run, 10, stream)
        gst = gstencil_s(p.steps, p.rows, p.cols, t)
        res[st] = {"gstencil_s": gst, "ms": t * 1e3, "tb": tb, "variant": VARIANT_NAMES[var], "march_seg_min": seg,
                   **_roofs(flop_per_update(9), 2.0 * xh.element_size() / tb, gst)}
        lib.stencil_destroy(plan)
        del xh, o, w2
    torch.cuda.empty_cache()
    return res


def extra_star9_profile(torch, lib, stream, variant: int = 2, tb: int = 6, storage: str = "f32") -> dict:
    """Star-2D9P 8192^2 with one fixed engine and depth and no tuning, 48 steps: a short run for
    counter profiles of one marching kernel."""
    p = wl.star9_precision(rows=8192, cols=8192, steps=48)
    xh = torch.from_numpy(p.u0).to("cuda")
    if storage != "f32":
        xh = xh.to(torch.bfloat16 if storage == "bf16" else torch.float16).view(torch.int16)
    o = torch.empty_like(xh)
    w2 = torch.empty_like(xh)
    plan = lib.stencil_plan(p.rows, p.cols, 2, p.weights, 0.0, storage, 0)
    lib.stencil_set_blocking(plan, tb)  # (the depth first: the default may be too deep for the variant)
    lib.stencil_set_variant(plan, variant)
    run = lambda: lib.stencil_run(plan, xh, o, p.steps, w2, stream)  # noqa: E731
    run()
    t = time_median(run, 3, stream)
    lib.stencil_destroy(plan)
    return {"storage": storage, "variant": VARIANT_NAMES[variant], "tb": tb,
            "gstencil_s": gstencil_s(p.steps, p.rows, p.cols, t)}


def extra_batched(torch, lib, stream) -> dict:
    """256 grids, one hipGraph launch of the batched kernels vs per-grid launches (each grid autotuned)."""
    probs = wl.batch_problems()
    ins = [torch.from_numpy(q.u0).to("cuda") for q in probs]
    outs = [torch.empty_like(i) for i in ins]
    wss = [torch.empty_like(i) for i in ins]
    plans = [lib.stencil_plan(q.rows, q.cols, q.radius, q.weights, 0.0, "f32", 0) for q in probs]
    tune_batch_plans(lib, probs, plans, ins, outs, wss, stream)
    per_grid = lambda: [lib.stencil_run(pl, i, o, q.steps, w, stream)  # noqa: E731
                        for q, pl, i, o, w in zip(probs, plans, ins, outs, wss)]
    per_grid()
    t_per = time_median(per_grid, 10, stream)
    batch = lib.stencil_batch_create(plans, [q.steps for q in probs], lib.ST_FLAG_GRAPH)
    bws = torch.empty(lib.stencil_batch_workspace_bytes(batch), dtype=torch.uint8, device="cuda")
    caps = lib.stencil_batch_autotune(batch, ins, outs, bws, stream)
    segs = {k: lib.stencil_batch_get_segment(batch, k[0], k[1]) for k in caps}
    runb = lambda: lib.stencil_run_batched(batch, ins, outs, bws, stream)  # noqa: E731
    runb()
    t_b = time_median(runb, 10, stream)
    cells = sum(q.rows * q.cols * q.steps for q in probs)
    lib.stencil_batch_destroy(batch)
    for pl in plans:
        lib.stencil_destroy(pl)
    del ins, outs, wss, bws
    torch.cuda.empty_cache()
    return {"gstencil_s": cells / t_b / 1e9, "ms": t_b * 1e3,
            "classes": {f"{k[0]}{k[1]}": f"{v[0]} x{v[1]}" + (f", {segs[k]}-row segments" if segs[k] else "")
                        for k, v in caps.items()},
            "per_grid_ms": t_per * 1e3,
            "per_grid_gstencil_s": cells / t_per / 1e9, "speedup_vs_per_grid": t_per / t_b}


def extra_batched_profile(torch, lib, stream, config: str = "", timed: bool = False) -> dict:
    """The 256-grid batch with a fixed configuration and no tuning, run 3 times (then timed over 10
    runs if `timed`): a short run for counter profiles and A/B timing.  `config`: comma-separated shape:radius:engine:depth:segment_rows entries,
    e.g. "star:1:march:8:0" (segment_rows 0: the default sizing)."""
    probs = wl.batch_problems()
    ins = [torch.from_numpy(q.u0).to("cuda") for q in probs]
    outs = [torch.empty_like(i) for i in ins]
    plans = [lib.stencil_plan(q.rows, q.cols, q.radius, q.weights, 0.0, "f32", 0) for q in probs]
    batch = lib.stencil_batch_create(plans, [q.steps for q in probs], lib.ST_FLAG_GRAPH)
    for ent in filter(None, config.split(",")):
        shape, r, engine, depth, seg = ent.split(":")
        lib.stencil_batch_set_class(batch, shape, int(r), engine, int(depth))
        lib.stencil_batch_set_segment(batch, shape, int(r), int(seg))
    bws = torch.empty(lib.stencil_batch_workspace_bytes(batch), dtype=torch.uint8, device="cuda")
    runb = lambda: lib.stencil_run_batched(batch, ins, outs, bws, stream)  # noqa: E731
    for _ in range(3):
        runb()
    torch.cuda.synchronize()
    t = time_median(runb, 10, stream) if timed else None
    lib.stencil_batch_destroy(batch)
    for pl in plans:
        lib.stencil_destroy(pl)
    return {"config": config, "updates": sum(q.rows * q.cols * q.steps for q in probs),
            "ms": t * 1e3 if t else None}


def extra_surrogate(torch, lib, stream) -> dict:
    """Surrogate inference on 1024^2 (75,456 FLOP per cell on the MFMA path) vs the fastest plain 16
    varcoef steps (autotuned tile and depth); timing only, the accuracy of a trained network is
    measured by the training driver."""
    u0, kap = wl.varcoef_problem(1024, 1024, seed=0)
    u = torch.from_numpy(u0).to("cuda")
    k = torch.from_numpy(kap).to("cuda")
    o = torch.empty_like(u)
    w = torch.empty_like(u)
    vplan = lib.stencil_plan_varcoef(1024, 1024, 0.0, lib.ST_FLAG_GRAPH)
    vtb, vtx, vty = lib.stencil_autotune_varcoef(vplan, u, k, o, w, 16, stream)  # every tile and depth
    run = lambda: lib.stencil_run_varcoef(vplan, u, k, o, 16, w, stream)  # noqa: E731
    run()
    best = time_median(run, 20, stream)
    m = lib.surrogate_create()
    pd = torch.empty(lib.SG_PARAM_COUNT, dtype=torch.float32, device="cuda")
    lib.surrogate_init(m, pd, None, 0)  # timing only: the weights' values do not matter
    sws = torch.empty(lib.surrogate_workspace_bytes(m, 1, 1024, 1024), dtype=torch.uint8, device="cuda")
    uh = torch.empty((1, 1024, 1024), device="cuda")
    run = lambda: lib.surrogate_infer(m, pd, u, k, uh, 1, 1024, 1024, sws, stream)  # noqa: E731
    run()
    ts = time_median(run, 10, stream)
    lib.surrogate_destroy(m)
    lib.stencil_destroy(vplan)
    return {"plain_16_steps_us": best * 1e6, "plain_blocking": {"tb": vtb, "tile": [vtx, vty]},
            "cnn_infer_us": ts * 1e6, "speedup_vs_plain": best / ts,
            "cnn_tflops": 75456.0 * 1024 * 1024 / ts / 1e12, "cnn_frac_of_bf16_mfma_peak": 75456.0 * 1024 * 1024 / ts / 2.5e15}


def extra_surrogate_trained(torch, lib, stream) -> dict:
    """The surrogate trained on 20k GPU-generated 1024^2 trajectories (about 10 s), then judged on 200
    held-out ones: mean rel-L2 of the trained network and of the identity predictor u_hat = u0
    against 16 plain steps, next to the times of inference, of judged inference (light-cone patch
    judge and whole-field judge) and of the plain 16 steps."""
    from paper_2605_07954_amd.surrogate import Trainer
    tr = Trainer(grid=1024, crop=256, batch=8, K=16, seed=0)
    try:
        t0 = time.perf_counter()
        tr.train(20000, log=None)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        e_tr, e_id = tr.evaluate(tr.params, 200)
        u0, kap = wl.varcoef_problem(1024, 1024, seed=0)
        u = torch.from_numpy(u0).to("cuda")
        k = torch.from_numpy(kap).to("cuda")
        o = torch.empty_like(u)
        w = torch.empty_like(u)
        judge = tr.judge
        vplan = lib.stencil_plan_varcoef(1024, 1024, 0.0, lib.ST_FLAG_GRAPH)
        lib.stencil_autotune_varcoef(vplan, u, k, o, w, 16, stream)
        plain = lambda: lib.stencil_run_varcoef(vplan, u, k, o, 16, w, stream)  # noqa: E731
        plain()
        t_plain = time_median(plain, 20, stream)
        cws = torch.empty(lib.surrogate_checked_ws_bytes(tr.model, 1024, 1024), dtype=torch.uint8, device="cuda")
        sws = torch.empty(lib.surrogate_workspace_bytes(tr.model, 1, 1024, 1024), dtype=torch.uint8, device="cuda")
        uh = torch.empty((1, 1024, 1024), device="cuda")
        inf = lambda: lib.surrogate_infer(tr.model, tr.params, u, k, uh, 1, 1024, 1024, sws, stream)  # noqa: E731
        inf()
        t_inf = time_median(inf, 20, stream)

        def checked(mode):
            t = []
            for _ in range(10):  # each call synchronises to read the judged error: host wall time
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lib.surrogate_infer_checked(tr.model, tr.params, u, k, o, 1024, 1024, judge, 16, 1.0, cws, mode, stream)
                t.append(time.perf_counter() - t0)
            return float(np.median(t))
        t_patch = checked(lib.SG_JUDGE_PATCH)
        t_full = checked(lib.SG_JUDGE_FULL)
        lib.stencil_destroy(vplan)
    finally:
        tr.close()
    return {"train_trajectories": 20000, "train_s": train_s, "heldout": 200,
            "rel_l2_trained_mean": float(e_tr.mean()), "rel_l2_identity_mean": float(e_id.mean()),
            "trained_over_identity": float(e_tr.mean() / e_id.mean()),
            "plain_16_steps_us": t_plain * 1e6, "infer_us": t_inf * 1e6,
            "checked_patch_us_host": t_patch * 1e6, "checked_full_us_host": t_full * 1e6,
            "speedup_infer_vs_plain": t_plain / t_inf}


def extra_surrogate_profile(torch, lib, stream) -> dict:
    """A short surrogate workload for counter profiles: 10 inferences on 1024^2 and 20 optimiser steps
    of training (batch 8, 256^2 crops of 1024^2 trajectories), every forward and backward kernel."""
    from paper_2605_07954_amd.surrogate import Trainer
    tr = Trainer(grid=1024, crop=256, batch=8, K=16, seed=0, chunk=20)
    try:
        u0, kap = wl.varcoef_problem(1024, 1024, seed=0)
        u = torch.from_numpy(u0).to("cuda")
        k = torch.from_numpy(kap).to("cuda")
        sws = torch.empty(lib.surrogate_workspace_bytes(tr.model, 1, 1024, 1024), dtype=torch.uint8, device="cuda")
        uh = torch.empty((1, 1024, 1024), device="cuda")
        for _ in range(10):
            lib.surrogate_infer(tr.model, tr.params, u, k, uh, 1, 1024, 1024, sws, stream)
        t0 = time.perf_counter()
        tr.train(160, log=None)
        torch.cuda.synchronize()
        return {"train_20_steps_s": time.perf_counter() - t0}
    finally:
        tr.close()


def extra_3d(torch, lib, stream) -> dict:
    """3D 7-point star (c0 0.4, 0.1 per neighbour) on 512^3 FP32, 50 steps: one level per pass, 8 bytes
    and 13 FLOP per update, against the HBM roof (1000 GStencil/s at 8 TB/s)."""
    n, T = 512, 50
    W = np.zeros((3, 3, 3), dtype=np.float32)
    W[1, 1, 1] = 0.4
    for d in [(0, 1, 1), (2, 1, 1), (1, 0, 1), (1, 2, 1), (1, 1, 0), (1, 1, 2)]:
        W[d] = 0.1
    x = torch.rand((n, n, n), device="cuda")
    out = torch.empty_like(x)
    ws = torch.empty_like(x)
    plan = lib.stencil_plan3d(n, n, n, 1, W, 0.0, "f32", 0)
    run = lambda: lib.stencil_run(plan, x, out, T, ws, stream)  # noqa: E731
    run()
    t = time_median(run, 10, stream)
    lib.stencil_destroy(plan)
    del x, out, ws
    torch.cuda.empty_cache()
    gst = T * n ** 3 / t / 1e9
    return {"gstencil_s": gst, "ms": t * 1e3, "alg_bytes_per_update": 8.0, "hbm_roof_gstencil": HBM_PEAK / 8 / 1e9,
            "frac_of_hbm_roof": gst / (HBM_PEAK / 8 / 1e9), "alg_hbm_gbps": gst * 8}


def extra_periodic(torch, lib, stream) -> dict:
    """Star-2D9P 8192^2 x 500 FP32 on a torus (periodic boundary; four-column marching kernels),
    autotuned, next to the same run with the zero halo."""
    p = wl.star9_precision(rows=8192, cols=8192, steps=500)
    x = torch.from_numpy(p.u0).to("cuda")
    o = torch.empty_like(x)
    w2 = torch.empty_like(x)
    res = {}
    for name, bc in (("periodic", lib.ST_BC_PERIODIC), ("dirichlet", lib.ST_BC_CONST)):
        plan = lib.stencil_plan(p.rows, p.cols, 2, p.weights, 0.0, "f32", 0)
        lib.stencil_set_boundary(plan, bc)
        tb, _, _ = lib.stencil_autotune(plan, x, o, w2, 120, stream)
        var = lib.stencil_get_variant(plan)
        run = lambda: lib.stencil_run(plan, x, o, p.steps, w2, stream)  # noqa: E731
        run()
        t = time_median(run, 10, stream)
        lib.stencil_destroy(plan)
        res[name] = {"gstencil_s": gstencil_s(p.steps, p.rows, p.cols, t), "tb": tb, "variant": VARIANT_NAMES[var]}
    del x, o, w2
    torch.cuda.empty_cache()
    return res


def extra_norms(torch, lib, stream) -> dict:
    """FP64 norms of a 16384^2 field and its predecessor (residual, energy, mass, next-step mass for
    the box49 weights): 8 bytes read per cell, against the HBM peak."""
    p = wl.box49(rows=16384, cols=16384)
    u = torch.from_numpy(p.u0).to("cuda")
    up = torch.roll(u, 1, 0).contiguous()
    plan = lib.stencil_plan(p.rows, p.cols, 3, p.weights, 0.0, "f32", 0)
    ws = torch.empty(lib.stencil_norms_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    o = torch.empty(4, dtype=torch.float64, device="cuda")
    run = lambda: lib.stencil_norms(plan, up, u, o, ws, stream)  # noqa: E731
    run()
    t = time_median(run, 20, stream)
    lib.stencil_destroy(plan)
    nbytes = 8.0 * p.rows * p.cols
    del u, up
    torch.cuda.empty_cache()
    return {"us": t * 1e6, "alg_bytes": nbytes, "gb_s": nbytes / t / 1e9, "hbm_peak_gb_s": HBM_PEAK / 1e9,
            "frac_of_hbm_peak": nbytes / t / HBM_PEAK}


EXTRAS = {"box49_tb1": ("box49_16384_tb1", extra_box49_tb1), "heat2d": ("heat2d_512_100", extra_heat2d),
          "star9": ("star9_8192_500", extra_star9),
          "batched": ("batched_256", extra_batched), "surrogate": ("surrogate_1024_K16", extra_surrogate),
          "surrogate_trained": ("surrogate_1024_K16_trained", extra_surrogate_trained),
          "star7_3d": ("star7_3d_512", extra_3d), "surrogate_profile": ("surrogate_profile", extra_surrogate_profile),
          "star9_profile": ("star9_profile", extra_star9_profile),
          "batched_profile": ("batched_profile", extra_batched_profile), "periodic": ("star9_8192_periodic", extra_periodic),
          "norms": ("norms_16384", extra_norms)}


PROFILE_ONLY = ("surrogate_profile", "star9_profile", "batched_profile")  # short runs for counter profiles, not figures


def extras(torch, lib, stream) -> dict:
    return {key: fn(torch, lib, stream) for key, fn in EXTRAS.values() if key not in PROFILE_ONLY}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=16384)
    ap.add_argument("--jacobi-steps", type=int, default=1000)
    ap.add_argument("--tb", type=int, default=0)
    ap.add_argument("--tile", type=int, nargs=2, default=None)
    ap.add_argument("--variant", type=int, default=0, help="with --tb: 0 = tiled, 1 = streaming, 2 = marching, 3 = marching with eight columns per lane, 4 = marching with one column per lane")
    ap.add_argument("--workload", default="box49", choices=["box49"] + sorted(EXTRAS),
                    help="box49: the benchmark line; any other: only that workload's figures (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB device buffer once (reference for the HBM byte counters) and exit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-oracle-timings", action="store_true",
                    help="only time the CPU oracle on every configuration (host cores; no GPU work)")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"], help="star9_profile: storage type")
    ap.add_argument("--batch-config", default="", help="batched_profile: shape:radius:engine:depth:segment_rows,...")
    ap.add_argument("--timed", action="store_true", help="batched_profile: also time 10 runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "row-slab decomposition is a design, not an implementation", file=sys.stderr)
        sys.exit(2)
    if args.cpu_oracle_timings:  # host cores only: nothing below touches the GPU
        print(json.dumps({"cpu_oracle_timings": cpu_oracle_timings()}), flush=True)
        return
    import torch
    torch.cuda.set_device(0)
    if args.copy_calibration:
        x = torch.rand(16384, 16384, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_read_bytes": x.numel() * 4, "copy_write_bytes": y.numel() * 4}), flush=True)
        return
    import paper_2605_07954_amd as lib
    stream = torch.cuda.current_stream()
    if args.workload != "box49":
        key, fn = EXTRAS[args.workload]
        if args.workload == "star9_profile":
            fn = functools.partial(fn, variant=args.variant or 2, tb=args.tb or 6, storage=args.storage)
        elif args.workload == "batched_profile":
            fn = functools.partial(fn, config=args.batch_config, timed=args.timed)
        print(json.dumps({"workload": key, **fn(torch, lib, stream)}), flush=True)
        return
    p, value, ms, roof, (tb, tx, ty, variant), tune_s = main_line(args, torch, lib, stream)
    line = {"metric": "GStencil/s", "value": value, "unit": "GStencil/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"box2d49p-{p.rows}x{p.cols}-{p.steps}steps", "stencil": "box", "radius": 3,
                       "grid": [p.rows, p.cols], "jacobi_steps": p.steps, "boundary": "dirichlet-0",
                       "tb": tb, "tile": [tx, ty], "variant": VARIANT_NAMES[variant],
                       "autotune_s": round(tune_s, 2)},
            "roofline": roof}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p)
    if not args.no_extras:
        try:
            line["extras"] = extras(torch, lib, stream)
        except Exception as e:  # noqa: BLE001 - the headline line is still valid; say what failed
            line["extras"] = {"error": repr(e)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
