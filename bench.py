"""Throughput of subcycled RK4 on the 7-level tower hierarchy, one MI355X.

Workload: scalar wave, 7 levels with refinement ratio 2 in space and time,
128^3 periodic coarse grid on [-1,1]^3, two nested towers of 128^3 cells at
x = -0.3 and +0.3 merging on the three coarsest levels, every level split
into seeded uneven blocks of 16^3..48^3; seeded sum of 8 Gaussian pulses.
27,424,754 owned points, 542,962,934 point-updates per coarse step.

A step is one coarse step of the whole schedule (every level advanced,
prolonged, and restricted).  `value` is grid-point updates per second
(owned points times level steps) in the HIP-graph batched FP64 mode; the
per-block, batched-eager and graph modes are reported side by side, with the
stencil kernel's HBM roofline from HIP events around its launches and the
CPU reference implementation timed on a bounded sample on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--modes ...] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point updates/s (subcycled RK4) batched/mixed vs plain FP64; % HBM peak"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_context(sc, spec, mode, data, precision=0):
    ctx = sc.Context(device="cuda:0", exec=mode, precision=precision)
    ctx.build_spec(spec, block_seed=1, min_block=16, max_block=48)
    ctx.bind()
    for l in range(spec.nlevels):
        for v in range(2):
            ctx.set_initial_data(0, l, v, data[l][v])
    return ctx


def timed(ctx, torch, steps):
    torch.cuda.synchronize()
    ctx.synchronize()
    t0 = time.perf_counter()
    ctx.advance(steps)
    ctx.synchronize()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_baseline():
    """Reference implementation, one coarse step of the same tower family at N0 = 64."""
    from oracle.evolve import OracleRun
    from oracle.hierarchy import Hierarchy
    from workloads import config_c3, pulses_on_spec
    spec = config_c3(64)
    run = OracleRun(Hierarchy(spec))
    for l in range(spec.nlevels):
        for v, f in enumerate(pulses_on_spec(spec, l)):
            run.set_data(l, v, f)
    t0 = time.perf_counter()
    run.advance(1)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    u = spec.updates_per_coarse_step()
    return {"value": u / dt, "unit": "grid-point updates/s", "cores": cores, "kind": "oracle",
            "sample": f"one coarse step of the 7-level tower hierarchy at N0=64 "
                      f"({spec.total_points()} points, {u} point-updates), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n0", type=int, default=128)
    ap.add_argument("--modes", default="graph,batched,per_block,mixed")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "layout is a design, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2503_09629_amd as sc
    from workloads import config_c3, pulses_on_spec

    spec = config_c3(args.n0)
    log(f"workload {spec.name}: {spec.total_points()} points, "
        f"{spec.updates_per_coarse_step()} updates per coarse step")
    data = [pulses_on_spec(spec, l) for l in range(spec.nlevels)]
    U = spec.updates_per_coarse_step()
    zc = spec.total_points() * (1 << (spec.nlevels - 1))   # as if unsubcycled
    modes = [m.strip() for m in args.modes.split(",") if m.strip()]
    res = {}
    roof = None
    for m in modes:
        log(f"mode {m} ...")
        mode = {"graph": sc.SC_EXEC_GRAPH, "batched": sc.SC_EXEC_BATCHED,
                "per_block": sc.SC_EXEC_PER_BLOCK, "mixed": sc.SC_EXEC_GRAPH,
                "mixed_batched": sc.SC_EXEC_BATCHED}[m]
        prec = sc.SC_MIXED if m.startswith("mixed") else sc.SC_FP64
        ctx = make_context(sc, spec, mode, data, prec)
        if m != "per_block" and not args.no_tune:
            ctx.autotune(3)
        shapes = [ctx.tile_shape(l) for l in range(spec.nlevels)]
        steps = args.steps if m != "per_block" else max(1, min(args.steps, 2))
        ctx.advance(max(1, args.warmup) if m != "per_block" else 1)
        ctx.synchronize()
        T = timed(ctx, torch, steps)
        res[m] = {"updates_per_s": U * steps / T, "ms_per_step": 1e3 * T / steps,
                  "steps": steps, "tz_per_level": [sh["tz"] for sh in shapes],
                  "grid_per_level": [sh["grid"] for sh in shapes]}
        log(f"{m}: {1e3 * T / steps:.2f} ms/step, {U * steps / T:.4g} updates/s")
        if m in ("batched", "mixed_batched"):
            label = "roofline" if m == "batched" else "roofline_mixed"
            ctx.profile_enable(True)
            ctx.advance(steps)
            n, ms, nbytes = ctx.profile_read()
            ctx.profile_enable(False)
            achieved = nbytes / (ms * 1e-3) / 1e9
            r = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                 "kernel": "k_wave_stage (all four stages, batched, "
                           + ("FP64" if m == "batched" else "FP32 stencil") + ")",
                 "launches": n, "avg_launch_us": 1e3 * ms / n,
                 "alg_bytes_per_launch": nbytes / n}
            if label == "roofline":
                roof = r
            else:
                res[m]["roofline"] = r
            log(f"stage kernel: {n} launches, avg {1e3 * ms / n:.1f} us, {achieved:.0f} GB/s")
        if ctx.check_finite() != sc.SC_OK:
            raise SystemExit(f"non-finite values in mode {m}")
        ctx.close()
        del ctx
        torch.cuda.empty_cache()

    primary = "graph" if "graph" in res else modes[0]
    out = {
        "metric": METRIC,
        "value": res[primary]["updates_per_s"],
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": res[primary]["steps"],
        "warmup": args.warmup,
        "ms_per_step": res[primary]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"scalar wave, 7-level two-tower hierarchy, N0={args.n0}, "
                               f"subcycled RK4, FP64, {primary} mode",
                   "owned_points": spec.total_points(), "updates_per_coarse_step": U,
                   "levels": spec.nlevels, "block_sides": "16..48", "block_seed": 1},
        "modes": res,
        "paper_style_zone_cycles_per_s": zc * res[primary]["updates_per_s"] / U,
    }
    if "per_block" in res:
        for m in res:
            res[m]["speedup_vs_per_block"] = res[m]["updates_per_s"] / res["per_block"]["updates_per_s"]
    if roof is not None:
        out["roofline"] = roof
    if not args.no_cpu:
        log("timing the CPU reference implementation ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
