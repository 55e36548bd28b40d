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
import glob
import hashlib
import json
import os
import re
import sqlite3
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point updates/s (subcycled RK4) batched/mixed vs plain FP64; % HBM peak"
HBM_PEAK_GBS = 8000.0
HBM_PEAK_BPS = HBM_PEAK_GBS * 1e9
FP64_VALU_PEAK = 78.6e12          # FP64 vector FLOP/s
# algorithmic HBM bytes per point-update (both variables, one RK4 step, interior
# only): reading y_n and the stage vectors and writing k1..k4, the stage
# vectors and y_{n+1} in FP64 (144 B per variable); with the FP32 stencil
# operands and slopes of the mixed mode 100 B per variable
SURVEY_BYTES = {"fp64": 288.0, "mixed": 200.0}


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "wave_stage_n0128_fp64_hbm_traffic.md")
Z4C_COUNTERS = os.path.join(ROOT, "profiles", "z4c_c5_fp64_step_counters.md")


def kernel_source_hash():
    """sha256 over the stencil kernel source and the host code that cuts its tiles."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "capi.cpp"):
        h.update(open(os.path.join(ROOT, "paper_2503_09629_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(mode_result):
    """HBM bytes per stage-kernel launch (scaled FETCH_SIZE + WRITE_SIZE) from the
    committed counter summary, or None unless it was taken on the current
    kernel source with the tile shapes this run uses."""
    try:
        txt = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch:\s*(\S+)", txt)
    h = re.search(r"kernel_source_sha256:\s*(\w+)", txt)
    sh = re.search(r"tile_shapes:\s*(\{.*\})", txt)
    if not m or not h or not sh or kernel_source_hash() != h.group(1):
        return None
    keys = ("tx_per_level", "tz_per_level", "grid_per_level", "depth_per_level",
            "slots_per_level", "threads_per_level")
    want = json.loads(sh.group(1))
    if any(want.get(k) != mode_result.get(k) for k in keys):
        return None
    return float(m.group(1))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# -- rocprofv3 output summaries (the text kept under profiles/) ---------------
def _rows_from_csv(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def trace_dispatches(folder):
    """Kernel dispatches of a rocprofv3 --kernel-trace run (CSV or SQLite output)
    as (name, start_ns, end_ns), in start order."""
    out = []
    for path in glob.glob(os.path.join(folder, "**", "*kernel_trace.csv"), recursive=True):
        for r in _rows_from_csv(path):
            out.append((r["Kernel_Name"], int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    if not out:
        for path in glob.glob(os.path.join(folder, "**", "*_results.db"), recursive=True):
            con = sqlite3.connect(path)
            out += [(n, int(a), int(b)) for n, a, b in
                    con.execute("select name, start, end from kernels")]
            con.close()
    out.sort(key=lambda r: r[1])
    return out


def counter_dispatches(folder, counter):
    """Per-dispatch values of one counter from a rocprofv3 --pmc run (CSV output)
    as (name, dispatch id, value) in dispatch order."""
    out = {}
    for path in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        for r in _rows_from_csv(path):
            if r.get("Counter_Name") != counter:
                continue
            key = int(r["Dispatch_Id"])
            name, val = r["Kernel_Name"], float(r["Counter_Value"])
            out[key] = (name, key, out.get(key, (name, key, 0.0))[2] + val)
    return [out[k] for k in sorted(out)]


def summarize_trace(folder, kernel_re, last, top=16):
    rows = trace_dispatches(folder)
    stats = {}
    for n, a, b in rows:
        d = stats.setdefault(n, [0, 0.0, 1e30, 0.0])
        us = (b - a) / 1e3
        d[0] += 1
        d[1] += us
        d[2] = min(d[2], us)
        d[3] = max(d[3], us)
    total = sum(d[1] for d in stats.values())
    lines = ["```", f"{'kernel':60s} {'calls':>6s} {'total_ms':>9s} {'avg_us':>8s} {'min_us':>8s} "
             f"{'max_us':>8s} {'%':>5s}"]
    for n, d in sorted(stats.items(), key=lambda kv: -kv[1][1])[:top]:
        short = re.sub(r"\([^()]*\)$", "", n.replace("void ", "", 1)
                       .replace("sc::(anonymous namespace)::", ""))[:60]
        lines.append(f"{short:60s} {d[0]:6d} {d[1] / 1e3:9.2f} {d[1] / d[0]:8.2f} {d[2]:8.2f} "
                     f"{d[3]:8.2f} {100 * d[1] / total:5.1f}")
    lines.append("```")
    sel = [r for r in rows if re.search(kernel_re, r[0])]
    if last:
        sel = sel[-last:]
    if sel:
        avg = sum(b - a for _, a, b in sel) / len(sel) / 1e3
        lines.append(f"\n{kernel_re}: last {len(sel)} dispatches, average {avg:.2f} us, "
                     f"total {sum(b - a for _, a, b in sel) / 1e6:.3f} ms")
    return "\n".join(lines)


def summarize_counters(fetch_dir, write_dir, probe_fetch_dir, probe_write_dir, kernel_re, last,
                       probe_bytes):
    """HBM bytes per dispatch of the kernels matching kernel_re: FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch, separate runs), each scaled by the ratio of
    the known bytes to the same counter's reading for the copy probe (the last
    launch of bench.py --copy-probe-mib, an elementwise kernel moving
    probe_bytes each way)."""
    def per_dispatch(folder, counter):
        sel = [v for n, _, v in counter_dispatches(folder, counter) if re.search(kernel_re, n)]
        sel = sel[-last:] if last else sel
        return sum(sel) / len(sel) * 1024.0, len(sel)
    fetch, nf = per_dispatch(fetch_dir, "FETCH_SIZE")
    write, nw = per_dispatch(write_dir, "WRITE_SIZE")
    pf = counter_dispatches(probe_fetch_dir, "FETCH_SIZE")[-1][2] * 1024.0
    pw = counter_dispatches(probe_write_dir, "WRITE_SIZE")[-1][2] * 1024.0
    sf, sw = probe_bytes / pf, probe_bytes / pw
    return {"dispatches": [nf, nw], "fetch_kib": fetch / 1024, "write_kib": write / 1024,
            "fetch_scale": sf, "write_scale": sw, "traffic_bytes_per_launch": fetch * sf + write * sw}


def z4c_source_hash():
    """sha256 over the Z4c kernels, the shared kernels and the host code that launches them."""
    h = hashlib.sha256()
    for f in ("z4c.hip", "kernels.hip", "capi.cpp"):
        h.update(open(os.path.join(ROOT, "paper_2503_09629_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def step_window(rows, anchor_re, per_step, step=1):
    """Dispatch index range [i0, i1) of one coarse step: from the first anchor
    dispatch of coarse step `step` (0-based) to the first of the next.  This is
    the step shifted cyclically, which holds the same dispatches as long as the
    two steps run the same launch sequence (no other work between them)."""
    idx = [i for i, r in enumerate(rows) if re.search(anchor_re, r[0])]
    if len(idx) <= (step + 1) * per_step:
        raise SystemExit(f"{len(idx)} dispatches of {anchor_re}: fewer than {step + 2} steps of "
                         f"{per_step}")
    return idx[step * per_step], idx[(step + 1) * per_step]


def short_name(n):
    return re.sub(r"\([^()]*\)$", "", n.replace("void ", "", 1)
                  .replace("sc::(anonymous namespace)::", ""))


def summarize_step(trace_dir, fetch_dir, write_dir, flops_dir, probe_fetch_dir, probe_write_dir,
                   anchor_re, per_step, probe_bytes):
    """Per-kernel time, HBM bytes and FP64 VALU FLOPs over one coarse step
    (step_window in each run), against 8 TB/s and 78.6 TFLOP/s."""
    pf = counter_dispatches(probe_fetch_dir, "FETCH_SIZE")[-1][2] * 1024.0
    pw = counter_dispatches(probe_write_dir, "WRITE_SIZE")[-1][2] * 1024.0
    sf, sw = probe_bytes / pf, probe_bytes / pw
    per = {}

    def add(rows, key, scale):
        i0, i1 = step_window(rows, anchor_re, per_step)
        for r in rows[i0:i1]:
            d = per.setdefault(short_name(r[0]), {"calls": 0, "us": 0.0, "fetch": 0.0, "write": 0.0,
                                                  "flops": 0.0})
            if key == "us":
                d["calls"] += 1
                d["us"] += (r[2] - r[1]) / 1e3
            else:
                d[key] += r[2] * scale
    add(trace_dispatches(trace_dir), "us", 1.0)
    add(counter_dispatches(fetch_dir, "FETCH_SIZE"), "fetch", 1024.0 * sf)
    add(counter_dispatches(write_dir, "WRITE_SIZE"), "write", 1024.0 * sw)
    # the counter adds each FP64 VALU instruction's operations per lane (FMA 2)
    # once per wave: times 64 lanes (an upper bound where lanes are masked off)
    add(counter_dispatches(flops_dir, "SQ_INSTS_VALU_FLOPS_FP64"), "flops", 64.0)
    fma = sum(r[2] for r in counter_dispatches(flops_dir, "SQ_INSTS_VALU_FMA_F64")[
        slice(*step_window(counter_dispatches(flops_dir, "SQ_INSTS_VALU_FMA_F64"), anchor_re,
                           per_step))])
    lines = ["| kernel | calls | ms | HBM GB | TB/s | % HBM | FP64 GFLOP | TFLOP/s | % FP64 VALU |",
             "|---|---|---|---|---|---|---|---|---|"]
    tot = {"us": 0.0, "bytes": 0.0, "flops": 0.0}
    for n, d in sorted(per.items(), key=lambda kv: -kv[1]["us"]):
        b = d["fetch"] + d["write"]
        tot["us"] += d["us"]
        tot["bytes"] += b
        tot["flops"] += d["flops"]
        if d["us"] <= 0:
            continue
        s_ = d["us"] * 1e-6
        lines.append(f"| `{n}` | {d['calls']} | {d['us'] / 1e3:.2f} | {b / 1e9:.2f} | "
                     f"{b / s_ / 1e12:.2f} | {100 * b / s_ / HBM_PEAK_BPS:.1f} | "
                     f"{d['flops'] / 1e9:.1f} | {d['flops'] / s_ / 1e12:.2f} | "
                     f"{100 * d['flops'] / s_ / FP64_VALU_PEAK:.1f} |")
    s_ = tot["us"] * 1e-6
    lines.append(f"| all kernels | | {tot['us'] / 1e3:.2f} | {tot['bytes'] / 1e9:.2f} | "
                 f"{tot['bytes'] / s_ / 1e12:.2f} | {100 * tot['bytes'] / s_ / HBM_PEAK_BPS:.1f} | "
                 f"{tot['flops'] / 1e9:.1f} | {tot['flops'] / s_ / 1e12:.2f} | "
                 f"{100 * tot['flops'] / s_ / FP64_VALU_PEAK:.1f} |")
    lines += ["", f"copy-probe scale FETCH / WRITE: {sf:.4f} / {sw:.4f}; "
                  f"FP64 FMA instructions (wave level) in the step: {fma:.4g}", "",
              f"hbm_bytes_per_coarse_step: {tot['bytes']:.6e}",
              f"fp64_flops_per_coarse_step: {tot['flops']:.6e}",
              f"kernel_ms_per_coarse_step: {tot['us'] / 1e3:.3f}",
              f"kernel_source_sha256: {z4c_source_hash()}"]
    return "\n".join(lines)


def z4c_roofline(step_s):
    """Whole-step %HBM and %FP64-VALU of the Z4c run: counted HBM bytes and FP64
    VALU FLOPs per coarse step from the committed counter summary (taken on the
    same kernels, FP64, frozen boundary, fourth order), over this run's time."""
    try:
        txt = open(Z4C_COUNTERS).read()
    except OSError:
        return {"unavailable": "no counter summary"}
    b = re.search(r"hbm_bytes_per_coarse_step:\s*(\S+)", txt)
    f = re.search(r"fp64_flops_per_coarse_step:\s*(\S+)", txt)
    h = re.search(r"kernel_source_sha256:\s*(\w+)", txt)
    if not (b and f and h) or h.group(1) != z4c_source_hash():
        return {"unavailable": "counter summary taken on other kernel sources"}
    by, fl = float(b.group(1)), float(f.group(1))
    hb, fp = by / step_s / HBM_PEAK_BPS, fl / step_s / FP64_VALU_PEAK
    return {"bound": "hbm" if hb >= fp else "alu", "scope": "whole coarse step, all kernels",
            "achieved": by / step_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hb,
            "traffic": by, "fp64_valu": {"achieved": fl / step_s / 1e12,
                                         "peak": FP64_VALU_PEAK / 1e12, "unit": "TFLOP/s",
                                         "frac": fp, "flops_per_coarse_step": fl},
            "counters": os.path.relpath(Z4C_COUNTERS, ROOT)}


def summarize_runs(folder, nruns, steps, anchor_re, per_step):
    """Kernel table per run of a trace holding several benchmark runs in one
    process (separated at the nruns - 1 longest idle gaps): the dispatches from
    the start of the last `steps` coarse steps of each run (located by the
    anchor kernel, per_step launches per coarse step), per kernel family
    (template arguments dropped), divided by `steps`."""
    rows = trace_dispatches(folder)
    gaps = sorted(range(1, len(rows)), key=lambda i: rows[i][1] - rows[i - 1][2])[-(nruns - 1):]
    cuts = [0] + sorted(gaps) + [len(rows)]
    out = []
    for r in range(nruns):
        run = rows[cuts[r]:cuts[r + 1]]
        idx = [i for i, x in enumerate(run) if re.search(anchor_re, x[0])]
        i0 = idx[-steps * per_step] if len(idx) >= steps * per_step else 0
        fam = {}
        for n, a, b in run[i0:]:
            k = re.sub(r"<.*", "", short_name(n))
            d = fam.setdefault(k, [0, 0.0])
            d[0] += 1
            d[1] += (b - a) / 1e3
        tot = sum(d[1] for d in fam.values())
        lines = [f"### run {r + 1}: kernels of its last {steps} coarse steps, per coarse step", "",
                 "| kernel | launches / step | ms / step | share |", "|---|---|---|---|"]
        for k, d in sorted(fam.items(), key=lambda kv: -kv[1][1]):
            lines.append(f"| `{k}` | {d[0] / steps:.1f} | {d[1] / steps / 1e3:.2f} | "
                         f"{100 * d[1] / tot:.1f} % |")
        lines.append(f"| total | {sum(d[0] for d in fam.values()) / steps:.1f} | "
                     f"{tot / steps / 1e3:.2f} | |")
        out.append("\n".join(lines))
    return "\n\n".join(out)


def summarize_markers(folder):
    """roctx ranges of a rocprofv3 --marker-trace run, grouped by name with the
    step counters taken out: calls, total and average host duration."""
    stats = {}
    for path in glob.glob(os.path.join(folder, "**", "*marker_api_trace.csv"), recursive=True):
        for r in _rows_from_csv(path):
            name = re.sub(r"step \d+", "step n", r["Function"])
            d = stats.setdefault(name, [0, 0.0])
            d[0] += 1
            d[1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    lines = ["| range | calls | total ms | average us |", "|---|---|---|---|"]
    for n, d in sorted(stats.items()):
        lines.append(f"| {n} | {d[0]} | {d[1] / 1e3:.2f} | {d[1] / d[0]:.1f} |")
    return "\n".join(lines)


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


def timed_reps(ctx, torch, steps, reps=5):
    """Exactly `steps` coarse steps, in `reps` groups each synchronised and
    timed: total seconds and the per-step milliseconds of every group."""
    sizes = [steps // reps + (1 if i < steps % reps else 0) for i in range(min(reps, steps))]
    total, per = 0.0, []
    for n in sizes:
        t = timed(ctx, torch, n)
        total += t
        per.append(1e3 * t / n)
    return total, per


def stage_roofline(ctx, steps, U, precision):
    """Stage-kernel roofline from HIP events around every batched stage launch
    (the context must be in an eager mode) over `steps` coarse steps."""
    ctx.profile_enable(True)
    ctx.advance(steps)
    n, ms, own_bytes = ctx.profile_read()
    ctx.profile_enable(False)
    alg = SURVEY_BYTES[precision] * U * steps          # algorithmic bytes of these launches
    achieved = alg / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "k_wave_stage (all four stages, batched, "
                      + ("FP64" if precision == "fp64" else "mixed: FP64 stage 1, FP32 stages 2-4") + ")",
            "launches": n, "avg_launch_us": 1e3 * ms / n,
            "alg_bytes_per_launch": alg / n,
            "alg_bytes_per_point_update": SURVEY_BYTES[precision],
            "achieved_kernel_minimum_bytes": own_bytes / (ms * 1e-3) / 1e9,
            "kernel_minimum_bytes_per_launch": own_bytes / n}


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        m = re.search(r"Model name:\s*(.+)", out)
        return m.group(1).strip() if m else None
    except (OSError, subprocess.SubprocessError):
        return None


def cpu_baseline(n0=128):
    """The CPU reference implementation on the benchmark hierarchy itself, timed
    on a bounded sample: the first descent of the subcycling recursion (one
    RK4 step of every level, coarse to fine, with each level's stage ghost
    fills and the prolongation from its parent), i.e. every owned point
    advanced once.  Median of three repetitions with all host threads, and
    one repetition with one thread."""
    import ctypes
    from oracle.evolve import OracleRun
    from oracle.hierarchy import Hierarchy
    from workloads import config_c3, pulses_on_spec
    spec = config_c3(n0)
    t0 = time.perf_counter()
    run = OracleRun(Hierarchy(spec))
    for l in range(spec.nlevels):
        for v, f in enumerate(pulses_on_spec(spec, l)):
            run.set_data(l, v, f)
    log(f"cpu reference: hierarchy and storage set up in {time.perf_counter() - t0:.0f} s")
    gomp = ctypes.CDLL("libgomp.so.1")
    nproc = len(os.sched_getaffinity(0))
    if "OMP_NUM_THREADS" in os.environ:
        nproc = min(nproc, int(os.environ["OMP_NUM_THREADS"]))

    def descent():
        t = time.perf_counter()
        for l in range(spec.nlevels):
            run.rk4_step(l)
            if l + 1 < spec.nlevels:
                run.prolongate(l + 1)
                run.theta0[l + 1] = 0.0
        return time.perf_counter() - t

    u = spec.total_points()
    legs = {}
    for threads, reps in ((nproc, 3), (1, 1)):
        gomp.omp_set_num_threads(threads)
        ts = sorted(descent() for _ in range(reps))
        legs[threads] = ts[len(ts) // 2]
        log(f"cpu reference, {threads} threads: {legs[threads]:.2f} s per sample "
            f"({u / legs[threads]:.4g} updates/s)")
    gomp.omp_set_num_threads(nproc)
    sample = (f"7-level tower hierarchy at N0={n0} ({u} points): one RK4 step of every level "
              f"(coarse to fine, with ghost fills and prolongations), {u} point-updates")
    return {"value": u / legs[nproc], "unit": "grid-point updates/s", "cores": nproc,
            "kind": "oracle", "sample": sample + f", median of 3: {legs[nproc]:.2f} s",
            "single_thread": {"value": u / legs[1], "seconds": legs[1], "cores": 1},
            "cpu_model": cpu_model()}


def ens_run(args):
    """C1 ensembles: B independent periodic 32^3 standing-wave members (seeded
    modes m_d in {1, 2, 3} and amplitudes in [0.5, 1.5]) advanced together, one
    batched launch per RK4 stage over all members, 64 steps of dt = 1/64 to
    t = 1, then 8 more.  Per B: the stage kernel's event-timed roofline over
    the first 8 steps (batched eager), graph-mode throughput over the other
    64 (one capture step, 63 timed in 5 groups, median) and the largest
    max-norm error of u against the members' exact solutions at t = 9/8."""
    import torch
    import paper_2503_09629_amd as sc
    from workloads import ensemble_c1
    from workloads.data import ensemble_params
    out = {"workload": "C1 ensembles: B members of a periodic 32^3 scalar-wave level on [-1,1]^3, "
                       "seeded standing waves (seed 2), dt = 1/64, 72 steps", "runs": []}
    for B in args.ens_b:
        spec = ensemble_c1(B, 32)
        U = B * spec.updates_per_coarse_step()
        ctx = sc.Context(device="cuda:0", exec=sc.SC_EXEC_BATCHED)
        ctx.build_spec(spec, block_seed=1, min_block=16, max_block=48)
        ctx.bind()
        ctx.set_initial_data_analytic(sc.SC_ID_STANDING_WAVE, (), seed=2)
        if not args.no_tune:
            ctx.autotune()
        roof = stage_roofline(ctx, 8, U, "fp64")        # the first 8 of 72 steps
        ctx.set_exec(sc.SC_EXEC_GRAPH)
        ctx.advance(1)                      # graph capture
        ctx.synchronize()
        total, per = timed_reps(ctx, torch, 63)
        t = ctx.level_time(0)
        err = 0.0
        for m, (modes, a0) in enumerate(ensemble_params(B, 2)):
            e = ctx.error_norms(m, 0, 0, sc.SC_ID_STANDING_WAVE, (a0,) + tuple(modes) + (t,))
            err = max(err, float(e[0]))
        ms = float(np.median(per))
        log(f"ens B={B}: {ms:.3f} ms per step, {U / ms * 1e3:.4g} updates/s, stage kernel "
            f"{roof['frac']:.3f} of HBM, max error {err:.3e} at t = {t}")
        out["runs"].append({"B": B, "points": B * spec.total_points(), "ms_per_step": ms,
                            "ms_per_step_groups": per, "updates_per_s": U / ms * 1e3,
                            "roofline": roof, "max_error_u": err, "t": t,
                            "tile_shape": ctx.tile_shape(0)})
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    return out


def z4c_run(args):
    """Z4c two-puncture evolution on the 7-level 96^3 tower hierarchy."""
    import torch
    import paper_2503_09629_amd as sc
    from workloads import canonical_coords, config_c5
    spec = config_c5(96)
    U = spec.updates_per_coarse_step()
    log(f"workload {spec.name}: {spec.total_points()} points, {U} updates per coarse step")
    mixed = args.z4c_precision == "mixed"
    radiative = args.z4c_bc == "radiative"
    ctx = sc.Context(device="cuda:0", rhs=sc.SC_RHS_Z4C, exec=sc.SC_EXEC_GRAPH,
                     precision=sc.SC_MIXED if mixed else sc.SC_FP64,
                     outer_bc=sc.SC_BC_RADIATIVE if radiative else sc.SC_BC_FROZEN,
                     fd_order=args.z4c_fd_order, ko_order=args.z4c_ko_order)
    ctx.build_spec(spec)
    ctx.bind()
    # Brill-Lindquist punctures m = 0.5 at x = +-3, evaluated on the device
    # (fields and the frozen physical-boundary ghosts)
    ctx.set_initial_data_analytic(sc.SC_ID_BRILL_LINDQUIST, (0.5, 0.5, 3.0, -3.0))
    x0, y0, z0 = canonical_coords(spec, 0)
    r0 = np.sqrt(x0 * x0 + y0 * y0 + z0 * z0)
    outer = (r0 > 64.0) & (np.maximum(np.maximum(abs(x0), abs(y0)), abs(z0)) < 112.0)

    def hnorm():
        # composite-grid L2 over r < 30 where alpha > 0.3, each point on the
        # finest level that has it, weight dx^3 (on the device)
        return float(ctx.constraint_norm(0, 30.0, 0.3)[0])

    def hnorm_outer():
        # level 0 between r = 64 and 6 points inside the outer boundary (|x_i| < 112)
        H = ctx.hamiltonian(0, 0)
        return float(np.sqrt(np.mean(H[outer] ** 2)))

    hist = []
    log("z4c: initial data set; first coarse step (graph capture) ...")
    t0 = time.perf_counter()
    ctx.advance(1)
    ctx.synchronize()
    log(f"z4c: first coarse step {time.perf_counter() - t0:.2f} s")
    hist.append((ctx.level_time(0), hnorm()))
    outer_hist = [(ctx.level_time(0), hnorm_outer())]
    log(f"z4c: t = {hist[-1][0]:.4f}, ||H|| = {hist[-1][1]:.4e}")
    steps = args.z4c_steps - 1
    torch.cuda.synchronize()
    T = 0.0
    for i in range(steps):
        t0 = time.perf_counter()
        ctx.advance(1)
        ctx.synchronize()
        T += time.perf_counter() - t0
        log(f"z4c: coarse step {i + 2}/{args.z4c_steps}: {T / (i + 1) * 1e3:.1f} ms per step")
        if args.z4c_h_every and (i + 2) % args.z4c_h_every == 0:
            outer_hist.append((ctx.level_time(0), hnorm_outer()))
            log(f"z4c: t = {outer_hist[-1][0]:.2f}: ||H|| near the outer boundary "
                f"{outer_hist[-1][1]:.4e}")
    hist.append((ctx.level_time(0), hnorm()))
    log(f"z4c: {1e3 * T / steps:.1f} ms per coarse step, {U * steps / T:.4g} updates/s")
    finite = ctx.check_finite() == sc.SC_OK
    profiled = not mixed and not radiative and args.z4c_fd_order == 4 and args.z4c_ko_order == 5
    return {"metric": "Z4c grid-point updates/s (subcycled RK4, 22 variables)",
            "value": U * steps / T, "unit": "grid-point updates/s", "n_gpus": 1,
            "steps": steps, "ms_per_step": 1e3 * T / steps,
            "roofline": z4c_roofline(T / steps) if profiled else None,
            "dtype": "f32 RHS, f64 state" if mixed else "f64",
            "config": {"workload": "Z4c Brill-Lindquist punctures m=0.5 at x=+-3, 7 levels of "
                                   "96^3, [-128,128]^3, graph mode"
                                   + (", FP32 right-hand side" if mixed else "")},
            "outer_bc": args.z4c_bc, "fd_order": args.z4c_fd_order,
            "ko_order": args.z4c_ko_order,
            "hamiltonian_L2": [{"t": t, "H": h} for t, h in hist],
            "hamiltonian_L2_outer_shell": [{"t": t, "H": h} for t, h in outer_hist],
            "finite": finite}


def e1_run(args):
    """The paper's scalar-wave test (Sec. IV.A): outgoing spherical Gaussian on a
    periodic [-6,6]^3 with refined boxes over [-4,4]^3 and [-1,1]^3, coarse
    spacing 0.032/1.2^k; max-norm error of u on the second refined level
    against the exact solution, subcycled and uniform time steps."""
    import torch
    import paper_2503_09629_amd as sc
    from workloads import canonical_coords, config_e1, grown_for_buffer_zones, spherical_gaussian
    from workloads.data import E1_AMPLITUDE, E1_SIGMA
    checkpoints = [round(0.4 * (i + 1), 10) for i in range(int(round(args.e1_t / 0.4)))]
    modes = [m.strip() for m in args.e1_modes.split(",") if m.strip()]
    out = {"workload": "scalar wave E1: spherical Gaussian A=1, sigma=0.25/sqrt(2), periodic "
                       "[-6,6]^3, refined boxes [-4,4]^3 and [-1,1]^3 (snapped outward)",
           "checkpoints": checkpoints, "runs": []}
    for mode in modes:
        uniform = mode == "uniform"
        buffered = mode == "buffer"
        for n0 in args.e1_n0:
            spec = config_e1(n0)
            if buffered:
                # buffer zones: the boxes grow by 10 so that the valid region
                # (9 buffer layers inside) covers the paper's boxes
                spec0, spec = spec, grown_for_buffer_zones(spec, 10)
            dt_steps = 0.25 * spec.dx(spec.nlevels - 1 if uniform else 0)
            U = spec.total_points() if uniform else spec.updates_per_coarse_step()
            log(f"e1 {mode} n0={n0}: {spec.total_points()} points, dt {dt_steps:.6g}")
            ts = (sc.SC_UNIFORM_DT if uniform else sc.SC_BUFFER_ZONES if buffered
                  else sc.SC_SUBCYCLED)
            ctx = sc.Context(device="cuda:0", exec=sc.SC_EXEC_GRAPH, time_stepping=ts)
            ctx.build_spec(spec, block_seed=1, min_block=16, max_block=48)
            ctx.bind()
            ctx.set_initial_data_analytic(sc.SC_ID_SPHERICAL_GAUSSIAN,
                                          (E1_AMPLITUDE, E1_SIGMA, 0.0))
            lev = spec.nlevels - 1
            x, y, z = canonical_coords(spec, lev)
            sel = slice(None)
            if buffered:   # the error is taken on the paper's finest box only
                (glo, ghi), = spec.fine_boxes[-1]
                (olo, ohi), = spec0.fine_boxes[-1]
                n = [ghi[d] - glo[d] + 1 for d in range(3)]
                idx = np.arange(n[0] * n[1] * n[2]).reshape(n[2], n[1], n[0])
                sel = idx[olo[2] - glo[2]:ohi[2] - glo[2] + 1, olo[1] - glo[1]:ohi[1] - glo[1] + 1,
                          olo[0] - glo[0]:ohi[0] - glo[0] + 1].ravel()
                x, y, z = x[sel], y[sel], z[sel]
            errs, steps_done, T = [], 0, 0.0
            for tc in checkpoints:
                nsteps = int(round(tc / dt_steps)) - steps_done
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.advance(nsteps)
                ctx.synchronize()
                T += time.perf_counter() - t0
                steps_done += nsteps
                t = ctx.level_time(lev)
                if buffered:   # a sub-box of the level: on the host
                    ue, _ = spherical_gaussian(t, x, y, z)
                    e = float(np.abs(ctx.read_back(0, lev, 0)[sel] - ue).max())
                else:
                    e = float(ctx.error_norms(0, lev, 0, sc.SC_ID_SPHERICAL_GAUSSIAN,
                                              (E1_AMPLITUDE, E1_SIGMA, t))[0])
                errs.append(e)
                log(f"  t = {t:.4f}: max |u - u_exact| on level {lev} = {e:.4e} "
                    f"({steps_done} steps, {U * steps_done / T:.4g} updates/s)")
            out["runs"].append({"mode": mode, "n0": n0, "coarse_dx": spec.dx(0),
                                "finest_dx": spec.dx(lev), "points": spec.total_points(),
                                "steps": steps_done, "errors": errs,
                                "updates_per_s": U * steps_done / T, "seconds": T})
            ctx.close()
            del ctx, x, y, z
            torch.cuda.empty_cache()
    # observed orders between successive resolutions (ratio 1.2)
    for mode in modes:
        runs = [r for r in out["runs"] if r["mode"] == mode]
        for a, b in zip(runs, runs[1:]):
            ratio = a["coarse_dx"] / b["coarse_dx"]
            b["order_vs_previous"] = [float(np.log(ea / eb) / np.log(ratio)) if eb > 0 else None
                                      for ea, eb in zip(a["errors"], b["errors"])]
    return out


def carpet_run(args):
    """The paper's cost comparison (Sec. II, Fig. 1) on the tower hierarchy:
    dense-output subcycling on the benchmark boxes against buffer-zone
    (Carpet) subcycling on the same boxes grown by 10 points per side, whose
    valid region (the boxes minus 3G = 9 buffer layers) covers the original
    boxes.  Both in graph mode with autotuned tile shapes."""
    import torch
    import paper_2503_09629_amd as sc
    from workloads import config_c3, grown_for_buffer_zones, pulses_on_spec
    base = config_c3(args.n0)
    grown = grown_for_buffer_zones(base, 10)
    out = {"workload": f"wave, 7-level towers N0={args.n0}: dense output on the benchmark boxes "
                       f"vs buffer zones on the boxes grown by 10", "runs": []}
    for name, spec, ts in (("dense-output", base, sc.SC_SUBCYCLED),
                           ("buffer-zones", grown, sc.SC_BUFFER_ZONES)):
        t0 = time.perf_counter()
        ctx = sc.Context(device="cuda:0", exec=sc.SC_EXEC_GRAPH, time_stepping=ts)
        ctx.build_spec(spec, block_seed=1, min_block=16, max_block=48)
        tbuild = time.perf_counter() - t0
        ctx.bind()
        for l in range(spec.nlevels):
            for v, f in enumerate(pulses_on_spec(spec, l)):
                ctx.set_initial_data(0, l, v, f)
        log(f"carpet: {name}: {spec.total_points()} points, hierarchy built in {tbuild:.1f} s")
        ctx.autotune(3)
        nl = spec.nlevels
        owned = [ctx.counts(l)[1] for l in range(nl)]
        nrb = [ctx.counts(l)[2] for l in range(nl)]
        nbuf = [ctx.buffer_count(l) for l in range(nl)]
        U = sum(owned[l] << l for l in range(nl))
        if ts == sc.SC_BUFFER_ZONES:
            # one state vector per fine step into RB and buffer points
            prolonged = sum((nrb[l] + nbuf[l]) << l for l in range(1, nl))
        else:
            # five vectors (y_n, k1..k4) once per parent step into the RB points
            prolonged = sum(5 * (nrb[l] << (l - 1)) for l in range(1, nl))
        for i in range(args.carpet_warmup):
            ctx.advance(1)
        ctx.synchronize()
        log(f"carpet: {name}: warm ({args.carpet_warmup} coarse steps)")
        T = timed(ctx, torch, args.carpet_steps)
        ms = 1e3 * T / args.carpet_steps
        log(f"carpet: {name}: {ms:.2f} ms per coarse step, {U * args.carpet_steps / T:.4g} updates/s")
        fin = ctx.norms(0, nl - 1, 0)
        out["runs"].append({
            "scheme": name, "ms_per_coarse_step": ms, "updates_per_coarse_step": U,
            "updates_per_s": U * args.carpet_steps / T,
            "owned_points": sum(owned), "buffer_points": sum(nbuf),
            "valid_points": sum(owned) - sum(nbuf), "rb_points": sum(nrb),
            "prolonged_points_per_coarse_step": prolonged,
            "per_level": {"owned": owned, "rb": nrb, "buffer": nbuf},
            "finest_level_max_abs_u": float(fin[0]), "finite": bool(fin[2] == 0)})
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    d, b = out["runs"]
    out["dense_over_buffer"] = {
        "time": d["ms_per_coarse_step"] / b["ms_per_coarse_step"],
        "prolonged_points": d["prolonged_points_per_coarse_step"] / b["prolonged_points_per_coarse_step"],
        "rhs_updates": d["updates_per_coarse_step"] / b["updates_per_coarse_step"]}
    return out


def fd8_run(args):
    """The tower hierarchy with the eighth-order Laplacian (four ghost
    layers, Sec. III.C's production stencil) against the fourth-order run, and
    the eighth-order one with the ninth-order dissipation (five ghost layers),
    all in graph mode with autotuned tiles."""
    import torch
    import paper_2503_09629_amd as sc
    from workloads import config_c3, pulses_on_spec
    spec = config_c3(args.n0)
    data = [pulses_on_spec(spec, l) for l in range(spec.nlevels)]
    U = spec.updates_per_coarse_step()
    out = {"workload": f"wave, 7-level towers N0={args.n0}, fourth vs eighth order "
                       "(fifth- and ninth-order dissipation)", "runs": []}
    for order, ko in ((4, 5), (8, 5), (8, 9)):
        ctx = sc.Context(device="cuda:0", exec=sc.SC_EXEC_GRAPH, fd_order=order, ko_order=ko)
        ctx.build_spec(spec, block_seed=1, min_block=16, max_block=48)
        ctx.bind()
        for l in range(spec.nlevels):
            for v in range(2):
                ctx.set_initial_data(0, l, v, data[l][v])
        ctx.autotune(3)
        for i in range(args.carpet_warmup):
            ctx.advance(1)
        ctx.synchronize()
        log(f"fd{order} ko{ko}: warm")
        T = timed(ctx, torch, args.carpet_steps)
        ms = 1e3 * T / args.carpet_steps
        fin = ctx.norms(0, spec.nlevels - 1, 0)
        log(f"fd{order} ko{ko}: {ms:.2f} ms per coarse step, "
            f"{U * args.carpet_steps / T:.4g} updates/s")
        out["runs"].append({"fd_order": order, "ko_order": ko, "ms_per_coarse_step": ms,
                            "updates_per_s": U * args.carpet_steps / T,
                            "arena_gib": ctx.device_bytes() / 2 ** 30,
                            "finest_level_max_abs_u": float(fin[0]), "finite": bool(fin[2] == 0)})
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    return out


def precision_report(args):
    """Mixed vs FP64 on the tower hierarchy at t = 1/8: max-norm difference of
    u and Pi per level, and observed orders of both precisions from the three
    resolutions (differences of successive resolutions on common points)."""
    import paper_2503_09629_amd as sc
    from workloads import config_c3, pulses_on_spec
    res = {}
    for n0 in args.report_n0:
        spec = config_c3(n0)
        nsteps = int(round(0.125 / (0.25 * 2.0 / n0)))
        out = {}
        log(f"precision report: N0={n0}, {spec.total_points()} points, {nsteps} coarse steps")
        data = [pulses_on_spec(spec, l) for l in range(spec.nlevels)]
        for prec in (sc.SC_FP64, sc.SC_MIXED):
            ctx = make_context(sc, spec, sc.SC_EXEC_GRAPH, data, prec)
            for i in range(nsteps):
                ctx.advance(1)
                if (i + 1) % 16 == 0 or i + 1 == nsteps:
                    ctx.synchronize()
                    log(f"  {'mixed' if prec == sc.SC_MIXED else 'fp64'}: {i + 1}/{nsteps} coarse steps")
            out[prec] = [[ctx.read_back(0, l, v) for v in range(2)] for l in range(spec.nlevels)]
            ctx.close()
        del data
        res[n0] = out
        log(f"precision report: N0={n0} done")
    levels = []
    n0s = list(args.report_n0)
    for l in range(7):
        row = {"level": l}
        for v, name in enumerate(("u", "Pi")):
            row[f"max_abs_mixed_minus_fp64_{name}"] = {
                n0: float(np.abs(res[n0][0][l][v] - res[n0][1][l][v]).max()) for n0 in n0s}
            row[f"max_abs_{name}_fp64"] = {n0: float(np.abs(res[n0][0][l][v]).max()) for n0 in n0s}
            if len(n0s) == 3:
                for prec, key in ((0, "fp64"), (1, "mixed")):
                    a, b, c = (res[n][prec][l][v] for n in n0s)
                    shp = [config_c3(n).boxes(l) for n in n0s]
                    e1 = np.abs(_common(a, shp[0], 1) - _common(b, shp[1], 2)).max()
                    e2 = np.abs(_common(b, shp[1], 2) - _common(c, shp[2], 4)).max()
                    row[f"diff_{name}_{key}"] = [float(e1), float(e2)]
                    row[f"order_{name}_{key}"] = float(np.log2(e1 / e2)) if e2 > 0 else None
        levels.append(row)
        log(json.dumps(row))
    return {"report": "mixed precision vs FP64, 7-level tower hierarchy, t = 1/8",
            "n0": n0s, "levels": levels}


def _common(u, boxes, stride):
    """Points of a level common to all three resolutions (every stride-th point)."""
    out, off = [], 0
    for lo, hi in boxes:
        n = [hi[d] - lo[d] + 1 for d in range(3)]
        a = u[off:off + n[0] * n[1] * n[2]].reshape(n[2], n[1], n[0])
        out.append(a[::stride, ::stride, ::stride].ravel())
        off += n[0] * n[1] * n[2]
    return np.concatenate(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n0", type=int, default=128)
    ap.add_argument("--modes", default="graph,batched,per_block,mixed")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the short C5 Z4c and C1-ensemble runs of the default line")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--shapes", default=None,
                    help="JSON line of an earlier run: take its tile shapes instead of tuning")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--workload", default="wave",
                    choices=("wave", "z4c", "precision", "e1", "carpet", "fd8", "ens"))
    ap.add_argument("--ens-b", type=int, nargs="+", default=[64, 512, 1024])
    ap.add_argument("--carpet-steps", type=int, default=8)
    ap.add_argument("--carpet-warmup", type=int, default=4)
    ap.add_argument("--e1-n0", type=int, nargs="+", default=[375, 450, 540])
    ap.add_argument("--e1-t", type=float, default=1.6)
    ap.add_argument("--e1-modes", default="subcycled,uniform")
    ap.add_argument("--z4c-steps", type=int, default=16)
    ap.add_argument("--z4c-precision", default="fp64", choices=("fp64", "mixed"))
    ap.add_argument("--z4c-bc", default="frozen", choices=("frozen", "radiative"))
    ap.add_argument("--z4c-fd-order", type=int, default=4, choices=(4, 8))
    ap.add_argument("--z4c-ko-order", type=int, default=5, choices=(5, 9),
                    help="dissipation order (9: the r = 8 operator, needs --z4c-fd-order 8)")
    ap.add_argument("--z4c-h-every", type=int, default=0,
                    help="also report the constraint near the outer boundary every N coarse steps")
    ap.add_argument("--report-n0", type=int, nargs="+", default=[64, 128, 256])
    ap.add_argument("--summarize-trace", metavar="DIR", default=None,
                    help="print a kernel table of a rocprofv3 --kernel-trace output folder")
    ap.add_argument("--summarize-counters", metavar="DIR", nargs=4, default=None,
                    help="FETCH_SIZE, WRITE_SIZE, copy-probe FETCH_SIZE, copy-probe WRITE_SIZE "
                         "output folders of rocprofv3 --pmc runs: HBM bytes per dispatch")
    ap.add_argument("--summarize-runs", metavar="DIR", default=None,
                    help="kernel table per run of a trace of several runs (--runs, --per-step, "
                         "--anchor k_wave_stage, --last: coarse steps per run)")
    ap.add_argument("--runs", type=int, default=2)
    ap.add_argument("--summarize-markers", metavar="DIR", default=None,
                    help="table of the roctx ranges of a rocprofv3 --marker-trace output folder")
    ap.add_argument("--summarize-step", metavar="DIR", nargs=6, default=None,
                    help="kernel-trace, FETCH_SIZE, WRITE_SIZE, FP64-FLOP counter, copy-probe "
                         "FETCH_SIZE and copy-probe WRITE_SIZE output folders: per-kernel time, "
                         "HBM bytes and FP64 FLOPs of one coarse step")
    ap.add_argument("--anchor", default="k_z4c_evol",
                    help="kernel launched a fixed number of times per coarse step (--summarize-step)")
    ap.add_argument("--per-step", type=int, default=508,
                    help="launches of the anchor kernel per coarse step (--summarize-step)")
    ap.add_argument("--kernel", default="k_wave_stage", help="kernel name regex for the summaries")
    ap.add_argument("--last", type=int, default=0, help="summarise only the last N matching dispatches")
    ap.add_argument("--probe-mib", type=int, default=1024)
    args = ap.parse_args()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace, args.kernel, args.last))
        return
    if args.summarize_runs:
        print(summarize_runs(args.summarize_runs, args.runs, args.last or 1, args.anchor,
                             args.per_step))
        return
    if args.summarize_markers:
        print(summarize_markers(args.summarize_markers))
        return
    if args.summarize_step:
        print(summarize_step(*args.summarize_step, args.anchor, args.per_step,
                             args.probe_mib << 20))
        return
    if args.summarize_counters:
        print(json.dumps(summarize_counters(*args.summarize_counters, args.kernel, args.last,
                                            args.probe_mib << 20)))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "layout is described in the design notes, not implemented", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe_mib > 0:
        import torch
        n = args.copy_probe_mib << 17          # float64 elements
        src = torch.ones(n + 1, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):                     # runtime copy kernel, 16 B per lane
            dst[:n].copy_(src[:n])
        for _ in range(3):                     # elementwise kernel at an odd offset: 8 B per lane
            torch.mul(src[1:], 1.0, out=dst[1:])
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": n * 8, "launches": 6}), flush=True)
        return
    if args.workload == "z4c":
        print(json.dumps(z4c_run(args)), flush=True)
        return
    if args.workload == "e1":
        print(json.dumps(e1_run(args)), flush=True)
        return
    if args.workload == "precision":
        print(json.dumps(precision_report(args)), flush=True)
        return
    if args.workload == "carpet":
        print(json.dumps(carpet_run(args)), flush=True)
        return
    if args.workload == "fd8":
        print(json.dumps(fd8_run(args)), flush=True)
        return
    if args.workload == "ens":
        print(json.dumps(ens_run(args)), flush=True)
        return

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
        if m != "per_block" and args.shapes:
            with open(args.shapes) as f:
                tuned = json.loads(f.read().strip().splitlines()[-1])["modes"][m]
            for l in range(spec.nlevels):
                ctx.set_tile_shape(l, tuned["tz_per_level"][l], tuned["grid_per_level"][l],
                                   tuned["depth_per_level"][l], tuned["slots_per_level"][l],
                                   tuned["threads_per_level"][l], tuned["tx_per_level"][l])
        elif m != "per_block" and not args.no_tune:
            ctx.autotune(3)
        shapes = [ctx.tile_shape(l) for l in range(spec.nlevels)]
        steps = args.steps if m != "per_block" else max(1, min(args.steps, 2))
        ctx.advance(max(1, args.warmup) if m != "per_block" else 1)
        ctx.synchronize()
        T, per = timed_reps(ctx, torch, steps)
        res[m] = {"updates_per_s": U * steps / T, "ms_per_step": 1e3 * T / steps,
                  "ms_per_step_reps": per, "ms_per_step_median": float(np.median(per)),
                  "steps": steps, "tx_per_level": [sh["tx"] for sh in shapes],
                  "tz_per_level": [sh["tz"] for sh in shapes],
                  "grid_per_level": [sh["grid"] for sh in shapes],
                  "depth_per_level": [sh["depth"] for sh in shapes],
                  "slots_per_level": [sh["slots"] for sh in shapes],
                  "threads_per_level": [sh["threads"] for sh in shapes]}
        log(f"{m}: {1e3 * T / steps:.2f} ms/step (median of {len(per)} groups "
            f"{np.median(per):.2f}), {U * steps / T:.4g} updates/s")
        if m in ("graph", "mixed"):
            # the same context and tile shapes, stage launches timed one by one
            ctx.set_exec(sc.SC_EXEC_BATCHED)
            r = stage_roofline(ctx, min(steps, 3), U, "mixed" if prec == sc.SC_MIXED else "fp64")
            if m == "graph":
                if args.n0 == 128:
                    t = measured_traffic(res[m])
                    if t is not None:
                        r["traffic"] = t
                        r["traffic_unit"] = "HBM bytes per launch (rocprofv3 counters)"
                        r["traffic_over_algorithmic"] = t / r["alg_bytes_per_launch"]
                        r["traffic_over_kernel_minimum"] = t / r["kernel_minimum_bytes_per_launch"]
                roof = r
            else:
                res[m]["roofline"] = r
            log(f"stage kernel ({m}): {r['launches']} launches, avg {r['avg_launch_us']:.1f} us, "
                f"{r['achieved']:.0f} GB/s of algorithmic bytes (frac {r['frac']:.3f})")
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
    if "mixed" in res and "graph" in res:
        res["mixed"]["speedup_vs_fp64_graph"] = res["mixed"]["updates_per_s"] / res["graph"]["updates_per_s"]
    out["kernel_source_sha256"] = kernel_source_hash()
    if roof is not None:
        out["roofline"] = roof
    if not args.no_secondary:
        # short runs of the other measured workloads, so that their numbers
        # come from the same benchmark invocation (reported, not the metric)
        sec = {}
        for name, fn in (("z4c_c5_fp64", lambda: z4c_run(argparse.Namespace(
                             z4c_steps=3, z4c_precision="fp64", z4c_bc="frozen",
                             z4c_fd_order=4, z4c_ko_order=5, z4c_h_every=0))),
                         ("c1_ensemble_b512", lambda: ens_run(argparse.Namespace(
                             ens_b=[512], no_tune=args.no_tune)))):
            log(f"secondary workload {name} ...")
            try:
                sec[name] = fn()
            except Exception as e:      # reported in the line, the metric stands
                sec[name] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.empty_cache()
        out["secondary"] = sec
    if not args.no_cpu:
        log("timing the CPU reference implementation ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
