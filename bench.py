#!/usr/bin/env python3
"""Benchmark of the dust-particle hot path on one MI355X.

One step = one pass of the whole hot path over the shearing-box workload
(3-D standard shearing box, 128^3 cells, 2^24 particles, TSC weights, FP32
storage): binning by tile, half drift, weights, gather, exponential-midpoint
kick, momentum + energy deposit, half drift with shear-periodic wrap, ghost
fill and fold, feedback onto the gas, FP64 conservation sums; the loop runs
eagerly (every launch asynchronous on one stream) so that HIP events can
bracket each fused-kernel launch; the same loop replayed from a captured
hipGraph is reported beside it.  Inputs are resident in HBM before the timed
region.

Prints one JSON line: particle-steps/s, the roofline of the dominant kernel
(the fused tile kernel, timed with HIP events on its own stream inside the
timed region) and the FP64 CPU oracle timed on a bounded sample; beside
them, outside the timed step, the gas predictor's drag source on the same
particles and gas ("drag_source") and the dust density deposit
("mass_density").
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rebin-every", type=int, default=1, help="with --no-tune")
    ap.add_argument("--tile", type=str, default="8,8,4,0", help="with --no-tune")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (dust_ctx_autotune) and use --tile / --rebin-every")
    ap.add_argument("--n", type=int, default=128, help="cells per axis")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2_000_000)
    ap.add_argument("--unfused", action="store_true", help="time the unfused per-phase chain")
    ap.add_argument("--arith", choices=("f64", "f32"), default="f32",
                    help="per-particle arithmetic of the FP32-storage path")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after the run, one device-to-device copy of this many MiB (the "
                         "reference kernel of the HBM byte counters)")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("RUN_DIR", "OUT"),
                    help="write the per-kernel summary of a rocprofv3 --kernel-trace run")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT"),
                    help="write the HBM byte summary of two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) taken with --calib-copy-mb")
    ap.add_argument("--command", type=str, default="",
                    help="the profiling command, recorded in the summary")
    return ap.parse_args()


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("dust_fused.hip", "dust_device.h", "dust_particle.h"):
        with open(os.path.join(HERE, "paper_1908_10793_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


COUNTER_SUMMARY = os.path.join(HERE, "profiles", "k_fused_shearing_box_128_hbm_bytes.txt")
FUSED_KERNEL = "k_fused"


def counter_traffic(kernel_hash: str, n_particles: int):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    if not os.path.exists(COUNTER_SUMMARY):
        return None
    d = {}
    with open(COUNTER_SUMMARY) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                d[k.strip()] = v.strip()
    if d.get("kernel_source_hash") != kernel_hash or d.get("n_particles") != str(n_particles):
        return None
    return float(d["hbm_bytes_per_launch"])


def _rocpd(run_dir: str) -> str:
    import glob
    dbs = sorted(glob.glob(os.path.join(run_dir, "**", "*.db"), recursive=True))
    if not dbs:
        raise SystemExit(f"no rocprofv3 database under {run_dir}")
    return dbs[0]


def _short(name: str) -> str:
    import re
    return re.sub(r"\(.*", "", name)


def summarize_trace(run_dir: str, out: str, command: str):
    """Per-kernel calls / total / average / min / max from a --kernel-trace run."""
    import collections
    import sqlite3
    con = sqlite3.connect(_rocpd(run_dir))
    agg = collections.defaultdict(list)
    for name, t0, t1 in con.execute("select name, start, end from kernels order by start"):
        agg[_short(name)].append((t1 - t0) * 1e-3)
    tot = sum(sum(v) for v in agg.values())
    lines = ["# rocprofv3 kernel trace summary (durations in microseconds; avg_warm_us leaves",
             "# out each kernel's first, cold launch)",
             f"# command: {command}", "",
             f"{'kernel':64s} {'calls':>6s} {'total_ms':>9s} {'avg_us':>9s} {'avg_warm_us':>11s} "
             f"{'min_us':>9s} {'max_us':>9s} {'pct':>6s}"]
    for nm, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        warm = v[1:] if len(v) > 1 else v
        lines.append(f"{nm[:64]:64s} {len(v):6d} {sum(v) / 1e3:9.3f} {sum(v) / len(v):9.2f} "
                     f"{sum(warm) / len(warm):11.2f} {min(v):9.2f} {max(v):9.2f} {100 * sum(v) / tot:6.2f}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _counter_per_dispatch(run_dir: str, counter: str):
    """Value of a counter for every dispatch: {kernel name: [values]}."""
    import collections
    import sqlite3
    con = sqlite3.connect(_rocpd(run_dir))
    per = collections.defaultdict(float)
    names = {}
    for di, name, val in con.execute(
            "select dispatch_id, kernel_name, value from counters_collection where counter_name = ?",
            (counter,)):
        per[di] += val
        names[di] = _short(name)
    out = collections.defaultdict(list)
    for di in sorted(per):
        out[names[di]].append(per[di])
    return out


def summarize_counters(fetch_dir: str, write_dir: str, out: str, command: str,
                       n_particles: int, copy_mb: int):
    """HBM bytes per launch of the fused kernel: FETCH_SIZE and WRITE_SIZE (KiB
    per dispatch), each scaled by the ratio of known to counted bytes of a
    device-to-device copy of copy_mb MiB."""
    fetch = _counter_per_dispatch(fetch_dir, "FETCH_SIZE")
    write = _counter_per_dispatch(write_dir, "WRITE_SIZE")
    copy_kib = copy_mb * 1024.0
    # the calibration copy is the largest copy dispatch of the run
    def is_copy(k):
        return "copy" in k.lower() or "elementwise" in k.lower()
    cf = max(max(v) for k, v in fetch.items() if is_copy(k))
    cw = max(max(v) for k, v in write.items() if is_copy(k))
    f_fetch, f_write = copy_kib / cf, copy_kib / cw
    # mean over the fused dispatches after the first (cold) one
    def warm_mean(v):
        w = v[1:] if len(v) > 1 else v
        return sum(w) / len(w), len(w)
    kf = [warm_mean(v) for k, v in fetch.items() if FUSED_KERNEL + "<" in k]
    kw = [warm_mean(v) for k, v in write.items() if FUSED_KERNEL + "<" in k]
    (kf, nfd), (kw, nwd) = kf[0], kw[0]
    kf, kw = [kf], [kw]
    fb = kf[0] * f_fetch * 1024.0
    wb = kw[0] * f_write * 1024.0
    lines = ["# HBM bytes of the fused kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per",
             "# dispatch), each scaled by known/counted bytes of a device copy of known size",
             f"# command: {command}",
             f"kernel: {FUSED_KERNEL}",
             f"kernel_source_hash: {source_hash()}",
             f"n_particles: {n_particles}",
             f"copy_mib: {copy_mb}",
             f"copy_fetch_kib_counted: {cf:.1f}",
             f"copy_write_kib_counted: {cw:.1f}",
             f"fetch_scale: {f_fetch:.4f}",
             f"write_scale: {f_write:.4f}",
             f"fused_dispatches_averaged: {nfd} (FETCH), {nwd} (WRITE); the first, cold one left out",
             f"fused_fetch_kib_counted: {kf[0]:.1f}",
             f"fused_write_kib_counted: {kw[0]:.1f}",
             f"fused_fetch_bytes: {fb:.4g}",
             f"fused_write_bytes: {wb:.4g}",
             f"hbm_bytes_per_launch: {fb + wb:.6g}"]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def cpu_baseline(w, sample: int):
    """The FP64 oracle (serial C, one core) on the first `sample` particles of
    the same workload, one step."""
    import numpy as np
    import dataclasses
    from oracle.run import OracleRun
    sel = np.arange(min(sample, w.n))
    ws = dataclasses.replace(w, cell=w.cell[sel], off=w.off[sel], mom=w.mom[sel],
                             species=w.species[sel] if w.species is not None else None)
    run = OracleRun(ws)
    t0 = time.perf_counter()
    run.step(1)
    dt = time.perf_counter() - t0
    return {"value": len(sel) / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 step of {len(sel)} of the {w.n} particles on the full {w.boxes[0]['n']} "
                      f"grid (serial FP64 C oracle, {dt:.1f} s)"}


def main():
    args = parse()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace[0], args.summarize_trace[1], args.command)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, args.command, 8 * args.n ** 3,
                           args.calib_copy_mb)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1908_10793_amd import dust, synth

    n = args.n
    w = synth.shearing_box(n=(n, n, n), dtype="f32")
    N = w.n
    ctx = dust.context_for(w)
    tx, ty, tz, slack = (int(v) for v in args.tile.split(","))
    ctx.set_tile(tx, ty, tz, slack)
    ctx.set_arith(args.arith)
    P, F = dust.upload(w, ctx, with_id=False)
    flags = dust.STEP_APPLY_FEEDBACK | dust.STEP_DIAG
    tuned = None
    if args.unfused:
        pass
    elif args.no_tune:
        flags |= dust.STEP_FUSED | dust.STEP_REBIN_EVERY(args.rebin_every)
    else:
        # tile shape and rebinning interval from the autotuner (on copies)
        tuned = ctx.autotune(P, F, w.dt, dust.forces_for(w, 0.0), flags, steps=12)
        (tx, ty, tz), rebin = tuned["tile"], tuned["rebin_every"]
        args.rebin_every = rebin
        flags |= dust.STEP_FUSED           # interval from the context
    K, W = args.steps, args.warmup
    t = 0.0
    torch.cuda.synchronize()
    # warm-up
    if W > 0:
        ctx.step(P, F, w.dt, dust.forces_for(w, t), W, flags)
        t += W * w.dt
    torch.cuda.synchronize()
    ctx.status()
    ctx.set_profile(K)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    ctx.step(P, F, w.dt, dust.forces_for(w, t), K, flags)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    t += K * w.dt
    kern = ctx.profile(K) if not args.unfused else []
    diag = ctx.status()
    value = N * K / (ms * 1e-3)
    ppc = N / (n ** 3)
    bytes_per_pstep = 56.0 + 48.0 / ppc          # algorithmic bytes per particle-step
    roof = None
    if kern:
        kavg = float(np.mean(kern)) * 1e-3
        achieved = bytes_per_pstep * N / kavg / 1e9
        khash = source_hash()
        traffic = counter_traffic(khash, N)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_fused", "kernel_avg_us": round(kavg * 1e6, 2),
                "algorithmic_bytes_per_launch": bytes_per_pstep * N, "kernel_source_hash": khash}
    res = float(np.max(np.abs(np.array(diag["p_part"]) + np.array(diag["p_grid"])))) / max(
        diag["sum_abs_j"], 1e-300)
    # the same loop replayed from a captured hipGraph (not the headline)
    ctx.set_profile(0)
    gflags = flags | dust.STEP_GRAPH
    ctx.step(P, F, w.dt, dust.forces_for(w, t), K, gflags)   # capture
    t += K * w.dt
    torch.cuda.synchronize()
    e0.record(stream)
    ctx.step(P, F, w.dt, dust.forces_for(w, t), K, gflags)
    e1.record(stream)
    torch.cuda.synchronize()
    graph_value = N * K / (e0.elapsed_time(e1) * 1e-3)
    t += K * w.dt
    ctx.status()
    # the gas predictor's drag source (Eq. f_D) on the same particles and gas,
    # reported beside the step (not part of it): one launch per call
    fr = dust.forces_for(w, t)
    ctx.drag_source(P, F, w.dt, fr)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(K):
        ctx.drag_source(P, F, w.dt, fr)
    e1.record(stream)
    torch.cuda.synchronize()
    ds_s = e0.elapsed_time(e1) * 1e-3 / K
    ds_bytes = (28.0 + 1.0 + 36.0 / ppc) * N       # state + species + gas read / deposit RMW
    drag_source = {"kernel": "k_drag_source", "us_per_launch": round(ds_s * 1e6, 2),
                   "algorithmic_bytes_per_launch": ds_bytes,
                   "achieved": round(ds_bytes / ds_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                   "unit": "GB/s", "frac": round(ds_bytes / ds_s / 1e9 / HBM_PEAK_GBS, 4)}
    # the dust density deposit on the same particles (beside the step)
    rho_d = torch.zeros_like(F["rho"])
    ctx.deposit_mass(P, rho_d)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(K):
        ctx.deposit_mass(P, rho_d)
    e1.record(stream)
    torch.cuda.synchronize()
    md_s = e0.elapsed_time(e1) * 1e-3 / K
    md_bytes = (16.0 + 1.0 + 8.0 / ppc) * N          # cell + offsets + species, density RMW
    mass_density = {"kernel": "k_mass_density", "us_per_launch": round(md_s * 1e6, 2),
                    "algorithmic_bytes_per_launch": md_bytes,
                    "achieved": round(md_bytes / md_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(md_bytes / md_s / 1e9 / HBM_PEAK_GBS, 4)}
    del rho_d
    # measured device-to-device copy bandwidth (read + write bytes), the
    # practical ceiling the fused kernel's rate is also compared with
    nel = 256 << 20                                   # 1 GiB of float32
    src = torch.ones(nel, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(5):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2.0 * 4 * nel * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    if roof is not None:
        roof["copy_gbs"] = round(copy_gbs, 1)
        roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)
    out = {
        "metric": "particle-steps/s (gather+exp-midpoint push+deposit)",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.arith, "data": "synthetic",
        "config": {"workload": f"shearing_box {n}^3 standard shearing box, {N} particles "
                               f"(8/cell, seeded sub-lattice), TSC, FP32 storage, {args.arith.upper()} push "
                               f"arithmetic, dt=0.005, feedback on",
                   "n_particles": N, "grid": [n, n, n], "tile": [tx, ty, tz], "slack": slack,
                   "rebin_every": args.rebin_every, "autotuned": tuned,
                   "fused": not args.unfused, "graph": False,
                   "storage": "f32", "push_arith": args.arith,
                   "deposit_accum": "f32 registers per cell, f64 LDS tile window, f32 HBM atomics"},
        "roofline": roof,
        "graph_value": graph_value,
        "drag_source": drag_source,
        "mass_density": mass_density,
        "diag": {"momentum_residual": res, "max_cells_per_step": diag["max_cells_per_step"],
                 "n_fallback": diag["n_fallback"], "flags": diag["flag_names"],
                 "steps": diag["steps"]},
    }
    if args.calib_copy_mb > 0:
        nel = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
