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
timed region) and the FP64 CPU oracle timed on a bounded sample.
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
    ap.add_argument("--rebin-every", type=int, default=1)
    ap.add_argument("--tile", type=str, default="8,8,4,1")
    ap.add_argument("--n", type=int, default=128, help="cells per axis")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2_000_000)
    ap.add_argument("--unfused", action="store_true", help="time the unfused per-phase chain")
    ap.add_argument("--arith", choices=("f64", "f32"), default="f32",
                    help="per-particle arithmetic of the FP32-storage path")
    return ap.parse_args()


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("dust_fused.hip", "dust_device.h", "dust_particle.h"):
        with open(os.path.join(HERE, "paper_1908_10793_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel_hash: str, n_particles: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    path = os.path.join(HERE, "profiles", "fused_shearing_box_128_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_hash or d.get("n_particles") != n_particles:
        return None
    return d.get("hbm_bytes_per_launch")


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
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
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
    flags = (dust.STEP_APPLY_FEEDBACK | dust.STEP_DIAG | dust.STEP_REBIN_EVERY(args.rebin_every))
    if not args.unfused:
        flags |= dust.STEP_FUSED
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
    out = {
        "metric": "particle-steps/s (gather+exp-midpoint push+deposit)",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.arith, "data": "synthetic",
        "config": {"workload": f"shearing_box {n}^3 standard shearing box, {N} particles "
                               f"(8/cell, seeded sub-lattice), TSC, FP32 storage, {args.arith.upper()} push "
                               f"arithmetic, dt=0.005, feedback on",
                   "n_particles": N, "grid": [n, n, n], "tile": [tx, ty, tz], "slack": slack,
                   "rebin_every": args.rebin_every, "fused": not args.unfused, "graph": False,
                   "storage": "f32", "push_arith": args.arith,
                   "deposit_accum": "f32 registers per cell, f64 LDS tile window, f32 HBM atomics"},
        "roofline": roof,
        "graph_value": graph_value,
        "diag": {"momentum_residual": res, "max_cells_per_step": diag["max_cells_per_step"],
                 "n_fallback": diag["n_fallback"], "flags": diag["flag_names"],
                 "steps": diag["steps"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
