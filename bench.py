#!/usr/bin/env python3
"""Benchmark of the dust-particle hot path on one MI355X.

One step = one pass of the whole hot path over one batch of synthetic input:
binning by tile (every k steps, k from the autotuner), half drift, weights,
gather, exponential-midpoint kick, momentum + energy deposit, half drift with
wrap, ghost fill and fold, feedback onto the gas, FP64 conservation sums.
Inputs are resident in HBM before the timed region.

Workloads (--config):
  5 (default, the headline)  8 independent periodic cubes of 32^3 .. 192^3
      cells of width 1/64 (15,073,280 cells), 4 species (tau = 0.01, 0.1, 1, 10), U{1..32}
      particles per cell and species (about 9.95e8 particles), TSC, FP32
      storage and push, dt = 0.01; one launch per step covers every box; the
      K-step loop is captured in a hipGraph and replayed.
  2  3-D shearing box 128^3, 2^24 particles (8 per cell), TSC, FP32.
  3  cylindrical disk 256x512x64 (log R), 2^25 particles, Stokes numbers.
  4  spherical disk 256x128x512, 2^26 particles, stiff stopping times.
  1  2-D periodic box 64^2, 65,536 particles, CIC, FP64.

Prints one JSON line: particle-steps/s (median of 5 timed runs of the K
steps, launched from the host), the roofline of the dominant kernel (the fused
tile kernel, timed with HIP events recorded on the library's stream around
every launch inside the timed runs), the same K steps replayed from a captured
hipGraph (timing.graph), the worst error of one step against the FP64 oracle on the box the
oracle can step (box 0 for config 5, a particle sample otherwise), the plain
FP64 GPU step (unfused, FP64 storage and arithmetic) with its own error and the
speed-up over it, and the oracle timed on the host cores (one thread, and
every core with OpenMP).  With config 5 the 128^3 shearing box is reported too
(key "config2").
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
CU_COUNT = 256           # MI355X compute units
CLOCK_HZ = 2.4e9         # peak engine clock
METRIC = "particle-steps/s (gather+exp-midpoint push+deposit)"
WORKLOAD_NAMES = {1: "cart2d_periodic", 2: "shearing_box", 3: "cylindrical_disk",
                  4: "spherical_disk", 5: "batched_boxes"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=5, choices=(1, 2, 3, 4, 5))
    ap.add_argument("--reps", type=int, default=5, help="timed replays of the K steps (median)")
    ap.add_argument("--rebin-every", type=int, default=1, help="with --no-tune")
    ap.add_argument("--tile", type=str, default="8,8,4,0", help="with --no-tune")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (dust_ctx_autotune) and use --tile / --rebin-every")
    ap.add_argument("--tune-steps", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 GPU step")
    ap.add_argument("--no-curvilinear", action="store_true",
                    help="skip the cylindrical and spherical disks (FP64 vs FP32 arithmetic)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the side measurements (drag source, dust density, config 2)")
    ap.add_argument("--no-check", action="store_true", help="skip the parity check against the oracle")
    ap.add_argument("--eager", action="store_true", help="time the eager loop, not the graph")
    ap.add_argument("--arith", choices=("f64", "f32"), default=None,
                    help="per-particle arithmetic of the FP32-storage path (default: the "
                         "context's, FP32)")
    ap.add_argument("--cpu-sample", type=int, default=2_000_000,
                    help="particles the oracle steps for the CPU baseline (configs 2-4)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after the run, one device-to-device copy of this many MiB (the "
                         "reference kernel of the HBM byte counters)")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("RUN_DIR", "OUT"),
                    help="write the per-kernel summary of a rocprofv3 --kernel-trace run")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT"),
                    help="write the HBM byte summary of two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) taken with --calib-copy-mb")
    ap.add_argument("--n-particles", type=int, default=0,
                    help="with --summarize-counters: particles of the profiled run")
    ap.add_argument("--command", type=str, default="",
                    help="the profiling command, recorded in the summary")
    return ap.parse_args()


# ------------------------------------------------------------------ profiles

def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "paper_1908_10793_amd", "csrc")
    for f in ("dust_fused_kern.h", "dust_cart3_kern.h", "dust_cart3.hip", "dust_device.h", "dust_particle.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# tile kernels of the fused step: FP32 uniform 3-D Cartesian boxes with the
# species table (shearing box, batched boxes), and the general one
TILE_KERNELS = ("k_c3", "k_fused")


def tile_kernel(cfg: int, dtype: str, arith: str) -> str:
    return "k_c3" if cfg in (2, 5) and dtype == "f32" and arith == "f32" else "k_fused"


def profile_path(kernel: str, name: str, what: str, tile, rebin: int) -> str:
    """A committed rocprofv3 summary of this workload and tiling (the file
    name carries the tile shape and the rebinning interval)."""
    tag = f"{tile[0]}x{tile[1]}x{tile[2]}_every{rebin}"
    return os.path.join(HERE, "profiles", f"{kernel}_{name}_{tag}_{what}.txt")


def counter_traffic(kernel: str, name: str, kernel_hash: str, n_particles: int, tile, rebin: int):
    """HBM bytes per launch of the tile kernel from the committed rocprofv3
    counter summary of this workload and tiling, if it was taken on the
    current kernel source and the same particle count."""
    path = profile_path(kernel, name, "hbm_bytes", tile, rebin)
    if not os.path.exists(path):
        return None
    d = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                d[k.strip()] = v.strip()
    if d.get("kernel_source_hash") != kernel_hash or d.get("n_particles") != str(n_particles):
        return None
    return float(d["hbm_bytes_per_launch"])


def counter_valu(kernel: str, name: str, kernel_hash: str, tile, rebin: int):
    """VALU wave-instructions per launch of the tile kernel (launch-weighted
    over its variants) from the committed rocprofv3 SQ counter summary of
    this workload and tiling, if it was taken on the current kernel source
    with the same tile shape and rebinning interval."""
    import re
    path = profile_path(kernel, name, "sq_counters", tile, rebin)
    if not os.path.exists(path):
        return None
    total = launches = 0.0
    ok_hash = ok_cfg = False
    with open(path) as fh:
        for line in fh:
            if line.startswith("# kernel_source_hash:"):
                ok_hash = line.split(":", 1)[1].strip() == kernel_hash
            elif line.startswith("# command:"):
                m = re.search(r"--tile (\d+),(\d+),(\d+)", line)
                k = re.search(r"--rebin-every (\d+)", line)
                ok_cfg = bool(m and k) and [int(m.group(i)) for i in (1, 2, 3)] == list(tile) and \
                    int(k.group(1)) == rebin
            elif "SQ_INSTS_VALU " in line and not line.startswith("#"):
                m = re.search(r"SQ_INSTS_VALU\s+([0-9.e+-]+)\s+\(launches (\d+)\)", line)
                if m:
                    total += float(m.group(1)) * int(m.group(2))
                    launches += int(m.group(2))
    if not (ok_hash and ok_cfg and launches):
        return None
    return total / launches


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
    # every template variant of a tile kernel together (what the bench's HIP
    # events average over)
    for kn in TILE_KERNELS:
        allv = []
        for t0, t1, name in con.execute("select start, end, name from kernels order by start"):
            if kn + "<" in _short(name):
                allv.append((t1 - t0) * 1e-3)
        if allv:
            agg[f"{kn} (all variants)"] = allv
    lines = ["# rocprofv3 kernel trace summary (durations in microseconds; avg_warm_us leaves",
             "# out each kernel's first, cold launch; 'all variants' lines repeat the launches",
             "# of every template variant of a tile kernel and are not counted in pct)",
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


def _kernel_dispatches(run_dir: str, counter: str, kernel: str):
    """The counter's value for every dispatch of any variant of a kernel, in
    dispatch order."""
    import collections
    import sqlite3
    con = sqlite3.connect(_rocpd(run_dir))
    per = collections.defaultdict(float)
    for di, name, val in con.execute(
            "select dispatch_id, kernel_name, value from counters_collection where counter_name = ?",
            (counter,)):
        if kernel + "<" in _short(name):
            per[di] += val
    return [per[di] for di in sorted(per)]


def _last_copy(run_dir: str, counter: str, is_copy):
    """The counter's value for the last copy dispatch of a run."""
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
    return per[max(di for di in per if is_copy(names[di]))]


def summarize_counters(fetch_dir: str, write_dir: str, out: str, command: str,
                       n_particles: int, copy_mb: int):
    """HBM bytes per launch of the fused kernel: FETCH_SIZE and WRITE_SIZE (KiB
    per dispatch), each scaled by the ratio of known to counted bytes of a
    device-to-device copy of copy_mb MiB."""
    fetch = _counter_per_dispatch(fetch_dir, "FETCH_SIZE")
    write = _counter_per_dispatch(write_dir, "WRITE_SIZE")
    copy_kib = copy_mb * 1024.0

    def is_copy(k):
        return "copy" in k.lower() or "elementwise" in k.lower()
    # the calibration copy is the run's last copy dispatch (made at its end)
    cf = _last_copy(fetch_dir, "FETCH_SIZE", is_copy)
    cw = _last_copy(write_dir, "WRITE_SIZE", is_copy)
    f_fetch, f_write = copy_kib / cf, copy_kib / cw

    def warm_mean(v):
        w = v[1:] if len(v) > 1 else v
        return sum(w) / len(w), len(w)
    kernel = [kn for kn in TILE_KERNELS if any(kn + "<" in k for k in fetch)][0]
    # every template variant, in dispatch order (the first, cold one left out)
    kf, nfd = warm_mean(_kernel_dispatches(fetch_dir, "FETCH_SIZE", kernel))
    kw, nwd = warm_mean(_kernel_dispatches(write_dir, "WRITE_SIZE", kernel))
    fb = kf * f_fetch * 1024.0
    wb = kw * f_write * 1024.0
    lines = ["# HBM bytes of the fused kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per",
             "# dispatch), each scaled by known/counted bytes of a device copy of known size",
             f"# command: {command}",
             f"kernel: {kernel}",
             f"kernel_source_hash: {source_hash()}",
             f"n_particles: {n_particles}",
             f"copy_mib: {copy_mb}",
             f"copy_fetch_kib_counted: {cf:.1f}",
             f"copy_write_kib_counted: {cw:.1f}",
             f"fetch_scale: {f_fetch:.4f}",
             f"write_scale: {f_write:.4f}",
             f"fused_dispatches_averaged: {nfd} (FETCH), {nwd} (WRITE); the first, cold one left out",
             f"fused_fetch_kib_counted: {kf:.1f}",
             f"fused_write_kib_counted: {kw:.1f}",
             f"fused_fetch_bytes: {fb:.4g}",
             f"fused_write_bytes: {wb:.4g}",
             f"hbm_bytes_per_launch: {fb + wb:.6g}"]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


# ------------------------------------------------------------------ host

def host_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"nproc": aff, "cpu_count": os.cpu_count(), "cpu_model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


# ------------------------------------------------------------------ workloads

def make_workload(cfg: int, dtype: str):
    from paper_1908_10793_amd import synth
    if cfg == 1:
        return synth.cart2d_periodic(dtype="f64")
    if cfg == 2:
        return synth.shearing_box(dtype=dtype)
    if cfg == 3:
        return synth.cylindrical_disk(dtype=dtype)
    if cfg == 4:
        return synth.spherical_disk(dtype=dtype)
    return synth.batched_boxes(dtype=dtype)


def describe(cfg: int, w, arith: str) -> str:
    if cfg == 5:
        sz = ",".join(str(b["n"][0]) for b in w.boxes)
        return (f"batched: {len(w.boxes)} periodic cubes of {sz} cells per side (cell width 1/64), 4 species "
                f"(tau = 0.01, 0.1, 1, 10), U{{1..32}} particles per cell and species, "
                f"{w.n} particles, TSC, FP32 storage, {arith.upper()} push, dt = {w.dt}, feedback on")
    if cfg == 2:
        return (f"shearing box 128^3, {w.n} particles (8/cell, seeded sub-lattice), TSC, FP32 storage, "
                f"{arith.upper()} push, dt = {w.dt}, feedback on")
    if cfg == 3:
        return f"cylindrical disk 256x512x64 (log R), {w.n} particles, Stokes numbers, TSC, FP32 storage"
    if cfg == 4:
        return f"spherical disk 256x128x512, {w.n} particles, stiff stopping times, TSC, FP32 storage"
    return f"2-D periodic box 64^2, {w.n} particles, CIC, FP64"


def oracle_subset(w, cfg: int, sample: int):
    """The part of w that the oracle steps for the parity check and the CPU
    baseline: box 0 of the batch (boxes are independent), or the first
    `sample` particles of a single box (all of them on the full grid).
    Returns (workload, particle index array into w)."""
    import numpy as np
    if cfg == 5:
        bases, _ = w.cell_bases()
        n0 = int(np.searchsorted(w.cell, bases[1], side="left"))
        assert np.all(w.cell[:n0] < bases[1])
        sel = np.arange(n0)
        sub = dataclasses.replace(w, boxes=[w.boxes[0]], cell=w.cell[:n0].copy(),
                                  off=w.off[:n0].copy(), mom=w.mom[:n0].copy(),
                                  species=w.species[:n0].copy(), gas=[w.gas[0]])
        return sub, sel
    sel = np.arange(min(sample, w.n))
    sub = dataclasses.replace(
        w, cell=w.cell[sel], off=w.off[sel], mom=w.mom[sel],
        species=w.species[sel] if w.species is not None else None,
        drag=w.drag[sel] if w.drag is not None else None,
        mass=w.mass[sel] if w.mass is not None else None)
    return sub, sel


def gpu_state_of(P, F, sel_ids, nstore0, full_box: bool):
    """The GPU particles whose id is in sel_ids (sorted by id) and, for a full
    box (box 0), its deposits and gas (first nstore0 stored cells)."""
    import numpy as np
    import torch
    torch.cuda.synchronize()
    ids = P["id"]
    lo, hi = int(sel_ids[0]), int(sel_ids[-1])
    m = (ids >= lo) & (ids <= hi)
    idx = torch.nonzero(m).squeeze(1)
    order = torch.argsort(ids[idx])
    idx = idx[order]
    st = {"id": ids[idx].cpu().numpy(), "cell": P["cell"][idx].cpu().numpy().astype(np.int64),
          "off": np.stack([t[idx].cpu().numpy().astype(np.float64) for t in P["off"]], 1),
          "mom": np.stack([t[idx].cpu().numpy().astype(np.float64) for t in P["mom"]], 1)}
    if full_box:
        st["dep"] = [d[:nstore0].cpu().numpy().astype(np.float64) for d in F["dep"]]
        st["vel"] = [v[:nstore0].cpu().numpy().astype(np.float64) for v in F["vel"]]
    return st


def parity_errors(sub, run, st, full_box: bool, tol: float):
    """Worst normwise errors of the GPU state after one step against the
    oracle run from the same input (positions in host-cell widths, momenta
    against |p| + |p_start| + max |gas momentum|, deposits and fed-back gas
    per channel against their maxima)."""
    import numpy as np
    import oracle as O
    box = run.boxes[0]
    cell_o, off_o, p_o, act = run.particle_state(0)
    nd = box.ndim
    cell_g = st["cell"]
    assert np.array_equal(act, cell_g >= 0), "removed-particle sets differ"
    a = act
    x_o = run.x[0][a]
    lo = 0
    x_g = O.to_global(box, cell_g[a] - lo, st["off"][a])
    dx = x_g - x_o
    idx = O.unravel(box, cell_o[a])
    ex = 0.0
    for d in range(nd):
        c, wd = O.centers_widths(box, d)
        if box.bc_lo[d] in ("periodic", "shear"):
            L = box.faces[d][-1] - box.faces[d][0]
            dx[:, d] = (dx[:, d] + 0.5 * L) % L - 0.5 * L
        ex = max(ex, float(np.abs(dx[:, d] / wd[idx[d]]).max()))
    nc = nd if box.geom == "cart" else 3
    p0 = np.asarray(sub.mom, dtype=np.float64)[a][:, :nc]
    gmax = max(float(np.abs(np.asarray(v)).max()) for v in sub.gas[0]["vel"][:nc])
    sc = np.ones((a.sum(), 3))
    if box.geom == "cyl":
        sc[:, 1] = x_o[:, 0]
    elif box.geom == "sph":
        sc[:, 1] = x_o[:, 0]
        sc[:, 2] = x_o[:, 0] * np.sin(x_o[:, 1])
    scale = np.abs(p_o[a][:, :nc]).max(1) + np.abs(p0).max(1) + gmax * sc[:, :nc].max(1) + 1e-300
    emom = float((np.abs(st["mom"][a][:, :nc] - p_o[a][:, :nc]).max(1) / scale).max())
    cells_diff = int((cell_g[a] != cell_o[a]).sum())
    out = {"pos": ex, "mom": emom, "cell_mismatch": cells_diff}
    if full_box:
        fo = run.fields[0]
        edep = 0.0
        for c in range(nc + 1):
            ref = fo.dep[c].reshape(-1)
            den = np.abs(ref).max()
            if den > 0:
                edep = max(edep, float(np.abs(st["dep"][c] - ref).max() / den))
        evel = 0.0
        # active cells (a missing axis of a 2-D box has extent 1 and no ghosts)
        act_sl = tuple(slice(1, -1) if g > 1 else slice(None) for g in box.ghosted_shape)
        for c in range(nc):
            ref = fo.vel[c].reshape(box.ghosted_shape)[act_sl]
            got = st["vel"][c].reshape(box.ghosted_shape)[act_sl]
            evel = max(evel, float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)))
        out["dep"] = edep
        out["vel"] = evel
    out["worst"] = max(v for k, v in out.items() if k != "cell_mismatch")
    out["tol"] = tol
    out["pass"] = out["worst"] <= tol
    return out


def check_step(ctx, dust, w, cfg, P, F, flags, t, sample, time_oracle: bool):
    """One GPU step (flags) from the current state against the FP64 oracle on
    the subset the oracle steps.  Returns (parity dict, cpu baseline dict)."""
    import numpy as np
    from oracle.run import OracleRun
    sub, sel = oracle_subset(w, cfg, sample)
    full_box = cfg == 5 or len(sel) == w.n
    nstore0 = int(np.prod([b + 2 for b in w.boxes[0]["n"][:w.boxes[0]["ndim"]]]))
    ctx.step(P, F, w.dt, dust.forces_for(w, t), 1, flags)
    st = gpu_state_of(P, F, sel, nstore0, full_box)
    run = OracleRun(dataclasses.replace(sub, t0=t))
    t0 = time.perf_counter()
    run.step(1)
    t_one = time.perf_counter() - t0
    # the oracle steps the sample with the gas of the whole grid; with a
    # particle sample the deposits cover only part of the particles
    par = parity_errors(sub, run, st, full_box, 1e-12 if w.dtype == "f64" else 1e-5)
    cpu = None
    if time_oracle:
        run_t = OracleRun(dataclasses.replace(sub, t0=t))
        t0 = time.perf_counter()
        run_t.step(1, threads=True)
        t_thr = time.perf_counter() - t0
        nthr = run_t.diags[-1][0].threads
        what = ("box 0 (32^3, every particle)" if cfg == 5 else
                f"the first {len(sel)} of the {w.n} particles on the full grid")
        cpu = {"value": len(sel) / t_one, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
               "sample": f"1 step of {what} ({len(sel)} particles, serial FP64 C oracle, "
                         f"{t_one:.1f} s)",
               "threads": {"value": len(sel) / t_thr, "cores": nthr,
                           "sample": f"the same step with the OpenMP variant on {nthr} threads "
                                     f"({t_thr:.2f} s)"},
               **host_info()}
    return par, cpu


def _tensors(d):
    """The tensors of a particles or fields dict, in key order."""
    out = []
    for k in sorted(d):
        v = d[k]
        out.extend(v if isinstance(v, list) else [v])
    return out


def _clone(d):
    return {k: ([x.clone() for x in v] if isinstance(v, list) else v.clone()) for k, v in d.items()}


def curvilinear(args, W):
    """The cylindrical (256x512x64, 2^25 particles) and spherical
    (256x128x512, 2^26) disks with FP64 per-particle arithmetic and with the
    default FP32 one (FP32 storage both): time per step and one step's
    parity against the oracle on a particle sample.  Fixed tile shape and
    rebinning interval (the autotuner's picks at full size), 10 timed
    steps."""
    import copy
    res = {}
    for cfg, tile, rebin in ((3, "4,16,4,0", 3), (4, "4,16,4,0", 2)):
        a2 = copy.copy(args)
        a2.no_tune, a2.tile, a2.rebin_every, a2.reps, a2.eager = True, tile, rebin, 3, True
        row = {}
        for arith in ("f64", "f32"):
            r, w = run_config(cfg, a2, extra=True, K=10, W=W, arith_override=arith)
            row[arith + "_arith"] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                                     "roofline_frac": r["roofline"]["frac"] if r["roofline"] else None,
                                     "parity_worst": r["parity"]["worst"] if r["parity"] else None,
                                     "parity_pass": r["parity"]["pass"] if r["parity"] else None}
            del w
        row["workload"] = WORKLOAD_NAMES[cfg]
        row["tile"], row["rebin_every"] = tile, rebin
        row["fp64_over_fp32_time"] = round(row["f64_arith"]["ms_per_step"] / row["f32_arith"]["ms_per_step"], 3)
        res[WORKLOAD_NAMES[cfg]] = row
    return res


def timed_kernel(ctx, fn, K, stream):
    """Average time of K calls of fn() (HIP events on the launch stream)."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(K):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / K


def run_config(cfg: int, args, extra: bool, K: int, W: int, arith_override=None):
    import numpy as np
    import torch
    from paper_1908_10793_amd import dust

    dtype = "f64" if cfg == 1 else "f32"
    t_gen = time.perf_counter()
    w = make_workload(cfg, dtype)
    log(f"config {cfg}: {w.n} particles generated in {time.perf_counter() - t_gen:.1f} s")
    N = w.n
    C = sum(int(np.prod(b["n"][:b["ndim"]])) for b in w.boxes)
    ctx = dust.context_for(w)
    arith = arith_override or args.arith or "f32"
    if dtype == "f32":
        ctx.set_arith(arith)
    tx, ty, tz, slack = (int(v) for v in args.tile.split(","))
    if cfg == 1 and args.tile == "8,8,4,0":
        tx, ty, tz = 16, 16, 1
    ctx.set_tile(tx, ty, tz, slack)
    check = not args.no_check
    P, F = dust.upload(w, ctx, with_id=check)
    torch.cuda.synchronize()
    log(f"uploaded ({torch.cuda.memory_allocated() / 2**30:.1f} GiB on the device)")
    flags = dust.STEP_APPLY_FEEDBACK | dust.STEP_DIAG | dust.STEP_FUSED
    tuned = None
    if args.no_tune:
        flags |= dust.STEP_REBIN_EVERY(args.rebin_every)
        rebin = args.rebin_every
    else:
        t0 = time.perf_counter()
        tuned = ctx.autotune(P, F, w.dt, dust.forces_for(w, 0.0), dust.STEP_APPLY_FEEDBACK | dust.STEP_DIAG,
                             steps=args.tune_steps)
        (tx, ty, tz), rebin = tuned["tile"], tuned["rebin_every"]
        log(f"autotuned in {time.perf_counter() - t0:.1f} s: {tuned}")
    t = 0.0
    out = {}
    # one step against the FP64 oracle (the first warm-up step)
    parity, cpu = None, None
    if check:
        parity, cpu = check_step(ctx, dust, w, cfg, P, F, flags, t, args.cpu_sample,
                                 time_oracle=not args.no_cpu_baseline and not extra)
        t += w.dt
        log(f"parity: {parity}")
        del P["id"]
        torch.cuda.empty_cache()
    if not check:
        # the first step: it also moves the particles from their generated
        # order into the library's binned layout
        ctx.step(P, F, w.dt, dust.forces_for(w, t), 1, flags)
        t += w.dt
    # the state every timed repetition starts from: after the first step, in
    # the layout the library keeps between calls
    P0, F0, t_start = _clone(P), _clone(F), t
    ctx.status()
    nw = max(W - 1, 0)
    if nw:
        ctx.step(P, F, w.dt, dust.forces_for(w, t), nw, flags)
        t += nw * w.dt
    torch.cuda.synchronize()
    ctx.status()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def restore():
        # every timed repetition starts from the same state, one step after
        # the generated one: the gas evolves only through the feedback, so
        # dust collects where its frozen velocity field converges and the
        # per-cell counts (the load of the tile kernel) would drift away from
        # the stated distribution over hundreds of steps
        nonlocal t
        for a, b in zip(_tensors(P), _tensors(P0)):
            a.copy_(b)
        for a, b in zip(_tensors(F), _tensors(F0)):
            a.copy_(b)
        t = t_start

    def timed(fl, profile: bool):
        nonlocal t
        times, kern = [], []
        for r in range(max(args.reps, 1)):
            restore()
            torch.cuda.synchronize()
            e0.record(stream)
            ctx.step(P, F, w.dt, dust.forces_for(w, t), K, fl)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
            if profile:
                kern.extend(ctx.profile(K))
            t += K * w.dt
            log(f"{'graph' if fl & dust.STEP_GRAPH else 'eager'} rep {r}: {times[-1] / K:.3f} ms/step")
        return times, kern

    # timed region: K steps launched from the host, each fused-kernel launch
    # bracketed by HIP events on the library's stream (events recorded inside
    # a captured graph cannot be timed on this runtime)
    ctx.set_profile(K)
    reps, kern = timed(flags, True)
    diag = ctx.status()
    ctx.set_profile(0)
    graph = None
    if not args.eager:
        gflags = flags | dust.STEP_GRAPH
        ctx.step(P, F, w.dt, dust.forces_for(w, t), K, gflags)   # capture (and run)
        t += K * w.dt
        torch.cuda.synchronize()
        ctx.status()
        greps, _ = timed(gflags, False)
        ctx.status()
        gms = float(np.median(greps))
        graph = {"value": N * K / (gms * 1e-3), "ms_per_step": gms / K,
                 "reps_ms": [round(x, 3) for x in greps]}
    ms = float(np.median(reps))
    value = N * K / (ms * 1e-3)
    ppc = N / C
    real = 8 if dtype == "f64" else 4
    state = 4 + 2 * 2 * real if cfg == 1 else 4 + 6 * real      # cell + offsets + momenta
    per_p = 2.0 * state + (4.0 if cfg in (3, 4) else 0.0)       # read + write (+ per-particle drag)
    per_cell = (4 + 8) * real if cfg != 1 else (3 + 6) * real    # gas rho + v read, deposit RMW
    bytes_per_pstep = per_p + per_cell / ppc
    roof = None
    if kern:
        kavg = float(np.mean(kern)) * 1e-3
        achieved = bytes_per_pstep * N / kavg / 1e9
        khash = source_hash()
        kname = tile_kernel(cfg, dtype, arith)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": counter_traffic(kname, WORKLOAD_NAMES[cfg], khash, N, (tx, ty, tz), rebin),
                "kernel": kname, "kernel_avg_us": round(kavg * 1e6, 2),
                "launches_timed": len(kern),
                "bytes_per_particle_step": round(bytes_per_pstep, 3),
                "algorithmic_bytes_per_launch": bytes_per_pstep * N, "kernel_source_hash": khash,
                "step_frac": round(bytes_per_pstep * value / 1e9 / HBM_PEAK_GBS, 4)}
        valu = counter_valu(kname, WORKLOAD_NAMES[cfg], khash, (tx, ty, tz), rebin)
        if valu:
            # non-packed FP32 VALU issue: one wave64 instruction per SIMD every
            # 4 cycles, 4 SIMDs per CU
            issue_s = valu * 4.0 / (CU_COUNT * 4 * CLOCK_HZ)
            roof["valu_issue"] = {"wave_instructions_per_launch": valu, "issue_ms": round(issue_s * 1e3, 3),
                                  "frac": round(issue_s / kavg, 4),
                                  "note": "SQ_INSTS_VALU from the committed counter summary of this tiling"}
    res = float(np.max(np.abs(np.array(diag["p_part"]) + np.array(diag["p_grid"])))) / max(
        diag["sum_abs_j"], 1e-300)
    out.update({
        "value": value, "ms_per_step": ms / K,
        "config": {"workload": describe(cfg, w, arith), "n_particles": N, "active_cells": C,
                   "boxes": [list(b["n"][:b["ndim"]]) for b in w.boxes],
                   "tile": [tx, ty, tz], "rebin_every": rebin, "autotuned": tuned,
                   "timed_loop": "eager (graph replay under timing.graph)", "steps_per_call": K,
                   "storage": dtype,
                   "push_arith": arith if dtype == "f32" else "f64",
                   "deposit_accum": "per-cell register sums, FP64 LDS tile window, HBM atomics"},
        "roofline": roof,
        "timing": {"reps_ms": [round(x, 3) for x in reps], "median_ms": ms,
                   "min_ms": float(np.min(reps)), "graph": graph},
        "parity": parity,
        "diag": {"momentum_residual": res, "max_cells_per_step": diag["max_cells_per_step"],
                 "n_fallback": diag["n_fallback"], "flags": diag["flag_names"], "steps": diag["steps"]},
    })
    if cpu:
        out["cpu_baseline"] = cpu
    if not args.no_extra:
        Kx = max(1, min(K, 10))
        fr = dust.forces_for(w, t)
        ds_s = timed_kernel(ctx, lambda: ctx.drag_source(P, F, w.dt, fr), Kx, stream)
        sp = 1.0 if "species" in P else 0.0
        ds_bytes = (4 + 6 * real + sp + (4 * real if w.drag is not None else 0) +
                    (4 + 3) * real / ppc) * N
        tiled = tile_kernel(cfg, dtype, arith) == "k_c3"   # the binned-layout kernel
        out["drag_source"] = {"kernel": "k_c3_aux" if tiled else "k_drag_source", "us_per_launch": round(ds_s * 1e6, 2),
                              "algorithmic_bytes_per_launch": ds_bytes,
                              "achieved": round(ds_bytes / ds_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": round(ds_bytes / ds_s / 1e9 / HBM_PEAK_GBS, 4)}
        rho_d = torch.zeros_like(F["rho"])
        md_s = timed_kernel(ctx, lambda: ctx.deposit_mass(P, rho_d), Kx, stream)
        md_bytes = (4 + 3 * real + sp + 2 * real / ppc) * N
        out["mass_density"] = {"kernel": "k_c3_aux" if tiled else "k_mass_density", "us_per_launch": round(md_s * 1e6, 2),
                               "algorithmic_bytes_per_launch": md_bytes,
                               "achieved": round(md_bytes / md_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": round(md_bytes / md_s / 1e9 / HBM_PEAK_GBS, 4)}
        del rho_d
        log(f"drag source {ds_s * 1e3:.2f} ms, dust density {md_s * 1e3:.2f} ms")
    ctx.close()
    del P, F, ctx
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if dtype == "f32" and not args.no_fp64 and not extra:
        out["fp64_plain"] = fp64_plain(w, cfg, args, K)
        if out["fp64_plain"]:
            out["fp64_plain"]["speedup_of_fp32_fused"] = round(
                out["fp64_plain"]["ms_per_step"] / (ms / K), 2)
    return out, w


def fp64_plain(w, cfg, args, K):
    """The plain FP64 GPU step: FP64 storage and arithmetic, the unfused
    per-phase chain (drift, gather, kick, deposit, drift, one thread per
    particle, HBM atomics), on the same inputs widened exactly; one step
    checked against the oracle at the FP64 bar, then a few steps timed."""
    import torch
    from paper_1908_10793_amd import dust
    w64 = dataclasses.replace(w, dtype="f64")
    ctx = dust.context_for(w64)
    check = not args.no_check
    P, F = dust.upload(w64, ctx, with_id=check)
    flags = dust.STEP_APPLY_FEEDBACK | dust.STEP_DIAG
    t = 0.0
    par = None
    if check:
        par, _ = check_step(ctx, dust, w64, cfg, P, F, flags, t, args.cpu_sample, time_oracle=False)
        t += w.dt
        log(f"fp64 plain parity: {par}")
        del P["id"]
        torch.cuda.empty_cache()
    K64 = max(1, min(K, 3))
    ctx.step(P, F, w.dt, dust.forces_for(w, t), 1, flags)
    t += w.dt
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    ctx.step(P, F, w.dt, dust.forces_for(w, t), K64, flags)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / K64
    log(f"fp64 plain: {ms:.2f} ms/step")
    ctx.close()
    del P, F, ctx
    torch.cuda.empty_cache()
    return {"value": w.n / (ms * 1e-3), "ms_per_step": ms, "steps_timed": K64,
            "what": "unfused per-phase chain, FP64 storage and arithmetic, same inputs",
            "parity": par}


def copy_bandwidth():
    """Measured device-to-device copy bandwidth (read + write bytes)."""
    import torch
    nel = 256 << 20
    src = torch.ones(nel, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    for _ in range(5):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    gbs = 2.0 * 4 * nel * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def main():
    args = parse()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace[0], args.summarize_trace[1], args.command)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, args.command, args.n_particles,
                           args.calib_copy_mb)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "the benchmark needs a GPU"
    K, W = args.steps, args.warmup
    res, w = run_config(args.config, args, extra=False, K=K, W=W)
    del w
    copy_gbs = copy_bandwidth()
    if res.get("roofline"):
        res["roofline"]["copy_gbs"] = round(copy_gbs, 1)
        res["roofline"]["frac_of_copy"] = round(res["roofline"]["achieved"] / copy_gbs, 4)
    out = {"metric": METRIC, "value": res["value"], "unit": "particle-steps/s", "n_gpus": 1,
           "steps": K, "warmup": W, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": res["config"]["push_arith"], "data": "synthetic"}
    out.update({k: v for k, v in res.items() if k not in ("value", "ms_per_step")})
    if args.config == 5 and not args.no_extra:
        r2, w2 = run_config(2, args, extra=True, K=min(K, 20), W=W)
        del w2
        out["config2"] = {"value": r2["value"], "ms_per_step": r2["ms_per_step"],
                          "workload": r2["config"]["workload"], "tile": r2["config"]["tile"],
                          "rebin_every": r2["config"]["rebin_every"], "roofline": r2["roofline"],
                          "parity": r2["parity"], "diag": r2["diag"],
                          "drag_source": r2.get("drag_source"), "mass_density": r2.get("mass_density")}
    if args.config == 5 and not args.no_extra and not args.no_curvilinear:
        out["curvilinear"] = curvilinear(args, W)
    if args.calib_copy_mb > 0:
        nel = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
