"""Parity at full size, in the launch configuration that bench.py times
(autotuned fused step), on sampled outputs.

The GPU steps the whole workload.  The oracle then steps only the particles
whose cells lie within `margin` cells of a set of sampled interior cells;
this is exact for those particles and, since a particle deposits at most two
cells away from its cell (stencil +-1 plus a half drift below one cell), for
the deposits and the fed-back gas of every cell within margin - 2 cells of a
sampled cell.  Particles are followed by id.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

from oracle.run import OracleRun
from paper_1908_10793_amd import synth

from gpu_common import TOL, compare_step

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")


def _box_cells(bd):
    n = bd["n"]
    return n[0] * n[1] * (n[2] if bd["ndim"] > 2 else 1)


def sampled_parity(w, ncenters=24, margin=3, seed=11, tune=True, label=""):
    from paper_1908_10793_amd import dust
    print(f"[fullsize] {label}: {w.n} particles, uploading", flush=True)
    ctx = dust.context_for(w)
    P, F = dust.upload(w, ctx)
    flags = dust.STEP_APPLY_FEEDBACK | dust.STEP_DIAG
    fr = dust.forces_for(w, w.t0)
    if tune:
        res = ctx.autotune(P, F, w.dt, fr, flags, steps=4)
        print(f"[fullsize] {label}: autotuned {res}", flush=True)
    ctx.step(P, F, w.dt, fr, 1, flags | dust.STEP_FUSED)
    torch.cuda.synchronize()
    diag = ctx.status()
    res_m = np.abs(np.array(diag["p_part"]) + np.array(diag["p_grid"])).max() / diag["sum_abs_j"]
    assert res_m < 2e-6, res_m
    order = np.argsort(P["id"].cpu().numpy())
    cell_g = P["cell"].cpu().numpy()[order].astype(np.int64)
    off_g = np.zeros((w.n, 3))
    mom_g = np.zeros((w.n, 3))
    for d, t in enumerate(P["off"]):
        off_g[:, d] = t.cpu().numpy()[order]
    for d, t in enumerate(P["mom"]):
        mom_g[:, d] = t.cpu().numpy()[order]
    dep_g = [t.cpu().numpy().astype(np.float64) for t in F["dep"]]
    vel_g = [t.cpu().numpy().astype(np.float64) for t in F["vel"]]
    print(f"[fullsize] {label}: GPU step done, sampling", flush=True)

    rng = np.random.default_rng(seed)
    bases, _ = w.cell_bases()
    cell0 = np.asarray(w.cell).astype(np.int64)
    sel_all, checks = [], []
    for b, bd in enumerate(w.boxes):
        n, nd = bd["n"], bd["ndim"]
        ext = [n[d] if d < nd else 1 for d in range(3)]
        lo = [margin if d < nd else 0 for d in range(3)]
        hi = [ext[d] - margin if d < nd else 1 for d in range(3)]
        centers = np.stack([rng.integers(lo[d], hi[d], size=ncenters) for d in range(3)], axis=1)
        near = np.zeros(ext[::-1], dtype=bool)        # (k, j, i)
        core = np.zeros(ext[::-1], dtype=bool)
        r2 = margin - 2
        for c in centers:
            sl = tuple(slice(max(c[d] - margin, 0), c[d] + margin + 1) if d < nd else slice(0, 1)
                       for d in (2, 1, 0))
            near[sl] = True
            sl = tuple(slice(c[d] - r2, c[d] + r2 + 1) if d < nd else slice(0, 1) for d in (2, 1, 0))
            core[sl] = True
        local = cell0 - bases[b]
        inb = (local >= 0) & (local < _box_cells(bd))
        sel_b = np.nonzero(inb)[0]
        sel_b = sel_b[near.ravel()[local[sel_b]]]
        sel_all.append(sel_b)
        checks.append((b, core))
    sel = np.concatenate(sel_all)
    # boxes with no sampled particles are dropped from the sub-workload
    keep = [b for b in range(len(w.boxes)) if len(sel_all[b])]
    sub = dataclasses.replace(
        w, cell=w.cell[sel], off=w.off[sel], mom=w.mom[sel],
        species=w.species[sel] if w.species is not None else None,
        drag=w.drag[sel] if w.drag is not None else None,
        mass=w.mass[sel] if w.mass is not None else None)
    print(f"[fullsize] {label}: oracle on {len(sel)} particles", flush=True)
    run = OracleRun(sub)
    run.step(1)
    st_in = {"cell": np.asarray(sub.cell).astype(np.int64), "off": np.asarray(sub.off, np.float64),
             "mom": np.asarray(sub.mom, np.float64), "id": np.arange(len(sel)),
             "drag": None, "mass": None, "species": None, "gas": w.gas}
    st_out = {"cell": cell_g[sel], "off": off_g[sel], "mom": mom_g[sel], "id": np.arange(len(sel))}
    rep = compare_step(sub, st_in, st_out, run, "f32", fields_too=False, label=label)
    # deposits and fed-back gas on the core cells of each box
    tol = TOL["f32"]
    store = 0
    worst = 0.0
    for b, bd in enumerate(w.boxes):
        nd = bd["ndim"]
        g = [bd["n"][d] + 2 if d < nd else 1 for d in range(3)]
        sz = g[0] * g[1] * g[2]
        shp = (g[2], g[1], g[0])
        core = checks[b][1]
        inner = (slice(1, -1),) * 3 if nd == 3 else (slice(0, 1), slice(1, -1), slice(1, -1))
        fo = run.fields[b]
        for c in range(len(F["dep"])):
            if c >= fo.nc + 1:
                continue
            got = dep_g[c][store:store + sz].reshape(shp)[inner][core]
            ref = fo.dep[c].reshape(shp)[inner][core]
            den = np.abs(ref).max()
            if den == 0:
                continue
            e = np.abs(got - ref).max() / den
            worst = max(worst, e)
            assert e <= tol, (label, "dep", b, c, e)
        if w.apply_feedback:
            for c in range(fo.nc):
                got = vel_g[c][store:store + sz].reshape(shp)[inner][core]
                ref = fo.vel[c].reshape(shp)[inner][core]
                e = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
                worst = max(worst, e)
                assert e <= tol, (label, "vel", b, c, e)
        store += sz
    rep["fields"] = worst
    print(f"[fullsize] {label}: {rep}", flush=True)
    return rep


def test_full_size_shearing_box():
    """128^3 standard shearing box, 2^24 particles, TSC, FP32 (the bench
    workload), one autotuned fused step."""
    sampled_parity(synth.shearing_box(), label="shearing_box 128^3")


def test_full_size_batched_boxes_subset():
    """Two boxes of the batched workload at their full sizes (32^3 and 64^3,
    four species, U{1..32} per cell and species); boxes are independent, so
    this is exact for them."""
    sampled_parity(synth.batched_boxes(sizes=(32, 64)), label="batched 32^3+64^3")
