"""Parity at full size, in the launch configuration that bench.py times
(the autotuned or the bench's fixed tiling of each workload), on sampled
outputs.

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


def sample_regions(w, ncenters, margin, seed):
    """Per box: `near` (cells within margin of a sampled interior cell; the
    particles of these cells are stepped by the oracle) and `core` (cells
    within margin - 2, where deposits and fed-back gas are exact)."""
    rng = np.random.default_rng(seed)
    out = []
    for bd in w.boxes:
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
        out.append((near, core))
    return out


def check_fields(w, run, dep_g, vel_g, regions, label):
    """Deposits and fed-back gas of the GPU (flat ghosted arrays, boxes
    concatenated) against the oracle on the core cells of every box."""
    tol = TOL["f32"]
    store = 0
    worst = 0.0
    for b, bd in enumerate(w.boxes):
        nd = bd["ndim"]
        g = [bd["n"][d] + 2 if d < nd else 1 for d in range(3)]
        sz = g[0] * g[1] * g[2]
        shp = (g[2], g[1], g[0])
        core = regions[b][1]
        inner = (slice(1, -1),) * 3 if nd == 3 else (slice(0, 1), slice(1, -1), slice(1, -1))
        fo = run.fields[b]
        for c in range(len(dep_g)):
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
    return worst


def sampled_parity(w, ncenters=24, margin=3, seed=11, tune=True, tile=None, label=""):
    from paper_1908_10793_amd import dust
    print(f"[fullsize] {label}: {w.n} particles, uploading", flush=True)
    ctx = dust.context_for(w)
    if tile:
        ctx.set_tile(*tile)
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

    regions = sample_regions(w, ncenters, margin, seed)
    bases, _ = w.cell_bases()
    cell0 = np.asarray(w.cell).astype(np.int64)
    sel_all = []
    for b, bd in enumerate(w.boxes):
        local = cell0 - bases[b]
        inb = (local >= 0) & (local < _box_cells(bd))
        sel_b = np.nonzero(inb)[0]
        sel_b = sel_b[regions[b][0].ravel()[local[sel_b]]]
        sel_all.append(sel_b)
    sel = np.concatenate(sel_all)
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
    rep["fields"] = check_fields(w, run, dep_g, vel_g, regions, label)
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


def test_full_size_cylindrical_disk():
    """Cylindrical (R, phi, z) 256x512x64 grid, log-spaced R in [0.4, 2.5],
    2^25 particles with surface density ~ 1/R and Stokes numbers
    log-uniform in [1e-3, 10], TSC with the curvilinear weights, FP32
    storage and arithmetic: one fused step with the bench's tiling of this
    workload (4x16x4; App. B.2 cylindrical step)."""
    sampled_parity(synth.cylindrical_disk(), ncenters=16, tune=False, tile=(4, 16, 4, 0),
                   label="cylindrical 256x512x64")


def test_full_size_spherical_disk():
    """Spherical (r, theta, phi) 256x128x512 grid, r in [0.5, 5], theta in
    pi/2 +- 0.3, 2^26 particles, stopping times log-uniform in [1e-6, 1]:
    one fused step in FP32 arithmetic with the bench's tiling of this
    workload (4x16x4; App. B.2 spherical step, App. C weights)."""
    sampled_parity(synth.spherical_disk(), ncenters=16, tune=False, tile=(4, 16, 4, 0),
                   label="spherical 256x128x512")


def last_step_parity(w, tile, rebin_every, nsteps, ncenters, margin, seed, label):
    """nsteps fused steps through captured graphs (nsteps-1, then the last
    one) with the given tiling and rebinning interval; the last step against
    the oracle started from the GPU state before it, on the particles within
    `margin` cells of sampled cells of every box (selected on the GPU by
    cell), and the conservation residual over all steps."""
    from paper_1908_10793_amd import dust
    print(f"[fullsize] {label}: {w.n} particles, uploading", flush=True)
    ctx = dust.context_for(w)
    ctx.set_tile(*tile)
    P, F = dust.upload(w, ctx, with_id=True)
    flags = (dust.STEP_APPLY_FEEDBACK | dust.STEP_DIAG | dust.STEP_FUSED | dust.STEP_GRAPH
             | dust.STEP_REBIN_EVERY(rebin_every))
    t = w.t0
    ctx.step(P, F, w.dt, dust.forces_for(w, t), nsteps - 1, flags)
    t += (nsteps - 1) * w.dt
    torch.cuda.synchronize()
    diag_a = ctx.status()
    print(f"[fullsize] {label}: {nsteps - 1} graph steps done", flush=True)

    # the state before the last step: gas of every box, and the particles of
    # the sampled regions (chosen on the GPU by their cell)
    regions = sample_regions(w, ncenters, margin, seed=seed)
    bases, C = w.cell_bases()
    near_all = torch.from_numpy(np.concatenate([r[0].ravel() for r in regions])).cuda()
    cell = P["cell"]
    pick = (cell >= 0) & near_all[cell.clamp(min=0).long()]
    pos = pick.nonzero().squeeze(1)
    ids = P["id"][pos].cpu().numpy()
    st_in = {"cell": cell[pos].cpu().numpy().astype(np.int64),
             "off": torch.stack([o[pos] for o in P["off"]], 1).cpu().numpy().astype(np.float64),
             "mom": torch.stack([m[pos] for m in P["mom"]], 1).cpu().numpy().astype(np.float64),
             "species": P["species"][pos].cpu().numpy(), "drag": None, "mass": None,
             "id": np.arange(len(pos))}
    gas = []
    base = 0
    for bd in w.boxes:
        g = [bd["n"][d] + 2 for d in range(3)]
        sz = g[0] * g[1] * g[2]
        shp = (g[2], g[1], g[0])
        gas.append(dict(rho=F["rho"][base:base + sz].cpu().numpy().reshape(shp).astype(np.float64),
                        vel=[v[base:base + sz].cpu().numpy().reshape(shp).astype(np.float64)
                             for v in F["vel"]]))
        base += sz
    st_in["gas"] = gas
    print(f"[fullsize] {label}: {len(pos)} particles sampled", flush=True)

    # the last step, and the sampled particles after it (found by id)
    ctx.step(P, F, w.dt, dust.forces_for(w, t), 1, flags)
    torch.cuda.synchronize()
    diag1 = ctx.status()
    want = torch.full((w.n,), -1, dtype=torch.int64, device="cuda")
    want[torch.from_numpy(ids).cuda().long()] = torch.arange(len(ids), device="cuda")
    slot_of = want[P["id"].long()]
    at = (slot_of >= 0).nonzero().squeeze(1)
    order = torch.empty(len(ids), dtype=torch.int64, device="cuda")
    order[slot_of[at]] = at
    st_out = {"cell": P["cell"][order].cpu().numpy().astype(np.int64),
              "off": torch.stack([o[order] for o in P["off"]], 1).cpu().numpy().astype(np.float64),
              "mom": torch.stack([m[order] for m in P["mom"]], 1).cpu().numpy().astype(np.float64),
              "id": np.arange(len(ids))}
    dep_g = [d.cpu().numpy().astype(np.float64) for d in F["dep"]]
    vel_g = [v.cpu().numpy().astype(np.float64) for v in F["vel"]]

    for dg in (diag_a, diag1):
        res_m = np.abs(np.array(dg["p_part"]) + np.array(dg["p_grid"])).max() / dg["sum_abs_j"]
        assert res_m < 2e-6, res_m
    assert diag_a["steps"] == nsteps - 1 and diag1["steps"] == 1 and not diag_a["flag_names"]

    sub = dataclasses.replace(w, cell=st_in["cell"].astype(np.int32), off=st_in["off"],
                              mom=st_in["mom"], species=st_in["species"], gas=gas, t0=t)
    print(f"[fullsize] {label}: oracle on {len(ids)} particles", flush=True)
    run = OracleRun(sub)
    run.step(1)
    rep = compare_step(sub, st_in, st_out, run, "f32", fields_too=False, label=label)
    rep["fields"] = check_fields(w, run, dep_g, vel_g, regions, label)
    print(f"[fullsize] {label}: {rep}", flush=True)


def test_full_size_batched_boxes_100_step_graph():
    """All eight boxes of the batched workload at full size (32^3 ... 192^3,
    four species, U{1..32} per cell and species, 994,755,343 particles),
    stepped 100 times through captured graphs (99 steps, then the last one),
    with the tile shape and rebinning interval the bench's autotuner picks
    (16x4x4, every 32 steps).  The last step is checked against the oracle
    started from the GPU state before it, on the particles within `margin`
    cells of sampled cells of every box (selected on the GPU by cell), and
    the conservation residual is checked over all 100 steps."""
    last_step_parity(synth.batched_boxes(), (16, 4, 4, 0), 32, 100, 6, 3, 13, "batched, all boxes")


def test_full_size_box_of_2_24_cells_stale_bins():
    """One periodic box of 256^3 = 2^24 cells (one species, one particle per
    cell): the tile kernel's path for boxes of 2^24 cells or more (FP64 cell
    division, 32-bit cell-id products), six steps rebinned every four, so
    that the checked last step runs on stale bins."""
    w = synth.batched_boxes(sizes=(256,), max_per_species=1, species_tau=(0.1,))
    last_step_parity(w, (16, 4, 4, 0), 4, 6, 8, 3, 17, "box of 256^3 cells")
