"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
the FP64 oracle on the same inputs, and compare them element by element.

Tolerances (reading of the "1e-5 relative (FP32) / 1e-12 (FP64)" bar,
normwise so that it is well posed where values cancel):
  positions  |x_gpu - x_oracle| / width_of_host_cell <= tol
  momenta    |p_gpu - p_oracle|_inf <= tol (|p_oracle| + |p_start| + |p_gas|), the
             last term the largest canonical gas momentum in the particle's
             neighbourhood (the kick is a weighted mean of p, p_gas and the
             external acceleration, so this is its natural scale)
  fields     max_i |f_gpu - f_oracle| <= tol max_i |f_oracle|, per channel
  cells      identical, except for particles whose oracle position lies within
             tol cell widths of a face (counted, and they must then agree in
             position as above).
Every comparison starts from identical inputs: multi-step runs are checked
step by step along the GPU trajectory (the oracle restarts each step from the
GPU's state), so FP32 rounding of the stored state is not compounded against
an FP64 trajectory.
"""
from __future__ import annotations

import copy
import dataclasses

import numpy as np
from scipy.ndimage import maximum_filter

import oracle as O
from oracle.run import OracleRun, locate_cells

TOL = {"f64": 1e-12, "f32": 1e-5}


def download(ctx, P, F, w):
    """GPU state -> numpy (particles ordered as stored; gas per box)."""
    import torch
    torch.cuda.synchronize()
    n = P["cell"].numel()
    st = {"cell": P["cell"].cpu().numpy().astype(np.int64)}
    off = np.zeros((n, 3))
    mom = np.zeros((n, 3))
    for d, t in enumerate(P["off"]):
        off[:, d] = t.cpu().numpy()
    for d, t in enumerate(P["mom"]):
        mom[:, d] = t.cpu().numpy()
    st["off"], st["mom"] = off, mom
    for k in ("drag", "mass", "species", "id"):
        st[k] = P[k].cpu().numpy() if k in P else None
    gas, dep = [], []
    base = 0
    for bd in w.boxes:
        nd = bd["ndim"]
        g = [bd["n"][d] + 2 if d < nd else 1 for d in range(3)]
        sz = g[0] * g[1] * g[2]
        shp = (g[2], g[1], g[0]) if nd == 3 else (g[1], g[0])
        gas.append(dict(rho=F["rho"][base:base + sz].cpu().numpy().reshape(shp).astype(np.float64),
                        vel=[v[base:base + sz].cpu().numpy().reshape(shp).astype(np.float64)
                             for v in F["vel"]]))
        dep.append([dd[base:base + sz].cpu().numpy().reshape(shp).astype(np.float64)
                    for dd in F["dep"]])
        base += sz
    st["gas"], st["dep"] = gas, dep
    return st


def workload_from_state(w, st, t):
    """A copy of workload w whose inputs are the state st (exact widening)."""
    w2 = copy.copy(w)
    w2 = dataclasses.replace(w, cell=st["cell"].astype(np.int32), off=st["off"], mom=st["mom"],
                             gas=st["gas"], t0=t,
                             drag=st["drag"] if st["drag"] is not None else None,
                             mass=st["mass"] if st["mass"] is not None else None,
                             species=st["species"] if st["species"] is not None else None)
    return w2


def _global_positions(box, cell_local, off):
    x = np.full((len(cell_local), 3), np.nan)
    ok = cell_local >= 0
    if ok.any():
        x[ok] = O.to_global(box, cell_local[ok], off[ok])
    return x


def oracle_diag(run: OracleRun, steps=1):
    """The oracle's FP64 diagnostics of its last `steps` steps, summed over
    boxes (maxima for the displacement bound), with the scale of the
    energy sums: the largest physical particle speed times sum |J| over the
    smallest canonical factor (a bound of sum |e_p|)."""
    out = dict(p_part=np.zeros(3), p_grid=np.zeros(3), e_part=0.0, e_grid=0.0, sum_abs_j=0.0,
               max_cells_per_step=0.0, n_removed=0)
    for ds in run.diags[-steps:]:
        for d in ds:
            out["p_part"] = out["p_part"] + d.p_part
            out["p_grid"] = out["p_grid"] + d.p_grid
            out["e_part"] += d.e_part
            out["e_grid"] += d.e_grid
            out["sum_abs_j"] += d.sum_abs_j
            out["max_cells_per_step"] = max(out["max_cells_per_step"], d.max_cells_per_step)
    out["n_removed"] = int(sum(int((a == 0).sum()) for a in run.active))
    vmax, scmin = 0.0, 1.0
    for b, box in enumerate(run.boxes):
        a = run.active[b].astype(bool)
        if not a.any():
            continue
        x, p = run.x[b][a], run.p[b][a]
        sc = np.ones_like(p)
        if box.geom == "cyl":
            sc[:, 1] = x[:, 0]
        elif box.geom == "sph":
            sc[:, 1] = x[:, 0]
            sc[:, 2] = x[:, 0] * np.abs(np.sin(x[:, 1]))
        vmax = max(vmax, float(np.abs(p / sc).max()))
        scmin = min(scmin, float(sc.min()))
    out["e_scale"] = vmax * out["sum_abs_j"] / scmin
    return out


def compare_diag(diag: dict, run: OracleRun, dtype: str, label="", steps=1, base: dict | None = None,
                 with_max=True):
    """Compare the GPU's FP64 diagnostics (ctx.status(), accumulated over the
    same steps; minus `base` when given, the diagnostics of a prefix of
    steps) with the oracle's: momentum and energy sums of the particles and
    of the grid normwise against sum |J| (energy: against its bound
    e_scale), the dust time-step bound (Eq. particles_dt) relative, the
    removal count exactly.  Returns the worst normwise errors."""
    tol = TOL[dtype]
    o = oracle_diag(run, steps)
    g = {k: (np.asarray(diag[k], dtype=np.float64) if k in ("p_part", "p_grid") else diag[k])
         for k in ("p_part", "p_grid", "e_part", "e_grid", "sum_abs_j", "max_cells_per_step",
                   "n_removed")}
    if base is not None:
        for k in ("p_part", "p_grid", "e_part", "e_grid", "sum_abs_j", "n_removed"):
            bv = np.asarray(base[k], dtype=np.float64) if k in ("p_part", "p_grid") else base[k]
            g[k] = g[k] - bv
    js = max(o["sum_abs_j"], 1e-300)
    es = max(o["e_scale"], 1e-300)
    rep = {"p_part": float(np.abs(g["p_part"] - o["p_part"]).max() / js),
           "p_grid": float(np.abs(g["p_grid"] - o["p_grid"]).max() / js),
           "sum_abs_j": abs(g["sum_abs_j"] - o["sum_abs_j"]) / js,
           "e_part": abs(g["e_part"] - o["e_part"]) / es,
           "e_grid": abs(g["e_grid"] - o["e_grid"]) / es}
    if with_max:
        rep["max_cells"] = abs(g["max_cells_per_step"] - o["max_cells_per_step"]) / max(
            o["max_cells_per_step"], 1e-300)
    for k, v in rep.items():
        assert v <= tol, (label, "diag", k, v, g, o)
    assert int(g["n_removed"]) == o["n_removed"], (label, "n_removed", g["n_removed"], o["n_removed"])
    rep["n_removed"] = o["n_removed"]
    return rep


def compare_step(w, st_in, st_out, run: OracleRun, dtype: str, fields_too=True, label="", diag=None):
    """Compare the GPU state after one step (st_out) with the oracle run
    started from st_in.  Returns a dict of the worst errors; asserts the bar.
    diag: the GPU's diagnostics of that step (ctx.status()), compared with
    the oracle's when given."""
    tol = TOL[dtype]
    report = {"label": label}
    bases, _ = w.cell_bases()
    ids_out = st_out["id"]
    order_out = np.argsort(ids_out) if ids_out is not None else np.arange(len(st_out["cell"]))
    ids_in = st_in["id"] if st_in["id"] is not None else np.arange(len(st_in["cell"]))
    worst_x = worst_p = 0.0
    near_face = 0
    for b, box in enumerate(run.boxes):
        sel = run.sel[b]                       # indices into st_in order
        ids = ids_in[sel]
        gi = order_out[ids] if st_out["id"] is not None else sel
        cell_o, off_o, p_o, act_o = run.particle_state(b)
        x_o = run.x[b]
        cell_g = st_out["cell"][gi]
        act_g = cell_g >= 0
        assert np.array_equal(act_o, act_g), f"{label}: removed-particle sets differ"
        a = act_o
        if not a.any():
            continue
        # positions
        lo = bases[b]
        x_g = _global_positions(box, cell_g[a] - lo, st_out["off"][gi][a])
        widths = np.zeros((a.sum(), 3))
        cl_o = cell_o[a] - lo
        idx = O.unravel(box, cl_o)
        dx = x_g - x_o[a]
        for d in range(box.ndim):
            c, wd = O.centers_widths(box, d)
            widths[:, d] = wd[idx[d]]
            if box.bc_lo[d] in ("periodic", "shear"):
                L = box.faces[d][-1] - box.faces[d][0]
                dx[:, d] = (dx[:, d] + 0.5 * L) % L - 0.5 * L
        ex = np.abs(dx[:, :box.ndim]) / widths[:, :box.ndim]
        worst_x = max(worst_x, float(ex.max()))
        # cells: exact except near faces
        diff = cell_g[a] != cell_o[a]
        if diff.any():
            offo = off_o[a][diff][:, :box.ndim]
            near = np.any(np.abs(np.abs(offo) - 0.5) <= max(tol, 1e-12) * 4, axis=1)
            near_face += int(near.sum())
            assert near.all(), f"{label}: {int((~near).sum())} cell mismatches away from faces"
        # momenta
        nc = box.ndim if box.geom == "cart" else 3
        pg = st_out["mom"][gi][a][:, :nc]
        po = p_o[a][:, :nc]
        p0 = st_in["mom"][sel][a][:, :nc]
        # |p_g| bound: the largest gas speed over the gather stencil at
        # x^{n+1/2}, whose cells lie within one cell of the half-step cell,
        # itself within one cell of the final cell (a half step moves a
        # particle less than a cell under the dust time step, Eq.
        # particles_dt): the 5x5x5 cells around the final cell
        vmax = np.max([np.abs(v) for v in st_in["gas"][b]["vel"][:nc]], axis=0)
        vmax = maximum_filter(vmax, size=5, mode="nearest").reshape(box.ghosted_shape)
        ci = O.unravel(box, cl_o)
        gmax = vmax[(ci[2] + (1 if box.ndim > 2 else 0), ci[1] + 1, ci[0] + 1)]
        xo = x_o[a]
        sc = np.ones((a.sum(), 3))
        if box.geom == "cyl":
            sc[:, 1] = xo[:, 0]
        elif box.geom == "sph":
            sc[:, 1] = xo[:, 0]
            sc[:, 2] = xo[:, 0] * np.sin(xo[:, 1])
        scale = (np.abs(po).max(axis=1) + np.abs(p0).max(axis=1) +
                 gmax * sc[:, :nc].max(axis=1) + 1e-300)
        ep = np.abs(pg - po).max(axis=1) / scale
        worst_p = max(worst_p, float(ep.max()))
    report["pos"] = worst_x
    report["mom"] = worst_p
    report["near_face"] = near_face
    assert worst_x <= tol, report
    assert worst_p <= tol, report
    if fields_too:
        worst_f = 0.0
        for b, box in enumerate(run.boxes):
            fo = run.fields[b]
            nc = fo.nc
            for c in range(nc + 1):
                ref = fo.dep[c].reshape(-1)
                got = st_out["dep"][b][c].reshape(-1)
                den = np.abs(ref).max()
                if den == 0:
                    assert np.abs(got).max() == 0, (label, "dep", c)
                    continue
                e = np.abs(got - ref).max() / den
                worst_f = max(worst_f, e)
                assert e <= tol, (label, "dep", b, c, e)
            if w.apply_feedback:
                for c in range(nc):
                    ref = fo.vel[c].reshape(fo.box.ghosted_shape)
                    got = st_out["gas"][b]["vel"][c].reshape(fo.box.ghosted_shape)
                    act = (slice(1, -1),) * 3 if box.ndim == 3 else (0, slice(1, -1), slice(1, -1))
                    den = np.abs(ref[act]).max()
                    e = np.abs(got[act] - ref[act]).max() / max(den, 1e-300)
                    worst_f = max(worst_f, e)
                    assert e <= tol, (label, "vel", b, c, e)
        report["fields"] = worst_f
    if diag is not None:
        report["diag"] = compare_diag(diag, run, dtype, label=label)
    return report
