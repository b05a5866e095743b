"""Run the oracle on a whole workload (test infrastructure only).

Takes any object with the attributes of a synthetic workload (boxes, gas,
particle arrays, species tables, dt, ...) and steps every box's particles
with the FP64 oracle.  Particle inputs given in single precision are widened
exactly; nothing here comes from the HIP library.
"""
from __future__ import annotations

import numpy as np

from . import Box, Fields, Forces, step, to_global


def make_box(bd: dict) -> Box:
    nd = bd["ndim"]
    return Box(geom=bd["geom"], n=tuple(bd["n"]), bc_lo=tuple(bd["bc_lo"]),
               bc_hi=tuple(bd["bc_hi"]), shape=tuple(bd["shape"]),
               faces=[np.asarray(f, dtype=np.float64) for f in bd["faces"][:nd]], ndim=nd)


def make_forces(fd: dict) -> Forces:
    return Forces(kind=fd.get("kind", "none"), Omega=fd.get("Omega", 0.0), q=fd.get("q", 0.0),
                  GM=fd.get("GM", 0.0), vertical_gravity=bool(fd.get("vertical_gravity", False)),
                  g=tuple(fd.get("g", (0.0, 0.0, 0.0))), integrator=fd.get("integrator", "em"))


def locate_cells(box: Box, x: np.ndarray):
    """(cell, delta) of global positions with half-open ownership, by a
    sorted search of the faces (library primitive)."""
    n = x.shape[0]
    idx = []
    off = np.zeros((n, 3))
    ok = np.ones(n, dtype=bool)
    for d in range(box.ndim):
        f = np.asarray(box.faces[d], dtype=np.float64)
        i = np.searchsorted(f, x[:, d], side="right") - 1
        good = (i >= 0) & (i < box.n[d])
        ok &= good
        i = np.clip(i, 0, box.n[d] - 1)
        c = 0.5 * (f[i] + f[i + 1])
        w = f[i + 1] - f[i]
        off[:, d] = (x[:, d] - c) / w
        idx.append(i)
    while len(idx) < 3:
        idx.append(np.zeros(n, dtype=np.int64))
    if box.ndim > 2:
        cell = idx[0] + box.n[0] * (idx[1] + box.n[1] * idx[2])
    else:
        cell = idx[0] + box.n[0] * idx[1]
    cell = np.where(ok, cell, -1)
    return cell.astype(np.int64), off


def per_particle_tables(w, sel):
    """drag (tau or St) and mass of the selected particles, FP64."""
    if w.drag_mode == "species":
        sp = np.asarray(w.species)[sel].astype(np.int64)
        drag = np.asarray(w.species_tau, dtype=np.float64)[sp]
        mass = np.asarray(w.species_mass, dtype=np.float64)[sp]
        mode = "tau"
    else:
        drag = np.asarray(w.drag)[sel].astype(np.float64)
        mode = w.drag_mode
        if w.mass is not None:
            mass = np.asarray(w.mass)[sel].astype(np.float64)
        else:
            mass = np.full(len(drag), float(w.species_mass[0]))
    return mode, drag, mass


class OracleRun:
    """State of one workload evolved by the oracle."""

    def __init__(self, w, particle_limit: int | None = None):
        self.w = w
        self.boxes = [make_box(b) for b in w.boxes]
        self.forces = make_forces(w.forces)
        bases, total = w.cell_bases()
        self.bases = bases
        cell = np.asarray(w.cell).astype(np.int64)
        self.sel, self.x, self.p, self.drag, self.mass, self.active, self.mode = \
            [], [], [], [], [], [], []
        self.fields = []
        for b, box in enumerate(self.boxes):
            lo, hi = bases[b], bases[b] + box.n_active
            sel = np.nonzero((cell >= lo) & (cell < hi))[0]
            if particle_limit is not None:
                sel = sel[:particle_limit]
            self.sel.append(sel)
            x = to_global(box, cell[sel] - lo, np.asarray(w.off)[sel].astype(np.float64))
            self.x.append(np.ascontiguousarray(x))
            self.p.append(np.ascontiguousarray(np.asarray(w.mom)[sel].astype(np.float64)))
            mode, drag, mass = per_particle_tables(w, sel)
            self.mode.append(mode)
            self.drag.append(drag)
            self.mass.append(mass)
            self.active.append(np.ones(len(sel), dtype=np.int32))
            g = w.gas[b]
            # copies: the step updates the gas in place (feedback)
            self.fields.append(Fields(box, np.array(g["rho"], dtype=np.float64),
                                      [np.array(v, dtype=np.float64) for v in g["vel"]]))
        self.t = float(w.t0)
        self.diags = []

    def step(self, nsteps: int = 1, apply_feedback: bool | None = None, threads: bool = False):
        """nsteps steps of every box (threads: the OpenMP variant of the
        step, for timing on every host core)."""
        fb = self.w.apply_feedback if apply_feedback is None else apply_feedback
        for _ in range(nsteps):
            ds = []
            for b, box in enumerate(self.boxes):
                ds.append(step(box, self.forces, self.mode[b], self.x[b], self.p[b],
                               self.drag[b], self.mass[b], self.active[b], self.fields[b],
                               self.w.dt, self.t, apply_feedback=fb, threads=threads))
            self.diags.append(ds)
            self.t += self.w.dt

    def particle_state(self, b: int):
        """(global cell id, delta, momenta, active) of box b's particles."""
        box = self.boxes[b]
        cell, off = locate_cells(box, self.x[b])
        act = self.active[b].astype(bool)
        cell = np.where(act & (cell >= 0), cell + self.bases[b], -1)
        return cell, off, self.p[b], act
