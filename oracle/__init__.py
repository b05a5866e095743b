"""FP64 CPU oracle of the dust-particle hot path (Mignone, Flock & Vaidya 2019).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never calls it and shares no code with it: the C core
(``dust_oracle.c``) has its own types, constants and arithmetic, and this
wrapper only marshals numpy arrays.

Conventions (independent of the HIP library's own):
  * positions are global FP64 coordinates (x, y, z) / (R, phi, z) /
    (r, theta, phi);
  * momenta are canonical: Cartesian v, cylindrical (v_R, l_phi, v_z),
    spherical (v_r, l_theta, l_phi)  (Eq. dust_cylindrical, dust_spherical);
  * fields are ghosted cell-centred arrays, axis 0 fastest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dust_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

GEOM = {"cart": 0, "cyl": 1, "sph": 2}
BC = {"periodic": 0, "shear": 1, "open": 2}
SHAPE = {"cic": 0, "tsc": 1, "vol": 2}   # vol: cylindrical radius only
FORCE = {"none": 0, "shearbox": 1, "pointmass": 2, "const": 3, "shearbox_fargo": 4}
DRAG = {"tau": 0, "stokes": 1, "epstein": 2}
STEP_APPLY_FEEDBACK = 1
STEP_FILL_GHOSTS = 2


def build(force: bool = True) -> str:
    """Compile the oracle with plain -O2 (no fast-math) into liboracle.so
    (with OpenMP for the threaded timing variant orc_step_threads)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_SO)
        _declare(_lib)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


GAS_FN = ctypes.CFUNCTYPE(None, _dp, _dp)


class _Box(ctypes.Structure):
    _fields_ = [("geom", ctypes.c_int32), ("ndim", ctypes.c_int32),
                ("n", ctypes.c_int32 * 3), ("bc_lo", ctypes.c_int32 * 3),
                ("bc_hi", ctypes.c_int32 * 3), ("shape", ctypes.c_int32 * 3),
                ("faces", _dp * 3)]


class _Forces(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("vertical_gravity", ctypes.c_int32),
                ("Omega", ctypes.c_double), ("q", ctypes.c_double),
                ("GM", ctypes.c_double), ("g", ctypes.c_double * 3), ("integrator", ctypes.c_int32)]


class _Particles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", _dp * 3), ("p", _dp * 3),
                ("drag", _dp), ("mass", _dp), ("active", _ip)]


class _Fields(ctypes.Structure):
    _fields_ = [("rho", _dp), ("vel", _dp * 3), ("dep", _dp * 4)]


class _Diag(ctypes.Structure):
    _fields_ = [("p_part", ctypes.c_double * 3), ("p_grid", ctypes.c_double * 3),
                ("e_part", ctypes.c_double), ("e_grid", ctypes.c_double),
                ("sum_abs_j", ctypes.c_double), ("max_cells_per_step", ctypes.c_double),
                ("n_inactive", ctypes.c_int64)]


def _declare(L):
    L.orc_locate.argtypes = [ctypes.POINTER(_Box), ctypes.c_int, ctypes.c_double]
    L.orc_locate.restype = ctypes.c_int
    L.orc_weights_axis.argtypes = [ctypes.POINTER(_Box), ctypes.c_int, ctypes.c_int,
                                   ctypes.c_double, _dp]
    L.orc_weight_any_cell.argtypes = [ctypes.POINTER(_Box), ctypes.c_int, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_int]
    L.orc_weight_any_cell.restype = ctypes.c_double
    L.orc_weights_paper.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
    L.orc_cell_volume.argtypes = [ctypes.POINTER(_Box), ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int]
    L.orc_cell_volume.restype = ctypes.c_double
    L.orc_fill_ghosts.argtypes = [ctypes.POINTER(_Box), ctypes.POINTER(_Forces),
                                  ctypes.c_double, ctypes.POINTER(_Fields)]
    L.orc_fold_ghosts.argtypes = L.orc_fill_ghosts.argtypes
    L.orc_gather.argtypes = [ctypes.POINTER(_Box), ctypes.POINTER(_Fields), _dp, _dp, _dp]
    L.orc_gather.restype = ctypes.c_int
    L.orc_kick.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Forces),
                           ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp]
    L.orc_step.argtypes = [ctypes.POINTER(_Box), ctypes.POINTER(_Forces), ctypes.c_int,
                           ctypes.POINTER(_Particles), ctypes.POINTER(_Fields),
                           ctypes.c_double, ctypes.c_double, ctypes.c_int,
                           ctypes.POINTER(_Diag)]
    L.orc_step.restype = ctypes.c_int
    L.orc_step_threads.argtypes = L.orc_step.argtypes
    L.orc_step_threads.restype = ctypes.c_int
    L.orc_drag_source.argtypes = [ctypes.POINTER(_Box), ctypes.POINTER(_Forces), ctypes.c_int,
                                  ctypes.POINTER(_Particles), ctypes.POINTER(_Fields),
                                  ctypes.c_double]
    L.orc_drag_source.restype = None
    L.orc_deposit_mass.argtypes = [ctypes.POINTER(_Box), ctypes.POINTER(_Particles), _dp]
    L.orc_deposit_mass.restype = None
    L.orc_gl_integrate_poly.argtypes = [_dp, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    L.orc_gl_integrate_poly.restype = ctypes.c_double
    L.orc_push_one.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Forces), ctypes.c_int,
                               ctypes.c_double, ctypes.c_double, _dp, _dp, GAS_FN, _dp]
    L.orc_n_ghosted.argtypes = [ctypes.POINTER(_Box)]
    L.orc_n_ghosted.restype = ctypes.c_int64


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


@dataclass
class Box:
    """One grid box: geometry name, active cells per axis, boundary names,
    shape names and FP64 face arrays (n[d]+1 each)."""
    geom: str
    n: tuple
    bc_lo: tuple
    bc_hi: tuple
    shape: tuple
    faces: list
    ndim: int = 3
    _c: _Box = field(default=None, repr=False)

    def c(self) -> _Box:
        if self._c is None:
            self.faces = [np.ascontiguousarray(f, dtype=np.float64) for f in self.faces]
            while len(self.faces) < 3:
                self.faces.append(np.array([0.0, 1.0]))
            b = _Box()
            b.geom = GEOM[self.geom]
            b.ndim = self.ndim
            n = list(self.n) + [1] * (3 - len(self.n))
            for d in range(3):
                b.n[d] = n[d]
                b.bc_lo[d] = BC[self.bc_lo[d]] if d < self.ndim else 0
                b.bc_hi[d] = BC[self.bc_hi[d]] if d < self.ndim else 0
                b.shape[d] = SHAPE[self.shape[d]] if d < self.ndim else 0
                if d < self.ndim and self.shape[d] == "vol" and (self.geom != "cyl" or d != 0):
                    raise ValueError("volume weighting is for the cylindrical radius only")
                b.faces[d] = _ptr(self.faces[d])
            self._c = b
        return self._c

    @property
    def ghosted_shape(self):
        """numpy shape (z, y, x) of a ghosted field."""
        g = [self.n[d] + 2 if d < self.ndim else 1 for d in range(3)]
        return (g[2], g[1], g[0])

    @property
    def n_active(self) -> int:
        return int(np.prod([self.n[d] for d in range(self.ndim)]))


@dataclass
class Forces:
    kind: str = "none"
    Omega: float = 0.0
    q: float = 0.0
    GM: float = 0.0
    vertical_gravity: bool = False
    g: tuple = (0.0, 0.0, 0.0)
    integrator: str = "em"   # "em" exponential midpoint, "si" semi-implicit (Cartesian)

    def c(self) -> _Forces:
        f = _Forces()
        f.kind = FORCE[self.kind]
        f.integrator = {"em": 0, "si": 1}[self.integrator]
        f.vertical_gravity = int(self.vertical_gravity)
        f.Omega, f.q, f.GM = self.Omega, self.q, self.GM
        for d in range(3):
            f.g[d] = self.g[d]
        return f


def centers_widths(box: Box, d: int):
    f = np.asarray(box.faces[d], dtype=np.float64)
    return 0.5 * (f[:-1] + f[1:]), f[1:] - f[:-1]


def unravel(box: Box, local_cell: np.ndarray):
    """Active linear cell index (axis 0 fastest) -> per-axis indices."""
    c = np.asarray(local_cell, dtype=np.int64)
    i = c % box.n[0]
    j = (c // box.n[0]) % box.n[1]
    k = c // (box.n[0] * box.n[1]) if box.ndim > 2 else np.zeros_like(c)
    return i, j, k


def ravel(box: Box, i, j, k):
    if box.ndim > 2:
        return (np.asarray(i) + box.n[0] * (np.asarray(j) + box.n[1] * np.asarray(k))).astype(np.int64)
    return (np.asarray(i) + box.n[0] * np.asarray(j)).astype(np.int64)


def to_global(box: Box, local_cell, off):
    """(cell, offset delta in host-cell widths) -> global FP64 coordinates:
    xi = centre_i + delta * width_i on every axis."""
    idx = unravel(box, local_cell)
    off = np.asarray(off, dtype=np.float64)
    x = np.zeros((len(idx[0]), 3))
    for d in range(box.ndim):
        c, w = centers_widths(box, d)
        x[:, d] = c[idx[d]] + off[:, d] * w[idx[d]]
    return x


def to_cell_offset(box: Box, x):
    """Global coordinates -> (local cell, delta); cell -1 if outside."""
    L = lib()
    b = box.c()
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    idx = np.zeros((3, n), dtype=np.int64)
    off = np.zeros((n, 3))
    ok = np.ones(n, dtype=bool)
    for d in range(box.ndim):
        c, w = centers_widths(box, d)
        for p in range(n):
            i = L.orc_locate(ctypes.byref(b), d, float(x[p, d]))
            if i < 0:
                ok[p] = False
                continue
            idx[d, p] = i
            off[p, d] = (x[p, d] - c[i]) / w[i]
    cell = ravel(box, idx[0], idx[1], idx[2])
    cell[~ok] = -1
    return cell, off


def weights_axis(box: Box, d: int, i: int, xi: float) -> np.ndarray:
    w = np.zeros(3)
    lib().orc_weights_axis(ctypes.byref(box.c()), d, i, xi, _ptr(w))
    return w


def weight_any_cell(box: Box, d: int, i_host: int, xi: float, k: int) -> float:
    return lib().orc_weight_any_cell(ctypes.byref(box.c()), d, i_host, xi, k)


def weights_paper(kind: str, shape: str, delta: float, nu: float = 0.0,
                  xlo: float = 0.0, xhi: float = 0.0) -> np.ndarray:
    k = {"cart": 0, "cyl_r": 1, "sph_r": 2, "sph_theta": 3}[kind]
    w = np.zeros(3)
    lib().orc_weights_paper(k, SHAPE[shape], delta, nu, xlo, xhi, _ptr(w))
    return w


def cell_volume(box: Box, i: int, j: int, k: int) -> float:
    return lib().orc_cell_volume(ctypes.byref(box.c()), i, j, k)


def gl_integrate_poly(coef, a, b) -> float:
    c = np.ascontiguousarray(coef, dtype=np.float64)
    return lib().orc_gl_integrate_poly(_ptr(c), len(c) - 1, a, b)


class Fields:
    """Ghosted FP64 gas and deposit arrays of one box."""

    def __init__(self, box: Box, rho, vel, dep=None):
        shp = box.ghosted_shape
        self.box = box
        self.rho = np.ascontiguousarray(np.asarray(rho, dtype=np.float64).reshape(shp))
        nc = box.ndim if box.geom == "cart" else 3
        self.nc = nc
        self.vel = [np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(shp))
                    for v in vel[:nc]]
        while len(self.vel) < 3:
            self.vel.append(np.zeros(shp))
        if dep is None:
            dep = [np.zeros(shp) for _ in range(nc + 1)]
        self.dep = [np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shp))
                    for a in dep]
        while len(self.dep) < 4:
            self.dep.append(np.zeros(shp))

    def c(self) -> _Fields:
        f = _Fields()
        f.rho = _ptr(self.rho)
        for m in range(3):
            f.vel[m] = _ptr(self.vel[m])
        for m in range(4):
            f.dep[m] = _ptr(self.dep[m])
        return f


def fill_ghosts(box: Box, forces: Forces, t: float, fields: Fields):
    lib().orc_fill_ghosts(ctypes.byref(box.c()), ctypes.byref(forces.c()), t,
                          ctypes.byref(fields.c()))


def fold_ghosts(box: Box, forces: Forces, t: float, fields: Fields):
    lib().orc_fold_ghosts(ctypes.byref(box.c()), ctypes.byref(forces.c()), t,
                          ctypes.byref(fields.c()))


def gather(box: Box, fields: Fields, x):
    """Weights + gather at global positions x (N,3) -> rho (N,), vg (N,3)."""
    L = lib()
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    rho = np.zeros(n)
    vg = np.zeros((n, 3))
    fc = fields.c()
    b = box.c()
    r = np.zeros(1)
    v = np.zeros(3)
    for p in range(n):
        xp = np.ascontiguousarray(x[p])
        ok = L.orc_gather(ctypes.byref(b), ctypes.byref(fc), _ptr(xp), _ptr(r), _ptr(v))
        if not ok:
            raise ValueError("particle outside the box")
        rho[p] = r[0]
        vg[p] = v
    return rho, vg


def kick(geom: str, ndim: int, forces: Forces, dt: float, inv_tau: float, x, p, pg):
    """One exponential-midpoint kick; returns (p_new, a_nondrag)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    pn = np.ascontiguousarray(p, dtype=np.float64).copy()
    pg = np.ascontiguousarray(pg, dtype=np.float64)
    a = np.zeros(3)
    lib().orc_kick(GEOM[geom], ndim, ctypes.byref(forces.c()), dt, inv_tau, _ptr(x),
                   _ptr(pn), _ptr(pg), _ptr(a))
    return pn, a


def push_one(geom: str, forces: Forces, drag_mode: str, dragval: float, dt: float, x, p,
             gas=None, ndim: int = 3):
    """Drift-kick-drift of one particle through gas given by gas(x) ->
    physical local-basis velocity (3,), no grid; x, p updated in place."""
    assert x.dtype == np.float64 and p.dtype == np.float64
    a = np.zeros(3)
    if gas is None:
        cb = GAS_FN(0)
    else:
        def _cb(xp, vp):
            v = gas(np.array([xp[0], xp[1], xp[2]]))
            vp[0], vp[1], vp[2] = float(v[0]), float(v[1]), float(v[2])
        cb = GAS_FN(_cb)
    lib().orc_push_one(GEOM[geom], ndim, ctypes.byref(forces.c()), DRAG[drag_mode], dragval, dt,
                       _ptr(x), _ptr(p), cb, _ptr(a))
    return a


@dataclass
class Diag:
    p_part: np.ndarray
    p_grid: np.ndarray
    e_part: float
    e_grid: float
    sum_abs_j: float
    max_cells_per_step: float
    n_inactive: int
    threads: int = 1


def step(box: Box, forces: Forces, drag_mode: str, x, p, drag, mass, active,
         fields: Fields, dt: float, t: float, apply_feedback: bool = False,
         fill_ghosts: bool = True, threads: bool = False) -> Diag:
    """One step of the hot path for the particles of one box, in place:
    x (N,3), p (N,3) FP64, drag (tau or St) and mass (N,), active (N,) int32;
    fields' velocities are updated if apply_feedback, deposits overwritten.
    threads: the OpenMP variant (particle ranges per host thread, private
    deposit arrays added in thread order), for timing on every core; the
    thread count is in the returned Diag's `threads`."""
    for a in (x, p):
        assert a.dtype == np.float64 and a.flags.c_contiguous and a.shape[1] == 3
    n = x.shape[0]
    xs = [np.ascontiguousarray(x[:, d]) for d in range(3)]
    ps = [np.ascontiguousarray(p[:, d]) for d in range(3)]
    drag = np.ascontiguousarray(drag, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    assert active.dtype == np.int32
    P = _Particles()
    P.n = n
    for d in range(3):
        P.x[d] = _ptr(xs[d])
        P.p[d] = _ptr(ps[d])
    P.drag = _ptr(drag)
    P.mass = _ptr(mass)
    P.active = active.ctypes.data_as(_ip)
    dg = _Diag()
    flags = (STEP_APPLY_FEEDBACK if apply_feedback else 0) | (STEP_FILL_GHOSTS if fill_ghosts else 0)
    fc = fields.c()
    fn = lib().orc_step_threads if threads else lib().orc_step
    nt = fn(ctypes.byref(box.c()), ctypes.byref(forces.c()), DRAG[drag_mode],
            ctypes.byref(P), ctypes.byref(fc), dt, t, flags, ctypes.byref(dg))
    if nt < 0:
        raise MemoryError("oracle: private deposit arrays")
    for d in range(3):
        x[:, d] = xs[d]
        p[:, d] = ps[d]
    return Diag(np.array(dg.p_part[:]), np.array(dg.p_grid[:]), dg.e_part, dg.e_grid,
                dg.sum_abs_j, dg.max_cells_per_step, dg.n_inactive, nt if threads else 1)


def drag_source(box: Box, forces: Forces, drag_mode: str, x, p, drag, mass, active,
                fields: Fields, dt: float) -> None:
    """Drag source of the gas predictor (Sec. 3.1, Eq. Delta_vp and f_D with
    tau <- max(tau, dt)) at the particles' current positions, accumulated
    into the momentum channels of fields.dep (force densities, canonical
    components); the energy channel is left as it is."""
    for a in (x, p):
        assert a.dtype == np.float64 and a.flags.c_contiguous and a.shape[1] == 3
    xs = [np.ascontiguousarray(x[:, d]) for d in range(3)]
    ps = [np.ascontiguousarray(p[:, d]) for d in range(3)]
    drag = np.ascontiguousarray(drag, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    assert active.dtype == np.int32 and active.flags.c_contiguous
    P = _Particles()
    P.n = x.shape[0]
    for d in range(3):
        P.x[d] = _ptr(xs[d])
        P.p[d] = _ptr(ps[d])
    P.drag = _ptr(drag)
    P.mass = _ptr(mass)
    P.active = active.ctypes.data_as(_ip)
    fc = fields.c()
    lib().orc_drag_source(ctypes.byref(box.c()), ctypes.byref(forces.c()), DRAG[drag_mode],
                          ctypes.byref(P), ctypes.byref(fc), dt)


def deposit_mass(box: Box, x, mass, active, rho_d) -> None:
    """Dust density of the particles at global positions x (N,3): each
    mass spread with the gather's weights over the cell volumes, added to
    the ghosted array rho_d (ghosts included, unfolded)."""
    assert x.dtype == np.float64 and x.flags.c_contiguous and x.shape[1] == 3
    assert rho_d.dtype == np.float64 and rho_d.flags.c_contiguous
    assert rho_d.size == int(np.prod(box.ghosted_shape))
    xs = [np.ascontiguousarray(x[:, d]) for d in range(3)]
    zeros = np.zeros(x.shape[0])
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    active = np.ascontiguousarray(active, dtype=np.int32)
    P = _Particles()
    P.n = x.shape[0]
    for d in range(3):
        P.x[d] = _ptr(xs[d])
        P.p[d] = _ptr(zeros)
    P.drag = _ptr(zeros)
    P.mass = _ptr(mass)
    P.active = active.ctypes.data_as(_ip)
    lib().orc_deposit_mass(ctypes.byref(box.c()), ctypes.byref(P), _ptr(rho_d))


# --------------------------------------------------------------------------
# Binning reference: a stable sort of integer keys (library primitive).

def bin_reference(keys, nbins: int):
    """Stable sort by key; keys outside [0, nbins) (inactive particles, key
    -1) go last.  Returns (perm, start) with start[k] the first sorted slot of
    bin k and start[nbins] the number of particles in bins."""
    k = np.asarray(keys, dtype=np.int64).copy()
    k[(k < 0) | (k >= nbins)] = nbins
    perm = np.argsort(k, kind="stable").astype(np.int32)
    counts = np.bincount(k, minlength=nbins + 1)[:nbins + 1]
    start = np.zeros(nbins + 1, dtype=np.int64)
    start[1:] = np.cumsum(counts[:nbins])
    return perm, start


def tile_major_keys(cells, n, tile):
    """Re-number active cells tile by tile (tiles of tile[0] x tile[1] x
    tile[2] cells, tiles and cells inside a tile both in axis-0-fastest order;
    edge tiles are clipped).  Returns the new numbering of each input cell id
    (local to one box); -1 stays -1."""
    c = np.asarray(cells, dtype=np.int64)
    ok = c >= 0
    cc = np.where(ok, c, 0)
    n = list(n) + [1] * (3 - len(n))
    tile = list(tile) + [1] * (3 - len(tile))
    i = cc % n[0]
    j = (cc // n[0]) % n[1]
    k = cc // (n[0] * n[1])
    nt = [(n[d] + tile[d] - 1) // tile[d] for d in range(3)]
    ti, tj, tk = i // tile[0], j // tile[1], k // tile[2]
    tid = ti + nt[0] * (tj + nt[1] * tk)
    # cells before tile tid in the renumbering: sum of clipped tile volumes.
    def tsize(a, d):
        return np.minimum(tile[d], n[d] - a * tile[d])
    ext0, ext1, ext2 = tsize(ti, 0), tsize(tj, 1), tsize(tk, 2)
    # number of cells in all tiles that come before (ti, tj, tk)
    full_planes = tk * tile[2] * n[0] * n[1]
    full_rows = tj * tile[1] * n[0] * ext2
    before_in_row = ti * tile[0] * ext1 * ext2
    li = (i - ti * tile[0]) + ext0 * ((j - tj * tile[1]) + ext1 * (k - tk * tile[2]))
    out = full_planes + full_rows + before_in_row + li
    return np.where(ok, out, -1)
