"""Seeded synthetic workloads shaped like the paper's test problems.

This module only draws inputs: grids, particle states and gas fields.  It
holds none of the method's arithmetic (no weights, no push, no deposit) and
is the one module that both the HIP path and the FP64 oracle take inputs
from.  Every array is produced from ``numpy.random.Generator(PCG64)`` seeded
with ``190810793 + k``.

Particle state is produced directly in the representation both sides accept:
global cell id (active cells, axis 0 fastest, boxes concatenated) plus the
offset ``delta`` in [-1/2, 1/2) of the host-cell width on every axis, and
canonical momenta (Cartesian v; cylindrical (v_R, l_phi, v_z); spherical
(v_r, l_theta, l_phi)).  Gas fields are ghosted, cell centred, shape
(n2+2, n1+2, n0+2) (2-D: (n1+2, n0+2)).

Workloads (recipes in the design notes):
  cart2d_periodic    2-D periodic box, uniform random particles, CIC, FP64
  shearing_box       3-D shearing box, YJ07-style seeded sub-lattice, TSC
  cylindrical_disk   log-spaced R, Keplerian disk gas (Nelson et al. 2013
                     profile of the radial-drift test), Stokes numbers
  spherical_disk     the same disk in (r, theta, phi), stiff stopping times
  batched_boxes      several periodic 3-D boxes (same cell width), four species
  rigid_disk         uniform dust density in a cylindrical grid, radii from
                     the inverse cumulative distribution (particle assignment)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED0 = 190810793


def rng(k: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED0 + k))


@dataclass
class Workload:
    name: str
    dtype: str                      # "f32" or "f64"
    boxes: list                     # dicts: geom, ndim, n, bc_lo, bc_hi, shape, faces
    forces: dict
    drag_mode: str                  # "tau", "stokes" or "species"
    cell: np.ndarray                # int32 (N,)
    off: np.ndarray                 # (N,3)
    mom: np.ndarray                 # (N,3)
    gas: list                       # per box: {"rho": arr, "vel": [arr]*nc}
    dt: float
    nsteps: int
    t0: float = 0.0
    drag: np.ndarray | None = None  # (N,) tau (+inf allowed) or St
    mass: np.ndarray | None = None  # (N,)
    species: np.ndarray | None = None
    species_tau: list | None = None
    species_mass: list | None = None
    apply_feedback: bool = True
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.cell.shape[0])

    @property
    def np_dtype(self):
        return np.float64 if self.dtype == "f64" else np.float32

    def cell_bases(self):
        base, out = 0, []
        for b in self.boxes:
            out.append(base)
            base += int(np.prod(b["n"][: b["ndim"]]))
        return out, base


def _ghost_shape(n, ndim):
    g = [n[d] + 2 if d < ndim else 1 for d in range(3)]
    return (g[2], g[1], g[0]) if ndim == 3 else (g[1], g[0])


def _uniform_faces(lo, hi, n):
    return np.linspace(lo, hi, n + 1)


def _ghosted_centres(faces):
    """Centres of cells -1..n with ghost widths equal to the adjacent cell."""
    f = np.asarray(faces, dtype=np.float64)
    ext = np.concatenate([[f[0] - (f[1] - f[0])], f, [f[-1] + (f[-1] - f[-2])]])
    return 0.5 * (ext[:-1] + ext[1:])


def _offsets(r: np.random.Generator, size, dt_np):
    """Offsets uniform in [-1/2, 1/2), drawn in the storage precision (a
    double rounded to single precision could reach +1/2)."""
    return r.random(size, dtype=dt_np) - dt_np(0.5)


def _active_centres(faces):
    f = np.asarray(faces, dtype=np.float64)
    return 0.5 * (f[:-1] + f[1:])


# ---------------------------------------------------------------------------

def cart2d_periodic(n=(64, 64), ppc=16, tau=0.1, dt=0.01, nsteps=10, dtype="f64",
                    shape="cic", seed=0) -> Workload:
    """2-D periodic unit square; particles uniform at random, at rest; gas
    rho = 1 + 1e-3 N(0,1), v ~ U(-0.01, 0.01); one species; eps = 1."""
    r = rng(seed)
    ncell = n[0] * n[1]
    N = ncell * ppc
    dt_np = np.float64 if dtype == "f64" else np.float32
    cell = r.integers(0, ncell, size=N).astype(np.int32)
    off = np.zeros((N, 3), dtype=dt_np)
    off[:, :2] = _offsets(r, (N, 2), dt_np)
    mom = np.zeros((N, 3), dtype=dt_np)
    gs = _ghost_shape(n, 2)
    rho = np.ones(gs)
    vel = [np.zeros(gs), np.zeros(gs)]
    rho[1:-1, 1:-1] = 1.0 + 1e-3 * r.standard_normal((n[1], n[0]))
    for c in range(2):
        vel[c][1:-1, 1:-1] = r.uniform(-0.01, 0.01, size=(n[1], n[0]))
    dV = 1.0 / ncell
    m = 1.0 * 1.0 * dV / ppc
    box = dict(geom="cart", ndim=2, n=(n[0], n[1], 1), bc_lo=("periodic",) * 3,
               bc_hi=("periodic",) * 3, shape=(shape, shape, shape),
               faces=[_uniform_faces(0, 1, n[0]), _uniform_faces(0, 1, n[1])])
    return Workload("cart2d_periodic", dtype, [box], dict(kind="none"), "species", cell, off,
                    mom, [dict(rho=rho.astype(dt_np), vel=[v.astype(dt_np) for v in vel])],
                    dt, nsteps, species=np.zeros(N, dtype=np.uint8), species_tau=[tau],
                    species_mass=[m])


def shearing_box(n=(128, 128, 128), L=2.0, Omega=1.0, q=1.5, tau_omega=0.1, A=0.01, dt=0.005,
                 nsteps=10, dtype="f32", seed=1, shape="tsc", fargo=False) -> Workload:
    """Unstratified standard shearing box [-L/2, L/2]^3: 8 particles per cell
    on the 2x2x2 sub-lattice (+-1/4 cell), displaced along x by
    xi_x = (A/k_x)(-sin(k_x x) + (A/2) sin(2 k_x x)) with k_x = 2 pi/L_x,
    moving with the shear (0, -q Omega x, 0); gas rho = 1 + A cos(k_x x),
    v = (0, -q Omega x, 0) + N(0, 1e-3).  fargo: the orbital-advection form
    (Eq. FARGO_SB_p): particle and gas velocities are the residuals
    v' = v + q Omega x e_y (the same draws, without the mean shear)."""
    r = rng(seed)
    dt_np = np.float64 if dtype == "f64" else np.float32
    dx = L / n[0]
    ncell = n[0] * n[1] * n[2]
    faces = [_uniform_faces(-L / 2, L / 2, n[d]) for d in range(3)]
    xc = _active_centres(faces[0])
    kx = 2 * np.pi / L
    cells = np.arange(ncell, dtype=np.int64)
    ci = cells % n[0]
    sub = np.array([[sx, sy, sz] for sz in (-0.25, 0.25) for sy in (-0.25, 0.25)
                    for sx in (-0.25, 0.25)])
    N = ncell * 8
    cell = np.repeat(cells, 8).astype(np.int32)
    off = np.tile(sub, (ncell, 1))
    x_eq = xc[np.repeat(ci, 8)] + off[:, 0] * dx
    xi = (A / kx) * (-np.sin(kx * x_eq) + 0.5 * A * np.sin(2 * kx * x_eq))
    off[:, 0] += xi / dx
    off = off.astype(dt_np)
    x_p = xc[np.repeat(ci, 8)] + off[:, 0].astype(np.float64) * dx
    mom = np.zeros((N, 3))
    mom[:, 1] = 0.0 if fargo else -q * Omega * x_p
    mom = mom.astype(dt_np)
    perm = r.permutation(N)
    cell, off, mom = cell[perm], off[perm], mom[perm]
    gs = _ghost_shape(n, 3)
    xg = _ghosted_centres(faces[0])[None, None, :]
    rho = np.broadcast_to(1.0 + A * np.cos(kx * xg), gs).copy()
    vx = 1e-3 * r.standard_normal(gs)
    vy = (0.0 if fargo else -q * Omega * xg) + 1e-3 * r.standard_normal(gs)
    vz = 1e-3 * r.standard_normal(gs)
    m = 1.0 * dx ** 3 / 8.0
    box = dict(geom="cart", ndim=3, n=tuple(n), bc_lo=("shear", "periodic", "periodic"),
               bc_hi=("shear", "periodic", "periodic"), shape=(shape,) * 3, faces=faces)
    return Workload("shearing_box", dtype, [box],
                    dict(kind="shearbox_fargo" if fargo else "shearbox", Omega=Omega, q=q,
                         vertical_gravity=False),
                    "species", cell, off, mom,
                    [dict(rho=rho.astype(dt_np), vel=[vx.astype(dt_np), vy.astype(dt_np),
                                                       vz.astype(dt_np)])],
                    dt, nsteps, species=np.zeros(N, dtype=np.uint8),
                    species_tau=[tau_omega / Omega], species_mass=[m])


# Disk gas of the radial-drift test: rho and Omega(R, z) (Nelson et al. 2013)
def _disk_rho_omega(R, z, p=-1.0, q=-0.5, H0=0.1, R0=1.0, GM=1.0, rho0=1.0):
    r = np.sqrt(R * R + z * z)
    omk = np.sqrt(GM / R ** 3)
    H = H0 * (R / R0) ** ((q + 3.0) / 2.0)
    cs2 = (H * omk) ** 2
    rho = rho0 * (R / R0) ** p * np.exp(GM / cs2 * (1.0 / r - 1.0 / R))
    om = omk * np.sqrt((p + q) * (H / R) ** 2 + (1.0 + q) - q * R / r)
    return rho, om


def cylindrical_disk(n=(256, 512, 64), npart=2 ** 25, Rin=0.4, Rout=2.5, zh=0.15,
                     st_range=(1e-3, 10.0), eps=0.01, dt=0.003, nsteps=10, dtype="f32",
                     seed=2, shape="tsc") -> Workload:
    """(R, phi, z) grid with log-spaced R faces, periodic phi and z; gas in
    the equilibrium of the radial-drift test; particles uniform in R (surface
    density ~ 1/R), phi and z, on Keplerian-gas angular momentum, Stokes
    numbers log-uniform."""
    r = rng(seed)
    dt_np = np.float64 if dtype == "f64" else np.float32
    fR = Rin * (Rout / Rin) ** (np.arange(n[0] + 1) / n[0])
    fP = _uniform_faces(0.0, 2 * np.pi, n[1])
    fZ = _uniform_faces(-zh, zh, n[2])
    wR = np.diff(fR)
    # uniform in R: host cell with probability ~ its width, uniform offset
    ci = r.choice(n[0], size=npart, p=wR / wR.sum())
    cj = r.integers(0, n[1], size=npart)
    ck = r.integers(0, n[2], size=npart)
    off = _offsets(r, (npart, 3), dt_np)
    cell = (ci + n[0] * (cj + n[1] * ck)).astype(np.int32)
    Rp = 0.5 * (fR[ci] + fR[ci + 1]) + off[:, 0].astype(np.float64) * wR[ci]
    zp = 0.5 * (fZ[ck] + fZ[ck + 1]) + off[:, 2].astype(np.float64) * (fZ[1] - fZ[0])
    _, omp = _disk_rho_omega(Rp, zp)
    mom = np.zeros((npart, 3))
    mom[:, 1] = Rp * (Rp * omp)
    mom = mom.astype(dt_np)
    St = np.exp(r.uniform(np.log(st_range[0]), np.log(st_range[1]), size=npart)).astype(dt_np)
    gs = _ghost_shape(n, 3)
    Rg = _ghosted_centres(fR)[None, None, :]
    zg = _ghosted_centres(fZ)[:, None, None]
    rho, om = _disk_rho_omega(Rg, zg)
    rho = np.broadcast_to(rho, gs).copy()
    vphi = np.broadcast_to(Rg * om, gs).copy()
    zero = np.zeros(gs)
    dV = (0.5 * (fR[1:] ** 2 - fR[:-1] ** 2))[None, None, :] * (fP[1] - fP[0]) * (fZ[1] - fZ[0])
    mgas = float((rho[1:-1, 1:-1, 1:-1] * dV).sum())
    m = eps * mgas / npart
    box = dict(geom="cyl", ndim=3, n=tuple(n), bc_lo=("open", "periodic", "periodic"),
               bc_hi=("open", "periodic", "periodic"), shape=(shape,) * 3,
               faces=[fR, fP, fZ])
    return Workload("cylindrical_disk", dtype, [box], dict(kind="pointmass", GM=1.0),
                    "stokes", cell, off, mom,
                    [dict(rho=rho.astype(dt_np), vel=[zero.astype(dt_np), vphi.astype(dt_np),
                                                       zero.astype(dt_np)])],
                    dt, nsteps, drag=St, mass=np.full(npart, m, dtype=dt_np),
                    apply_feedback=False)


def rigid_disk(n_r=50, ratio=4, rb=0.5, re=5.5, nphi=4, nz=2, eps=1.0, shape="tsc",
               dtype="f64", seed=5) -> Workload:
    """Uniform dust density eps * rho_g (rho_g = 1) on a cylindrical grid
    with n_r uniform radial zones in [rb, re] (Sec. 4.3.1, particle
    assignment): N_p = ratio * n_r particles with radii from the inverse of
    the cumulative distribution, R(xi) = sqrt(xi (re^2 - rb^2) + rb^2)
    (Eq. Rxi_constant), xi = (k + 1/2) / N_p equally spaced; phi and z
    uniform random (periodic, nphi x nz zones); gas at rest."""
    r = rng(seed)
    dt_np = np.float64 if dtype == "f64" else np.float32
    npart = int(ratio * n_r)
    fR = _uniform_faces(rb, re, n_r)
    fP = _uniform_faces(0.0, 2 * np.pi, nphi)
    fZ = _uniform_faces(-0.5, 0.5, nz)
    xi = (np.arange(npart) + 0.5) / npart
    R = np.sqrt(xi * (re ** 2 - rb ** 2) + rb ** 2)
    phi = r.uniform(0.0, 2 * np.pi, npart)
    z = r.uniform(-0.5, 0.5, npart)
    idx, off = [], np.zeros((npart, 3))
    for d, (x, f) in enumerate(((R, fR), (phi, fP), (z, fZ))):
        i = np.clip(np.searchsorted(f, x, side="right") - 1, 0, len(f) - 2)
        o = (x - 0.5 * (f[i] + f[i + 1])) / (f[i + 1] - f[i])
        off[:, d] = np.clip(o, -0.5, np.nextafter(dt_np(0.5), dt_np(0)))
        idx.append(i)
    cell = (idx[0] + n_r * (idx[1] + nphi * idx[2])).astype(np.int32)
    n = (n_r, nphi, nz)
    gs = _ghost_shape(n, 3)
    zero = np.zeros(gs, dtype=dt_np)
    vol = np.pi * (re ** 2 - rb ** 2) * 1.0
    m = eps * 1.0 * vol / npart
    shp = (shape,) * 3 if isinstance(shape, str) else tuple(shape)   # a name or one per axis
    box = dict(geom="cyl", ndim=3, n=n, bc_lo=("open", "periodic", "periodic"),
               bc_hi=("open", "periodic", "periodic"), shape=shp, faces=[fR, fP, fZ])
    return Workload("rigid_disk", dtype, [box], dict(kind="none"), "tau", cell,
                    off.astype(dt_np), np.zeros((npart, 3), dtype=dt_np),
                    [dict(rho=np.ones(gs, dtype=dt_np), vel=[zero, zero, zero])], 0.01, 1,
                    drag=np.ones(npart, dtype=dt_np), mass=np.full(npart, m, dtype=dt_np),
                    apply_feedback=False)


def spherical_disk(n=(256, 128, 512), ppc=4, rin=0.5, rout=5.0, dth=0.3,
                   tau_range=(1e-6, 1.0), eps=0.01, dt=0.004, nsteps=10, dtype="f32",
                   seed=3, shape="tsc") -> Workload:
    """(r, theta, phi) grid, uniform in r and theta (pi/2 +- dth), periodic
    phi; the disk gas above in spherical components; particles uniform in
    (r, theta, phi), on the gas angular momentum, stopping times log-uniform
    (down to the stiff limit dt/tau ~ 4e3)."""
    r = rng(seed)
    dt_np = np.float64 if dtype == "f64" else np.float32
    fr = _uniform_faces(rin, rout, n[0])
    ft = _uniform_faces(np.pi / 2 - dth, np.pi / 2 + dth, n[1])
    fp = _uniform_faces(0.0, 2 * np.pi, n[2])
    ncell = n[0] * n[1] * n[2]
    N = ncell * ppc
    cell = r.integers(0, ncell, size=N).astype(np.int32)
    off = _offsets(r, (N, 3), dt_np)
    ci = cell % n[0]
    cj = (cell // n[0]) % n[1]
    rp = _active_centres(fr)[ci] + off[:, 0].astype(np.float64) * (fr[1] - fr[0])
    tp = _active_centres(ft)[cj] + off[:, 1].astype(np.float64) * (ft[1] - ft[0])
    Rp, zp = rp * np.sin(tp), rp * np.cos(tp)
    _, omp = _disk_rho_omega(Rp, zp)
    mom = np.zeros((N, 3))
    mom[:, 2] = Rp * (Rp * omp)
    mom = mom.astype(dt_np)
    tau = np.exp(r.uniform(np.log(tau_range[0]), np.log(tau_range[1]), size=N)).astype(dt_np)
    gs = _ghost_shape(n, 3)
    rg = _ghosted_centres(fr)[None, None, :]
    tg = _ghosted_centres(ft)[None, :, None]
    Rg, zg = rg * np.sin(tg), rg * np.cos(tg)
    rho, om = _disk_rho_omega(Rg, zg)
    rho = np.broadcast_to(rho, gs).copy()
    vphi = np.broadcast_to(Rg * om, gs).copy()
    zero = np.zeros(gs)
    dV = ((fr[1:] ** 3 - fr[:-1] ** 3) / 3.0)[None, None, :] * \
        (np.cos(ft[:-1]) - np.cos(ft[1:]))[None, :, None] * (fp[1] - fp[0])
    mgas = float((rho[1:-1, 1:-1, 1:-1] * dV).sum())
    m = eps * mgas / N
    box = dict(geom="sph", ndim=3, n=tuple(n), bc_lo=("open", "open", "periodic"),
               bc_hi=("open", "open", "periodic"), shape=(shape,) * 3, faces=[fr, ft, fp])
    return Workload("spherical_disk", dtype, [box], dict(kind="pointmass", GM=1.0), "tau",
                    cell, off, mom,
                    [dict(rho=rho.astype(dt_np), vel=[zero.astype(dt_np), zero.astype(dt_np),
                                                       vphi.astype(dt_np)])],
                    dt, nsteps, drag=tau, mass=np.full(N, m, dtype=dt_np),
                    apply_feedback=False)


def batched_boxes(sizes=(32, 48, 64, 80, 96, 128, 160, 192), max_per_species=32,
                  species_tau=(0.01, 0.1, 1.0, 10.0), eps_species=0.25, dt=0.01,
                  nsteps=100, dtype="f32", seed=4, shape="tsc", dx=1.0 / 64) -> Workload:
    """Independent periodic cubes of uneven sizes n^3 with the same cell
    width (1/64 by default, so a box spans n/64 per side); in every cell each
    species has U{1..max} particles at uniform random offsets, at rest; gas
    rho = 1 + 1e-3 N(0,1), v ~ U(-0.01, 0.01).  Species masses give a dust
    to gas ratio of eps_species per species at the mean count: with one
    species table for all boxes this holds in every box only because the
    cells have the same volume (in unit cubes of n^3 cells the ratio would
    grow as n^3, reaching 27 in a 192^3 box, where the explicit feedback of
    the impulse is unstable).

    Every box draws from its own stream (spawned from the seed), so a box's
    inputs do not depend on the other boxes: a subset of boxes generated
    alone (same sizes list, ``boxes=``) holds the same particles and gas as
    in the whole batch.  Offsets are drawn in the storage precision, so they
    lie in [-1/2, 1/2) exactly.  Arrays are allocated once at their full size
    (about 29 bytes per particle in FP32 for the 8-box batch of ~1e9
    particles)."""
    streams = np.random.SeedSequence(SEED0 + seed).spawn(len(sizes))
    dt_np = np.float64 if dtype == "f64" else np.float32
    ns = len(species_tau)
    ncells = [nb ** 3 for nb in sizes]
    bases = np.concatenate([[0], np.cumsum(ncells)]).astype(np.int64)
    # counts first (one draw per box stream), then every array at its size
    gens, counts = [], []
    for b in range(len(sizes)):
        r = np.random.Generator(np.random.PCG64(streams[b]))
        gens.append(r)
        counts.append(r.integers(1, max_per_species + 1, size=ncells[b] * ns, dtype=np.int32))
    nper = [int(c.sum(dtype=np.int64)) for c in counts]
    N = int(sum(nper))
    cell = np.empty(N, dtype=np.int32)
    species = np.empty(N, dtype=np.uint8)
    off = np.empty((N, 3), dtype=dt_np)
    boxes, gas = [], []
    at = 0
    for b, nb in enumerate(sizes):
        r = gens[b]
        n = (nb, nb, nb)
        faces = [_uniform_faces(0.0, nb * dx, nb) for _ in range(3)]
        boxes.append(dict(geom="cart", ndim=3, n=n, bc_lo=("periodic",) * 3,
                          bc_hi=("periodic",) * 3, shape=(shape,) * 3, faces=faces))
        k = np.repeat(np.arange(ncells[b] * ns, dtype=np.int32), counts[b])
        sl = slice(at, at + nper[b])
        np.floor_divide(k, ns, out=cell[sl])
        cell[sl] += np.int32(bases[b])
        species[sl] = k % ns
        del k
        off[sl] = r.random((nper[b], 3), dtype=dt_np)
        off[sl] -= dt_np(0.5)
        at += nper[b]
        gs = _ghost_shape(n, 3)
        rho = np.ones(gs)
        rho[1:-1, 1:-1, 1:-1] = 1.0 + 1e-3 * r.standard_normal((nb, nb, nb))
        vel = []
        for _ in range(3):
            v = np.zeros(gs)
            v[1:-1, 1:-1, 1:-1] = r.uniform(-0.01, 0.01, size=(nb, nb, nb))
            vel.append(v.astype(dt_np))
        gas.append(dict(rho=rho.astype(dt_np), vel=vel))
    mom = np.zeros((N, 3), dtype=dt_np)
    mean_count = 0.5 * (1 + max_per_species)
    mass = [eps_species * dx ** 3 / mean_count for _ in range(ns)]
    return Workload("batched_boxes", dtype, boxes, dict(kind="none"), "species", cell, off,
                    mom, gas, dt, nsteps, species=species, species_tau=list(species_tau),
                    species_mass=mass)


WORKLOADS = {
    "cart2d_periodic": cart2d_periodic,
    "shearing_box": shearing_box,
    "cylindrical_disk": cylindrical_disk,
    "spherical_disk": spherical_disk,
    "batched_boxes": batched_boxes,
}
