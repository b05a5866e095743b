"""Pins of the oracle's dust-density deposit (the particle mass spread with
the gather's weights, Sec. 3.4; Sec. 4.3.1 compares it with eps rho_g):
textbook weights at a cell centre, a one-per-cell lattice giving a uniform
density exactly, total mass over every stored cell in curvilinear boxes,
and the paper's particle-assignment comparison (Fig. distribution): with
radii from the inverse cumulative distribution, TSC leaves less grid noise
than CIC and its error falls as particles are added."""
import math

import numpy as np
import pytest

import oracle as O
from oracle.run import OracleRun
from paper_1908_10793_amd import synth

RNG = np.random.default_rng(21)


def _fold(box, rho):
    f = O.Fields(box, np.ones(box.ghosted_shape), [np.zeros(box.ghosted_shape)] * 3,
                 dep=[rho, np.zeros_like(rho), np.zeros_like(rho), np.zeros_like(rho)])
    O.fold_ghosts(box, O.Forces(), 0.0, f)
    return f.dep[0]


@pytest.mark.parametrize("shape", ["cic", "tsc"])
def test_mass_of_a_particle_at_a_cell_centre(shape):
    n, L = (6, 5, 4), (1.2, 0.5, 0.8)
    box = O.Box("cart", n, ("periodic",) * 3, ("periodic",) * 3, (shape,) * 3,
                [np.linspace(0, L[d], n[d] + 1) for d in range(3)])
    dx = [L[d] / n[d] for d in range(3)]
    x = np.array([[2.5 * dx[0], 2.5 * dx[1], 1.5 * dx[2]]])
    rho = np.zeros(box.ghosted_shape)
    O.deposit_mass(box, x, np.array([3.0]), np.ones(1, np.int32), rho)
    w1 = {"cic": [0.0, 1.0, 0.0], "tsc": [0.125, 0.75, 0.125]}[shape]
    want = np.zeros(box.ghosted_shape)
    dV = dx[0] * dx[1] * dx[2]
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                want[2 + c, 3 + b, 3 + a] = 3.0 * w1[a + 1] * w1[b + 1] * w1[c + 1] / dV
    np.testing.assert_allclose(rho, want, rtol=1e-13, atol=1e-14 * want.max())


@pytest.mark.parametrize("shape", ["cic", "tsc"])
def test_lattice_gives_uniform_density(shape):
    """One particle per cell, all at the same offset, on a periodic box:
    after the ghost fold every cell holds m / dV (partition of unity)."""
    n = (8, 6, 5)
    box = O.Box("cart", n, ("periodic",) * 3, ("periodic",) * 3, (shape,) * 3,
                [np.linspace(0, 1, n[d] + 1) for d in range(3)])
    i, j, k = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    o = RNG.uniform(-0.5, 0.5, 3)
    x = np.ascontiguousarray(np.stack([(i.ravel() + 0.5 + o[0]) / n[0],
                                       (j.ravel() + 0.5 + o[1]) / n[1],
                                       (k.ravel() + 0.5 + o[2]) / n[2]], 1) % 1.0)
    m = 0.7
    rho = np.zeros(box.ghosted_shape)
    O.deposit_mass(box, x, np.full(len(x), m), np.ones(len(x), np.int32), rho)
    rho = _fold(box, rho)
    dV = 1.0 / (n[0] * n[1] * n[2])
    np.testing.assert_allclose(rho[1:-1, 1:-1, 1:-1], m / dV, rtol=1e-13)


@pytest.mark.parametrize("geom", ["cyl", "sph"])
def test_total_mass_over_stored_cells(geom):
    if geom == "cyl":
        box = O.Box("cyl", (8, 12, 4), ("open", "periodic", "periodic"),
                    ("open", "periodic", "periodic"), ("tsc",) * 3,
                    [0.5 * np.geomspace(1.0, 3.0, 9), np.linspace(0, 2 * np.pi, 13),
                     np.linspace(-0.1, 0.1, 5)])
    else:
        box = O.Box("sph", (8, 8, 12), ("open", "open", "periodic"),
                    ("open", "open", "periodic"), ("tsc",) * 3,
                    [np.geomspace(0.6, 1.8, 9), np.linspace(0.9, math.pi - 0.9, 9),
                     np.linspace(0, 2 * np.pi, 13)])
    N = 300
    x = np.zeros((N, 3))
    for d in range(3):
        f = np.asarray(box.faces[d])
        lo, hi = (f[0], f[-1]) if box.bc_lo[d] == "periodic" else (f[2], f[-3])
        x[:, d] = RNG.uniform(lo, hi, N)
    mass = RNG.uniform(0.5, 2.0, N)
    rho = np.zeros(box.ghosted_shape)
    O.deposit_mass(box, x, mass, np.ones(N, np.int32), rho)
    total = 0.0
    n0, n1, n2 = box.n
    for k in range(-1, n2 + 1):
        for j in range(-1, n1 + 1):
            for i in range(-1, n0 + 1):
                total += O.cell_volume(box, i, j, k) * rho[k + 1, j + 1, i + 1]
    assert abs(total - mass.sum()) <= 1e-12 * mass.sum()


def rigid_disk_l1(ratio, shape, n_r=50):
    """Eq. rigid_err over the zones with 1 <= R <= 5, on the ring averages
    of the folded density (phi and z are periodic and uniform)."""
    w = synth.rigid_disk(n_r=n_r, ratio=ratio, shape=shape)
    run = OracleRun(w)
    box = run.boxes[0]
    rho = np.zeros(box.ghosted_shape)
    O.deposit_mass(box, run.x[0], run.mass[0], run.active[0], rho)
    rho = _fold(box, rho)
    ring = rho[1:-1, 1:-1, 1:-1].mean(axis=(0, 1))
    f = np.asarray(box.faces[0])
    Rc = 0.5 * (f[1:] + f[:-1])
    dV = 0.5 * (f[1:] ** 2 - f[:-1] ** 2)
    sel = (Rc >= 1.0) & (Rc <= 5.0)
    return float((np.abs(ring[sel] - 1.0) * dV[sel]).sum() / dV[sel].sum()), run


def test_rigid_disk_assignment_noise():
    """Fig. distribution: at N_p/N_R = 4 TSC leaves less noise than CIC, and
    the TSC error falls as N_p/N_R grows (4, 16, 64); the deposited mass
    equals the particles' total."""
    l1 = {s: rigid_disk_l1(4, s)[0] for s in ("cic", "tsc")}
    assert l1["tsc"] < l1["cic"], l1
    errs = [rigid_disk_l1(r, "tsc")[0] for r in (4, 16, 64)]
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 0.01, errs


def test_volume_weighting_interpolates_the_volume_coordinate():
    """Eq. CIC_vol: the two weights interpolate R^2 (and constants) exactly
    between the cell centres around the particle, are non-negative, and put
    everything on the host at its centre."""
    R = 0.5 * np.geomspace(1.0, 3.0, 13)
    box = O.Box("cyl", (12, 4, 2), ("open", "periodic", "periodic"),
                ("open", "periodic", "periodic"), ("vol", "tsc", "tsc"),
                [R, np.linspace(0, 2 * np.pi, 5), np.linspace(-0.1, 0.1, 3)])
    c = 0.5 * (R[1:] + R[:-1])
    cg = np.concatenate([[R[0] - 0.5 * (R[1] - R[0])], c, [R[-1] + 0.5 * (R[-1] - R[-2])]])
    for _ in range(200):
        i = int(RNG.integers(0, 12))
        xp = RNG.uniform(R[i], R[i + 1])
        w = O.weights_axis(box, 0, i, xp)
        assert np.all(w >= -1e-15)
        assert abs(w.sum() - 1.0) < 1e-14
        nodes = cg[i:i + 3]            # centres of cells i-1, i, i+1 (ghosts included)
        assert abs((w * nodes ** 2).sum() - xp ** 2) < 1e-13 * xp ** 2
        assert w[0] == 0.0 or w[2] == 0.0
    w = O.weights_axis(box, 0, 5, c[5])
    np.testing.assert_allclose(w, [0.0, 1.0, 0.0], atol=1e-15)


def test_rigid_disk_volume_weighting_is_noisier_than_tsc():
    """Fig. distribution: volume weighting (like CIC, two-zone support)
    leaves more assignment noise than TSC at N_p/N_R = 4."""
    vol = rigid_disk_l1(4, ("vol", "tsc", "tsc"))[0]
    tsc = rigid_disk_l1(4, "tsc")[0]
    assert vol > 2 * tsc, (vol, tsc)
