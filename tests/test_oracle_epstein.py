"""Pins of the oracle's Epstein stopping time (Sec. 2: tau_s = rho_s a /
(rho_g v_t), with rho_g the gas density weighted to the particle and the
particle's drag value holding rho_s a / v_t): in gas of uniform density it
is the plain stopping-time mode with tau = C / rho; in a non-uniform
density, the drag-only kick relaxes exactly with the rate rho~/C, rho~ from
the textbook TSC weights at the particle; and the predictor's drag source
uses the same rate."""
import math

import numpy as np

import oracle as O

RNG = np.random.default_rng(31)


def _box(n=(8, 6)):
    faces = [np.linspace(0, 1, n[0] + 1), np.linspace(0, 0.75, n[1] + 1)]
    return O.Box("cart", n, ("periodic",) * 2, ("periodic",) * 2, ("tsc",) * 2, faces, ndim=2)


def _particles(N):
    x = np.zeros((N, 3))
    x[:, 0] = RNG.uniform(0, 1, N)
    x[:, 1] = RNG.uniform(0, 0.75, N)
    p = np.zeros((N, 3))
    p[:, :2] = RNG.standard_normal((N, 2))
    return x, p


def test_uniform_density_equals_stopping_time_mode():
    box = _box()
    gs = box.ghosted_shape
    rho0, tau0, dt = 2.5, 0.07, 0.05
    vel = [RNG.standard_normal(gs), RNG.standard_normal(gs)]
    N = 60
    x0, p0 = _particles(N)
    mass = RNG.uniform(0.5, 2.0, N)
    out = {}
    for mode, dval in (("tau", tau0), ("epstein", tau0 * rho0)):
        x, p = x0.copy(), p0.copy()
        f = O.Fields(box, np.full(gs, rho0), [v.copy() for v in vel])
        O.step(box, O.Forces(), mode, x, p, np.full(N, dval), mass, np.ones(N, np.int32), f, dt, 0.0)
        out[mode] = (x, p, [d.copy() for d in f.dep[:3]])
    np.testing.assert_allclose(out["epstein"][0], out["tau"][0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(out["epstein"][1], out["tau"][1], rtol=0, atol=1e-13)
    for a, b in zip(out["epstein"][2], out["tau"][2]):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(b).max())


def test_drag_only_kick_relaxes_with_weighted_density():
    """One particle reaching a cell centre at the half step, uniform gas
    velocity U, non-uniform density: v^{n+1} = U + (v^n - U) exp(-dt rho~/C)
    with rho~ = sum of the textbook TSC weights (1/8, 3/4, 1/8)^2 times rho."""
    box = _box()
    gs = box.ghosted_shape
    rho = RNG.uniform(0.5, 3.0, gs)
    U = np.array([0.3, -0.2])
    C, dt = 0.4, 0.05
    p0 = np.array([[0.7, 0.4, 0.0]])
    centre = np.array([3.5 / 8, 2.5 * 0.125, 0.0])      # cell (3, 2)
    x = (centre - 0.5 * dt * p0[0])[None, :].copy()
    p = p0.copy()
    f = O.Fields(box, rho.copy(), [np.full(gs, U[0]), np.full(gs, U[1])])
    O.step(box, O.Forces(), "epstein", x, p, np.array([C]), np.array([1.0]), np.ones(1, np.int32),
           f, dt, 0.0, fill_ghosts=False)
    w = [0.125, 0.75, 0.125]
    rt = sum(w[a] * w[b] * rho[0, 2 + 1 + b - 1, 3 + 1 + a - 1] for a in range(3) for b in range(3))
    want = U + (p0[0, :2] - U) * math.exp(-dt * rt / C)
    np.testing.assert_allclose(p[0, :2], want, rtol=1e-13)


def test_drag_source_uses_weighted_density():
    """The predictor's source with Epstein drag equals the stopping-time
    mode with each particle's tau = C / rho~ (rho~ gathered at x^n)."""
    box = _box()
    gs = box.ghosted_shape
    rho = RNG.uniform(0.5, 3.0, gs)
    vel = [RNG.standard_normal(gs), RNG.standard_normal(gs)]
    N = 40
    x, p = _particles(N)
    mass = RNG.uniform(0.5, 2.0, N)
    C = RNG.uniform(0.02, 0.5, N)
    dt = 0.03
    f1 = O.Fields(box, rho.copy(), [v.copy() for v in vel])
    O.drag_source(box, O.Forces(), "epstein", x, p, C, mass, np.ones(N, np.int32), f1, dt)
    r_p, _ = O.gather(box, f1, x)
    f2 = O.Fields(box, rho.copy(), [v.copy() for v in vel])
    O.drag_source(box, O.Forces(), "tau", x, p, C / r_p, mass, np.ones(N, np.int32), f2, dt)
    for c in range(2):
        np.testing.assert_allclose(f1.dep[c], f2.dep[c], rtol=0, atol=1e-13 * np.abs(f2.dep[c]).max())
