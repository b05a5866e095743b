"""Pins of the oracle's weights (not GPU).

The oracle evaluates every weight by Gauss-Legendre quadrature of its
definition (Eq. weight with Eq. shape_cart / shape_curv).  These tests pin it
to things other than itself: the quadrature rule against exact polynomial
integrals, the paper's closed forms (Eq. CIC_cylindrical, TSC_cylindrical,
CIC_spherical_r, TSC_spherical_r, CIC_spherical_theta with its minus branch
corrected), textbook b-spline overlaps in Cartesian coordinates, antiderivatives
derived here for the theta-TSC weights that the paper does not print, the
partition of unity (Eq. shape_norm), the zero-curvature limits (Sec. 3.4.1)
and brute force over every cell of small uniform grids.
"""
import math

import numpy as np
import pytest

import oracle as O

RNG = np.random.default_rng(7)


def test_gauss_legendre_integrates_polynomials_exactly():
    for deg in range(0, 32):
        coef = RNG.standard_normal(deg + 1)
        a, b = -0.7, 1.9
        exact = sum(c * (b ** (k + 1) - a ** (k + 1)) / (k + 1) for k, c in enumerate(coef))
        got = O.gl_integrate_poly(coef, a, b)
        assert abs(got - exact) <= 1e-12 * max(1.0, abs(exact)), deg


def _cart_box(shape, n=8):
    f = np.linspace(0.0, 1.0, n + 1)
    return O.Box("cart", (n, n, n), ("periodic",) * 3, ("periodic",) * 3, (shape,) * 3, [f] * 3)


@pytest.mark.parametrize("shape", ["cic", "tsc"])
def test_cartesian_weights_are_bspline_overlaps(shape):
    """Textbook CIC/TSC (overlap of a unit top hat / triangle with the cells)."""
    box = _cart_box(shape)
    for delta in np.concatenate([[-0.5, 0.0, 0.4999999], RNG.uniform(-0.5, 0.5, 50)]):
        i = 3
        xi = (i + 0.5 + delta) / 8
        w = O.weights_axis(box, 0, i, xi)
        if shape == "cic":
            ref = [max(0.0, -delta), 1 - abs(delta), max(0.0, delta)]
        else:
            ref = [0.5 * (0.5 - delta) ** 2, 0.75 - delta ** 2, 0.5 * (0.5 + delta) ** 2]
        np.testing.assert_allclose(w, ref, atol=1e-14)
        np.testing.assert_allclose(O.weights_paper("cart", shape, delta), ref, atol=1e-15)


@pytest.mark.parametrize("shape", ["cic", "tsc"])
def test_cylindrical_radial_weights_match_paper_closed_form(shape):
    R = np.linspace(0.3, 2.3, 41)
    dR = R[1] - R[0]
    box = O.Box("cyl", (40, 4, 4), ("open", "periodic", "periodic"),
                ("open", "periodic", "periodic"), (shape,) * 3,
                [R, np.linspace(0, 2 * np.pi, 5), np.linspace(-1, 1, 5)])
    for _ in range(60):
        i = int(RNG.integers(1, 39))
        delta = RNG.uniform(-0.5, 0.5)
        Ri = 0.5 * (R[i] + R[i + 1])
        w = O.weights_axis(box, 0, i, Ri + delta * dR)
        ref = O.weights_paper("cyl_r", shape, delta, Ri / dR)
        np.testing.assert_allclose(w, ref, atol=2e-14)


@pytest.mark.parametrize("shape", ["cic", "tsc"])
def test_spherical_radial_weights_match_paper_closed_form(shape):
    r = np.linspace(0.5, 5.0, 31)
    dr = r[1] - r[0]
    th = np.linspace(np.pi / 2 - 0.3, np.pi / 2 + 0.3, 9)
    box = O.Box("sph", (30, 8, 4), ("open", "open", "periodic"), ("open", "open", "periodic"),
                (shape,) * 3, [r, th, np.linspace(0, 2 * np.pi, 5)])
    for _ in range(60):
        i = int(RNG.integers(1, 29))
        delta = RNG.uniform(-0.5, 0.5)
        ri = 0.5 * (r[i] + r[i + 1])
        w = O.weights_axis(box, 0, i, ri + delta * dr)
        ref = O.weights_paper("sph_r", shape, delta, ri / dr)
        np.testing.assert_allclose(w, ref, atol=2e-14)


def test_theta_cic_weights_match_corrected_paper_form_and_printed_one_is_garbled():
    th = np.linspace(np.pi / 2 - 0.3, np.pi / 2 + 0.3, 17)
    dth = th[1] - th[0]
    box = O.Box("sph", (4, 16, 4), ("open", "open", "periodic"), ("open", "open", "periodic"),
                ("cic",) * 3, [np.linspace(1, 2, 5), th, np.linspace(0, 2 * np.pi, 5)])
    worst_printed = 0.0
    for _ in range(60):
        j = int(RNG.integers(0, 16))
        d = RNG.uniform(-0.5, 0.5) * dth
        tj = 0.5 * (th[j] + th[j + 1])
        w = O.weights_axis(box, 1, j, tj + d)
        ref = O.weights_paper("sph_theta", "cic", d, 0.0, th[j], th[j + 1])
        np.testing.assert_allclose(w, ref, atol=1e-12)
        if d < 0:
            # the minus branch as printed: [-cos(x_{i-1/2}) - cos(x_{i-1/2}+delta)] H(-delta)/den
            den = math.cos(th[j] + d) - math.cos(th[j + 1] + d)
            printed = (-math.cos(th[j]) - math.cos(th[j] + d)) / den
            worst_printed = max(worst_printed, abs(printed - w[0]))
    assert worst_printed > 1.0  # the printed sign cannot be right


def _theta_tsc_closed(tlo, thi, tp):
    """theta-TSC weights from antiderivatives of (1 -+ (t - tp)/D) sin t,
    D = thi - tlo; the tails beyond the host faces go to the neighbours."""
    D = thi - tlo
    norm = math.sin(tp) * 2.0 * (1.0 - math.cos(D)) / D
    # upper tail [thi, tp + D]: int (1 - (t-tp)/D) sin t
    A, B = thi, tp + D
    up = ((B - A) * math.cos(A) - (math.sin(B) - math.sin(A))) / D
    # lower tail [tp - D, tlo]: int (1 + (t-tp)/D) sin t
    A, B = tp - D, tlo
    lo = (-(B - A) * math.cos(B) + (math.sin(B) - math.sin(A))) / D
    return np.array([lo, norm - lo - up, up]) / norm


def test_theta_tsc_weights_match_antiderivatives():
    th = np.linspace(np.pi / 2 - 0.3, np.pi / 2 + 0.3, 129)
    box = O.Box("sph", (4, 128, 4), ("open", "open", "periodic"), ("open", "open", "periodic"),
                ("tsc",) * 3, [np.linspace(1, 2, 5), th, np.linspace(0, 2 * np.pi, 5)])
    for _ in range(60):
        j = int(RNG.integers(0, 128))
        d = RNG.uniform(-0.5, 0.5)
        tj = 0.5 * (th[j] + th[j + 1])
        D = th[j + 1] - th[j]
        w = O.weights_axis(box, 1, j, tj + d * D)
        ref = _theta_tsc_closed(th[j], th[j + 1], tj + d * D)
        np.testing.assert_allclose(w, ref, atol=5e-11)
        # a narrow polar cell is nearly flat: Cartesian TSC limit
        cart = [0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2]
        np.testing.assert_allclose(w, cart, atol=5 * D)


@pytest.mark.parametrize("geom,shape", [("cyl", "cic"), ("cyl", "tsc"), ("sph", "cic"),
                                        ("sph", "tsc")])
def test_zero_curvature_limit_gives_cartesian(geom, shape):
    kind = "cyl_r" if geom == "cyl" else "sph_r"
    for delta in RNG.uniform(-0.5, 0.5, 20):
        w = O.weights_paper(kind, shape, delta, 1e7)
        np.testing.assert_allclose(w, O.weights_paper("cart", shape, delta), atol=1e-6)


def _log_cyl_box(shape, n=24):
    fR = 0.4 * 6.25 ** (np.arange(n + 1) / n)
    return O.Box("cyl", (n, 4, 4), ("open", "periodic", "periodic"),
                 ("open", "periodic", "periodic"), (shape,) * 3,
                 [fR, np.linspace(0, 2 * np.pi, 5), np.linspace(-0.15, 0.15, 5)])


@pytest.mark.parametrize("shape", ["cic", "tsc"])
def test_log_radial_grid_weights(shape):
    """Non-uniform radial faces: partition of unity, and the host-cell reading
    reduces to the uniform closed form with nu = R_i / Delta R_i."""
    box = _log_cyl_box(shape)
    f = box.faces[0]
    for _ in range(40):
        i = int(RNG.integers(1, 23))
        delta = RNG.uniform(-0.5, 0.5)
        Ri, dR = 0.5 * (f[i] + f[i + 1]), f[i + 1] - f[i]
        w = O.weights_axis(box, 0, i, Ri + delta * dR)
        assert abs(w.sum() - 1.0) < 1e-13
        np.testing.assert_allclose(w, O.weights_paper("cyl_r", shape, delta, Ri / dR), atol=2e-14)


def test_partition_of_unity_everywhere():
    boxes = [
        (_cart_box("cic"), 0), (_cart_box("tsc"), 0), (_log_cyl_box("tsc"), 0),
        (O.Box("sph", (10, 16, 4), ("open", "open", "periodic"), ("open", "open", "periodic"),
               ("tsc", "tsc", "tsc"), [np.linspace(0.5, 5, 11),
                                       np.linspace(np.pi / 2 - 0.3, np.pi / 2 + 0.3, 17),
                                       np.linspace(0, 2 * np.pi, 5)]), 1),
    ]
    for box, d in boxes:
        f = box.faces[d]
        for _ in range(50):
            i = int(RNG.integers(1, len(f) - 2))
            xi = RNG.uniform(f[i], f[i + 1])
            assert abs(O.weights_axis(box, d, i, xi).sum() - 1.0) < 1e-13


@pytest.mark.parametrize("geom,shape", [("cart", "cic"), ("cart", "tsc"), ("cyl", "cic"),
                                        ("cyl", "tsc"), ("sph", "tsc")])
def test_stencil_equals_brute_force_overlap_on_uniform_grid(geom, shape):
    """On uniform grids the 3-zone weights equal the overlap of the shape with
    every cell of the axis, and every other cell gets exactly zero (Sec. 3.1)."""
    n = 12
    if geom == "cart":
        f = np.linspace(0, 1, n + 1)
        box = O.Box("cart", (n, n, n), ("periodic",) * 3, ("periodic",) * 3, (shape,) * 3, [f] * 3)
    elif geom == "cyl":
        f = np.linspace(0.2, 1.4, n + 1)
        box = O.Box("cyl", (n, n, n), ("open", "periodic", "periodic"),
                    ("open", "periodic", "periodic"), (shape,) * 3,
                    [f, np.linspace(0, 2 * np.pi, n + 1), np.linspace(0, 1, n + 1)])
    else:
        f = np.linspace(0.5, 2.5, n + 1)
        box = O.Box("sph", (n, n, n), ("open", "open", "periodic"), ("open", "open", "periodic"),
                    (shape,) * 3, [f, np.linspace(1.2, 1.9, n + 1), np.linspace(0, 2 * np.pi, n + 1)])
    for _ in range(20):
        i = int(RNG.integers(1, n - 1))
        xi = RNG.uniform(f[i], f[i + 1])
        w = O.weights_axis(box, 0, i, xi)
        full = np.array([O.weight_any_cell(box, 0, i, xi, k) for k in range(n)])
        np.testing.assert_allclose(full[i - 1:i + 2], w, atol=1e-14)
        mask = np.ones(n, bool)
        mask[i - 1:i + 2] = False
        assert np.all(full[mask] == 0.0)


def test_cell_volumes():
    fR = np.array([1.0, 2.0])
    box = O.Box("cyl", (1, 1, 1), ("open",) * 3, ("open",) * 3, ("cic",) * 3,
                [fR, np.array([0.0, 0.5]), np.array([0.0, 2.0])])
    assert abs(O.cell_volume(box, 0, 0, 0) - 0.5 * 3.0 * 0.5 * 2.0) < 1e-15
    box = O.Box("sph", (1, 1, 1), ("open",) * 3, ("open",) * 3, ("cic",) * 3,
                [np.array([1.0, 2.0]), np.array([0.0, np.pi]), np.array([0.0, 2 * np.pi])])
    assert abs(O.cell_volume(box, 0, 0, 0) - 4.0 / 3.0 * np.pi * 7.0) < 1e-13
