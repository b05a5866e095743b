"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Every workload is one of the paper-shaped synthetic inputs at a size the
oracle finishes in seconds, spanning several fused tiles with ragged edges.
Each step is compared from identical inputs (see gpu_common).
"""
import dataclasses

import numpy as np
import pytest

from oracle.run import OracleRun
from paper_1908_10793_amd import synth

from gpu_common import TOL, compare_step, download, workload_from_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dust():
    from paper_1908_10793_amd import dust
    return dust


def small(name):
    if name == "cart2d_f64":       # the 2-D FP64 workload at its full size
        return synth.cart2d_periodic()
    if name == "shearing_box":
        return synth.shearing_box(n=(20, 20, 12), dt=0.05)
    if name == "shearing_box_fargo":   # orbital advection: residual velocities
        return synth.shearing_box(n=(20, 20, 12), dt=0.05, fargo=True)
    if name == "cylindrical_disk":
        return synth.cylindrical_disk(n=(24, 40, 12), npart=30000, dt=0.02)
    if name == "spherical_disk":
        return synth.spherical_disk(n=(24, 20, 36), ppc=2, dt=0.02)
    if name == "batched_boxes":
        return synth.batched_boxes(sizes=(6, 10, 13), max_per_species=4, dt=0.05)
    raise KeyError(name)


WORKLOADS = ["cart2d_f64", "shearing_box", "shearing_box_fargo", "cylindrical_disk", "spherical_disk",
             "batched_boxes"]


def _run(name, fused, nsteps=3, arith=None, tile=None, integrator=None):
    dust = _dust()
    w = small(name)
    if integrator:
        w = dataclasses.replace(w, forces={**w.forces, "integrator": integrator})
    print(f"[parity] {name} fused={fused} n={w.n}", flush=True)
    ctx = dust.context_for(w)
    if arith:
        ctx.set_arith(arith)
    if tile:
        ctx.set_tile(*tile)
    P, F = dust.upload(w, ctx)
    flags = dust.STEP_DIAG | (dust.STEP_APPLY_FEEDBACK if w.apply_feedback else 0)
    if fused:
        flags |= dust.STEP_FUSED
    t = w.t0
    reports = []
    for s in range(nsteps):
        st_in = download(ctx, P, F, w)
        ctx.step(P, F, w.dt, dust.forces_for(w, t), 1, flags)
        st_out = download(ctx, P, F, w)
        diag = ctx.status()
        wi = workload_from_state(w, st_in, t)
        run = OracleRun(wi)
        run.step(1)
        rep = compare_step(wi, st_in, st_out, run, w.dtype, label=f"{name} step {s}", diag=diag)
        # FP64 conservation on the device: sum_p J + sum_i dV D = 0
        scale = max(diag["sum_abs_j"], 1e-300)
        res = np.abs(np.array(diag["p_part"]) + np.array(diag["p_grid"])).max() / scale
        assert res < (1e-12 if w.dtype == "f64" else 2e-6), (name, s, res)
        assert not (set(diag["flag_names"]) - {"left_open", "tile_overflow"}), diag
        rep["cons"] = res
        reports.append(rep)
        t += w.dt
    print(reports, flush=True)
    return reports


@pytest.mark.parametrize("name", WORKLOADS)
def test_unfused_step_matches_oracle(name):
    """Ten steps, each against the oracle from the GPU state before it."""
    _run(name, fused=False, nsteps=10)


@pytest.mark.parametrize("name", WORKLOADS)
def test_fused_step_matches_oracle(name):
    """Ten steps (rebinning every step), each against the oracle from the GPU
    state before it."""
    _run(name, fused=True, nsteps=10)


def test_fused_with_other_tile_shapes():
    _run("shearing_box", fused=True, nsteps=2, tile=(4, 16, 4, 0))
    _run("batched_boxes", fused=True, nsteps=2, tile=(4, 4, 16, 0))
    _run("spherical_disk", fused=True, nsteps=1, tile=(8, 4, 8, 0))
    dust = _dust()
    ctx = dust.context_for(small("shearing_box"))
    with pytest.raises(dust.DustError) as e:
        ctx.set_tile(5, 3, 7, 0)
    assert e.value.code == -5


@pytest.mark.parametrize("name", ["shearing_box", "batched_boxes", "cylindrical_disk", "spherical_disk"])
def test_fused_fp64_arithmetic_variant_matches_oracle(name):
    """FP32 storage with FP64 per-particle arithmetic in the fused kernel."""
    _run(name, fused=True, nsteps=2, arith="f64")


@pytest.mark.parametrize("name", ["cart2d_f64", "shearing_box", "shearing_box_fargo", "batched_boxes"])
def test_semi_implicit_unfused_step_matches_oracle(name):
    """The semi-implicit comparison kick (Sec. 3.2) through the unfused step."""
    _run(name, fused=False, integrator="si")


def test_semi_implicit_is_refused_by_the_fused_step():
    dust = _dust()
    w = small("shearing_box")
    ctx = dust.context_for(w)
    P, F = dust.upload(w, ctx)
    fr = dust.forces_for(w)
    fr.integrator = dust.INTEGRATOR["si"]
    with pytest.raises(dust.DustError):
        ctx.step(P, F, w.dt, fr, 1, dust.STEP_FUSED)


@pytest.mark.parametrize("name", ["cylindrical_disk", "spherical_disk"])
def test_fused_fp32_curvilinear_steps_match_oracle(name):
    """FP32 per-particle arithmetic (the default) in curvilinear boxes over
    ten steps, each against the oracle from the GPU state before it.  As
    particles lock to the gas (tau down to 1e-6 in the spherical disk) their
    azimuthal slips fall towards the FP32 rounding of their angular momenta;
    the scale factors as two-word FP64 values at the particle and the FP64
    azimuthal gather keep those slips, and so the l_phi and energy deposits,
    within the bar (one FP32 word for the radius, or FP32 radial weights,
    leave 2e-5 to 3e-5 there by the fifth step)."""
    _run(name, fused=True, nsteps=10, arith="f32")
