"""GPU parity of the Epstein stopping time (tau = C / rho_g with the gas
density weighted to the particle, Sec. 2) against the oracle through the C
ABI: the unfused step on Cartesian, shearing-box and cylindrical workloads
with a non-uniform gas density, the predictor's drag source, and the calls
that refuse it (fused step, autotuner, the phase kick)."""
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


def _epstein(name):
    """A workload turned to Epstein drag: C = tau rho_mean of its stopping
    times (so tau is unchanged where rho is the mean), per-particle masses,
    and a gas density with 20 % seeded variations."""
    if name == "cart2d":
        w = synth.cart2d_periodic(n=(24, 20), ppc=3, dtype="f64")
    elif name == "shearing_box":
        w = synth.shearing_box(n=(12, 10, 8), dtype="f32", dt=0.05)
    else:
        w = synth.cylindrical_disk(n=(16, 12, 8), npart=3001, dtype="f64", dt=0.05)
    rng = np.random.default_rng(12)
    if w.drag_mode == "species":
        sp = w.species.astype(np.int64)
        tau = np.asarray(w.species_tau, dtype=np.float64)[sp]
        mass = np.asarray(w.species_mass, dtype=np.float64)[sp]
    elif w.drag_mode == "stokes":
        # Stokes numbers turned into stopping times of 0.1 .. 10 (the stiff
        # regime has its own tests; here the density dependence is checked)
        tau = np.asarray(w.drag, dtype=np.float64) + 0.1
        mass = np.asarray(w.mass, dtype=np.float64)
        # the generator starts the particles on the gas rotation: give them a
        # 1 % slip so that the impulses are not pure rounding
        mom = np.array(w.mom, dtype=np.float64)
        mom[:, 1] *= 1.01
        w = dataclasses.replace(w, mom=mom.astype(np.asarray(w.mom).dtype))
    else:
        tau = np.asarray(w.drag, dtype=np.float64)
        mass = np.asarray(w.mass if w.mass is not None else np.full(w.n, w.species_mass[0]))
    gas = []
    for g in w.gas:
        rho = np.asarray(g["rho"]) * (1 + 0.2 * rng.uniform(-1, 1, np.shape(g["rho"])))
        gas.append(dict(rho=rho.astype(np.asarray(g["rho"]).dtype), vel=g["vel"]))
    rho_mean = float(np.mean([np.mean(g["rho"]) for g in gas]))
    dt_np = np.float64 if w.dtype == "f64" else np.float32
    return dataclasses.replace(w, drag_mode="epstein", drag=(tau * rho_mean).astype(dt_np),
                               mass=mass.astype(dt_np), species=None, gas=gas)


@pytest.mark.parametrize("name", ["cart2d", "shearing_box", "cylindrical_disk"])
def test_epstein_unfused_step_matches_oracle(name):
    dust = _dust()
    w = _epstein(name)
    ctx = dust.context_for(w)
    P, F = dust.upload(w, ctx)
    flags = dust.STEP_DIAG | (dust.STEP_APPLY_FEEDBACK if w.apply_feedback else 0)
    t = w.t0
    for s in range(2):
        st_in = download(ctx, P, F, w)
        ctx.step(P, F, w.dt, dust.forces_for(w, t), 1, flags)
        st_out = download(ctx, P, F, w)
        wi = workload_from_state(w, st_in, t)
        run = OracleRun(wi)
        run.step(1)
        rep = compare_step(wi, st_in, st_out, run, w.dtype, label=f"epstein {name} step {s}")
        print("[epstein]", rep, flush=True)
        t += w.dt


def test_epstein_drag_source_matches_oracle():
    import oracle as O
    dust = _dust()
    w = _epstein("cylindrical_disk")
    ctx = dust.context_for(w)
    P, F = dust.upload(w, ctx)
    fr = dust.forces_for(w, 0.0)
    ctx.fill_ghosts(F, fr, 0.0)
    for d in F["dep"]:
        d.zero_()
    ctx.drag_source(P, F, w.dt, fr)
    st = download(ctx, P, F, w)
    run = OracleRun(workload_from_state(w, st, 0.0))
    box = run.boxes[0]
    f = run.fields[0]
    O.drag_source(box, run.forces, run.mode[0], run.x[0], run.p[0], run.drag[0], run.mass[0],
                  run.active[0], f, w.dt)
    scale = max(np.abs(f.dep[c]).max() for c in range(3))   # v_R slips are zero here
    assert scale > 0
    for c in range(3):
        got, want = st["dep"][0][c].ravel(), f.dep[c].ravel()
        err = np.abs(got - want).max() / scale
        assert err <= 1e-12, (c, err)


def test_epstein_is_refused_where_unsupported():
    dust = _dust()
    w = _epstein("shearing_box")
    ctx = dust.context_for(w)
    P, F = dust.upload(w, ctx)
    fr = dust.forces_for(w, 0.0)
    with pytest.raises(dust.DustError) as e:
        ctx.step(P, F, w.dt, fr, 1, dust.STEP_FUSED)
    assert e.value.code == -5
    with pytest.raises(dust.DustError) as e:
        ctx.autotune(P, F, w.dt, fr, 0, steps=1)
    assert e.value.code == -5
    vg = [torch.zeros(w.n, dtype=ctx.real_dtype, device="cuda") for _ in range(3)]
    with pytest.raises(dust.DustError) as e:
        ctx.push_expmid(P, vg, w.dt, fr, dust.PHASE_KICK)
    assert e.value.code == -5
