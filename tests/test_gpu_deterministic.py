"""GPU tests of the deterministic mode (dust_ctx_set_deterministic): a step
against the oracle at the FP64 bar, the same bits on every run (eager and
graph), the stage calls equal to dust_step bit for bit, and a run resumed
from a saved state equal to the uninterrupted one."""
import dataclasses

import numpy as np
import pytest

from oracle.run import OracleRun
from paper_1908_10793_amd import synth

import test_gpu_drag_source as DS
import test_gpu_mass as MD
import test_gpu_parity
from gpu_common import TOL, compare_step, download, workload_from_state

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dust():
    from paper_1908_10793_amd import dust
    return dust


def workload(name, dtype="f64"):
    if name == "cart2d":
        return synth.cart2d_periodic(n=(32, 32), ppc=8, dtype=dtype)
    if name == "shearing_box":
        return synth.shearing_box(n=(16, 16, 12), dt=0.05, dtype=dtype)
    if name == "shearing_box_fargo":
        return synth.shearing_box(n=(16, 16, 12), dt=0.05, dtype=dtype, fargo=True)
    if name == "cylindrical_disk":
        return synth.cylindrical_disk(n=(24, 40, 12), npart=30000, dt=0.02, dtype=dtype)
    if name == "spherical_disk":
        return synth.spherical_disk(n=(24, 20, 36), ppc=2, dt=0.02, dtype=dtype)
    if name == "batched_boxes":
        return synth.batched_boxes(sizes=(6, 10, 13), max_per_species=4, dt=0.05, dtype=dtype)
    raise KeyError(name)


NAMES = ["cart2d", "shearing_box", "shearing_box_fargo", "cylindrical_disk", "spherical_disk",
         "batched_boxes"]
DIAG_KEYS = ["p_part", "p_grid", "e_part", "e_grid", "sum_abs_j", "max_cells_per_step", "n_removed",
             "flags", "steps"]


def _flags(dust, w):
    return dust.STEP_DIAG | (dust.STEP_APPLY_FEEDBACK if w.apply_feedback else 0)


def _same(P1, F1, P2, F2):
    """Every particle and field array equal bit for bit."""
    assert torch.equal(P1["cell"], P2["cell"])
    for d in range(len(P1["off"])):
        assert torch.equal(P1["off"][d], P2["off"][d]), d
        assert torch.equal(P1["mom"][d], P2["mom"][d]), d
    for key in ("vel", "dep"):
        for a, b in zip(F1[key], F2[key]):
            assert torch.equal(a, b), key
    assert torch.equal(F1["rho"], F2["rho"])


@pytest.mark.parametrize("name", test_gpu_parity.WORKLOADS)
def test_deterministic_step_matches_oracle(name):
    """The parity workloads (FP32 storage, the 2-D box FP64) at their bars."""
    dust = _dust()
    w = test_gpu_parity.small(name)
    print(f"[det] oracle {name} n={w.n}", flush=True)
    ctx = dust.context_for(w)
    ctx.set_deterministic(True)
    P, F = dust.upload(w, ctx)
    # the fused flag is ignored in this mode: the unfused chain runs
    flags = _flags(dust, w) | dust.STEP_FUSED
    t = w.t0
    for s in range(2):
        st_in = download(ctx, P, F, w)
        ctx.step(P, F, w.dt, dust.forces_for(w, t), 1, flags)
        st_out = download(ctx, P, F, w)
        diag = ctx.status()
        wi = workload_from_state(w, st_in, t)
        run = OracleRun(wi)
        run.step(1)
        compare_step(wi, st_in, st_out, run, w.dtype, label=f"det {name} step {s}", diag=diag)
        t += w.dt


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name", NAMES)
def test_runs_are_bitwise_identical(name, dtype):
    """Three steps, run three times from the same state (twice eagerly, once
    through a captured graph): the same bits, diagnostics included."""
    dust = _dust()
    w = workload(name, dtype)
    print(f"[det] repeat {name} {dtype} n={w.n}", flush=True)
    ctx = dust.context_for(w)
    ctx.set_deterministic(True)
    out = []
    for rep in range(3):
        P, F = dust.upload(w, ctx)
        ctx.status()
        flags = _flags(dust, w) | (dust.STEP_GRAPH if rep == 2 else 0)
        ctx.step(P, F, w.dt, dust.forces_for(w, w.t0), 3, flags)
        torch.cuda.synchronize()
        out.append((P, F, ctx.status()))
    P0, F0, d0 = out[0]
    assert d0["steps"] == 3 and d0["sum_abs_j"] > 0
    for P, F, d in out[1:]:
        _same(P0, F0, P, F)
        for k in DIAG_KEYS:
            assert d[k] == d0[k], (k, d[k], d0[k])


@pytest.mark.parametrize("name", ["shearing_box", "cylindrical_disk", "batched_boxes"])
def test_stage_calls_equal_step_bitwise(name):
    """fill, DRIFT1, gather, KICK, deposit, DRIFT2, fold, feedback through the
    stage calls give the bits of dust_step."""
    dust = _dust()
    w = workload(name)
    print(f"[det] stages {name} n={w.n}", flush=True)
    ctx = dust.context_for(w)
    ctx.set_deterministic(True)
    P1, F1 = dust.upload(w, ctx)
    P2, F2 = dust.upload(w, ctx)
    n = w.n
    t = w.t0
    fr = dust.forces_for(w, t)
    ctx.step(P1, F1, w.dt, fr, 1, dust.STEP_APPLY_FEEDBACK if w.apply_feedback else 0)
    vg = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    imp = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(4)]
    ctx.fill_ghosts(F2, fr, t + 0.5 * w.dt)
    for d in F2["dep"]:
        d.zero_()
    ctx.push_expmid(P2, None, w.dt, fr, dust.PHASE_DRIFT1)
    ctx.gather(P2, F2, None, vg)
    ctx.push_expmid(P2, vg, w.dt, fr, dust.PHASE_KICK, imp)
    ctx.deposit(P2, imp, F2)
    ctx.push_expmid(P2, None, w.dt, fr, dust.PHASE_DRIFT2)
    ctx.fold_ghosts(F2, fr, t + 0.5 * w.dt)
    if w.apply_feedback:
        ctx.apply_feedback(F2)
    torch.cuda.synchronize()
    assert torch.equal(P1["cell"], P2["cell"])
    for d in range(3):
        assert torch.equal(P1["off"][d], P2["off"][d])
        assert torch.equal(P1["mom"][d], P2["mom"][d])
    for a, b in zip(F1["dep"], F2["dep"]):
        assert torch.equal(a, b)
    for a, b in zip(F1["vel"], F2["vel"]):
        assert torch.equal(a, b)
    assert max(F1["dep"][c].abs().max().item() for c in range(4)) > 0


@pytest.mark.parametrize("name", ["shearing_box", "batched_boxes"])
def test_resume_from_saved_state_is_bitwise(name):
    """4 steps in one call equal 2 steps, a copy of the state through host
    memory into new device arrays (and a new context), and 2 more steps."""
    dust = _dust()
    w = workload(name)
    print(f"[det] resume {name} n={w.n}", flush=True)
    flags = _flags(dust, w)
    ctx = dust.context_for(w)
    ctx.set_deterministic(True)
    P1, F1 = dust.upload(w, ctx)
    ctx.step(P1, F1, w.dt, dust.forces_for(w, w.t0), 4, flags)
    P2, F2 = dust.upload(w, ctx)
    ctx.step(P2, F2, w.dt, dust.forces_for(w, w.t0), 2, flags)
    t = w.t0
    for _ in range(2):
        t += w.dt   # the same additions as the step's own clock
    saved = download(ctx, P2, F2, w)
    w2 = workload_from_state(w, saved, t)
    ctx2 = dust.context_for(w2)
    ctx2.set_deterministic(True)
    P3, F3 = dust.upload(w2, ctx2)
    ctx2.step(P3, F3, w.dt, dust.forces_for(w2, t), 2, flags)
    torch.cuda.synchronize()
    assert torch.equal(P1["cell"], P3["cell"])
    for d in range(3):
        assert torch.equal(P1["off"][d], P3["off"][d])
        assert torch.equal(P1["mom"][d], P3["mom"][d])
    # active gas (the ghosts are refilled at the start of every step)
    for a, b in zip(F1["vel"], F3["vel"]):
        assert torch.equal(a, b)
    for a, b in zip(F1["dep"], F3["dep"]):
        assert torch.equal(a, b)


def test_set_deterministic_rejects_other_values():
    dust = _dust()
    w = workload("shearing_box")
    ctx = dust.context_for(w)
    L = dust.load_library()
    assert L.dust_ctx_set_deterministic(ctx.handle, 2) == -1   # DUST_EINVAL
    assert L.dust_ctx_set_deterministic(ctx.handle, 0) == 0


def test_autotune_is_refused_in_deterministic_mode():
    dust = _dust()
    w = workload("shearing_box", "f32")
    ctx = dust.context_for(w)
    ctx.set_deterministic(True)
    P, F = dust.upload(w, ctx)
    with pytest.raises(dust.DustError) as e:
        ctx.autotune(P, F, w.dt, dust.forces_for(w), steps=1)
    assert e.value.code == -5   # DUST_EUNSUPPORTED


SOURCE_CASES = [("shearing_box", "f32"), ("shearing_box", "f64"), ("cylindrical_disk", "f64"),
                ("spherical_disk", "f64"), ("batched", "f32"), ("cart2d", "f64")]


@pytest.mark.parametrize("name,dtype", SOURCE_CASES)
def test_deterministic_sources_repeat_and_match_oracle(name, dtype):
    """dust_drag_source and dust_deposit_mass in the deterministic mode: the
    same bits on a second run, and the oracle's source and density at the
    bars of their own tests (particles in a shuffled order)."""
    dust = _dust()
    w = DS._workload(name, dtype)
    perm = np.random.default_rng(12).permutation(w.n)
    kw = dict(cell=w.cell[perm], off=w.off[perm], mom=w.mom[perm])
    for k in ("drag", "mass", "species"):
        if getattr(w, k) is not None:
            kw[k] = getattr(w, k)[perm]
    w = dataclasses.replace(w, **kw)
    print(f"[det] sources {name} {dtype} n={w.n}", flush=True)
    t, dt = 0.3, float(w.dt)
    ctx = dust.context_for(w)
    ctx.set_deterministic(True)
    runs = []
    for rep in range(2):
        P, F = dust.upload(w, ctx)
        fr = dust.forces_for(w, t)
        ctx.fill_ghosts(F, fr, t)
        for d in F["dep"]:
            d.zero_()
        ctx.drag_source(P, F, dt, fr)
        rho = torch.zeros_like(F["dep"][0])
        ctx.deposit_mass(P, rho)
        torch.cuda.synchronize()
        runs.append((P, F, rho))
    (P0, F0, r0), (P1, F1, r1) = runs
    for a, b in zip(F0["dep"], F1["dep"]):
        assert torch.equal(a, b)
    assert torch.equal(r0, r1)
    st = download(ctx, P0, F0, w)
    DS._compare(w, st, DS._oracle_source(w, st, t, dt), TOL[dtype], f"det source {name} {dtype}")
    for d in F0["dep"]:
        d.zero_()
    F0["dep"][0].copy_(r0)
    st = download(ctx, P0, F0, w)
    MD._compare(w, st, TOL[dtype], f"det density {name} {dtype}")
