"""Thin Python binding of libdust.so (include/dust.h), same names as the C ABI.

Argument marshalling only: every step of the hot path runs in the HIP
kernels of libdust.so.  Arrays are torch tensors on the GPU (device memory
and streams come from PyTorch); this module checks dtype / device /
contiguity, passes raw pointers, and raises DustError on any non-zero status.
There is no CPU fallback: if the library is missing or no GPU is present the
calls fail.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdust.so")

CART, CYL, SPH = 0, 1, 2
CIC, TSC = 0, 1
F32, F64 = 0, 1
ARITH_F64, ARITH_F32 = 0, 1
BC = {"periodic": 0, "shear": 1, "open": 2}
GEOM = {"cart": CART, "cyl": CYL, "sph": SPH}
SHAPE = {"cic": CIC, "tsc": TSC, "vol": 2}   # vol: Eq. CIC_vol, cylindrical radius only
FORCE = {"none": 0, "shearbox": 1, "pointmass": 2, "const": 3, "shearbox_fargo": 4}
DRAG = {"tau": 0, "stokes": 1, "species": 2, "epstein": 3}
PHASE_DRIFT1, PHASE_KICK, PHASE_DRIFT2 = 1, 2, 4
BIN_CELL, BIN_TILE = 0, 1
BIN_NOALLOC_MAX = 1 << 20   # particles of one dust_bin_noalloc call
STEP_APPLY_FEEDBACK, STEP_FUSED, STEP_DIAG, STEP_GRAPH, STEP_NO_FILL = 1, 2, 4, 8, 16
FLAG_NAMES = {1: "nonfinite", 2: "offset_range", 4: "cfl", 8: "left_open", 16: "tile_overflow",
              32: "bad_cell"}


def STEP_REBIN_EVERY(k: int) -> int:
    return (int(k) & 0xFF) << 8


class DustError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dust error {code}: {msg}")
        self.code = code


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


class dust_box_t(ctypes.Structure):
    _fields_ = [("geom", ctypes.c_int32), ("ndim", ctypes.c_int32), ("n", ctypes.c_int32 * 3),
                ("bc_lo", ctypes.c_int32 * 3), ("bc_hi", ctypes.c_int32 * 3),
                ("shape", ctypes.c_int32 * 3), ("faces", _dp * 3)]


class dust_forces_t(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("vertical_gravity", ctypes.c_int32),
                ("Omega", ctypes.c_double), ("q", ctypes.c_double), ("GM", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("t", ctypes.c_double), ("integrator", ctypes.c_int32)]


class dust_particles_t(ctypes.Structure):
    _fields_ = [("cell", _vp), ("off", _vp * 3), ("mom", _vp * 3), ("drag", _vp), ("mass", _vp),
                ("species", _vp), ("id", _vp), ("n", ctypes.c_int64)]


class dust_fields_t(ctypes.Structure):
    _fields_ = [("rho", _vp), ("vel", _vp * 3), ("dep", _vp * 4)]


class dust_diag_t(ctypes.Structure):
    _fields_ = [("p_part", ctypes.c_double * 3), ("p_grid", ctypes.c_double * 3),
                ("e_part", ctypes.c_double), ("e_grid", ctypes.c_double),
                ("sum_abs_j", ctypes.c_double), ("max_cells_per_step", ctypes.c_double),
                ("n_removed", ctypes.c_int64), ("n_fallback", ctypes.c_int64),
                ("flags", ctypes.c_int32), ("steps", ctypes.c_int32)]


EXPORTS = ["dust_ctx_create", "dust_ctx_destroy", "dust_ctx_set_arith", "dust_ctx_set_deterministic",
           "dust_ctx_set_tile",
           "dust_ctx_grid_size", "dust_ctx_status", "dust_last_error", "dust_bin", "dust_bin_noalloc",
           "dust_fill_ghosts", "dust_gather", "dust_push_expmid", "dust_deposit",
           "dust_fold_ghosts", "dust_apply_feedback", "dust_step", "dust_ctx_set_profile",
           "dust_ctx_profile", "dust_ctx_autotune", "dust_drag_source",
           "dust_deposit_mass"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libdust.so (ctypes); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1908_10793_amd.build.build()")
    L = ctypes.CDLL(path)
    i32 = ctypes.c_int32
    L.dust_last_error.restype = ctypes.c_char_p
    L.dust_ctx_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(dust_box_t),
                                  ctypes.c_int, i32, i32, _dp, _dp, ctypes.c_int]
    L.dust_ctx_destroy.argtypes = [_vp]
    L.dust_ctx_set_arith.argtypes = [_vp, i32]
    L.dust_ctx_set_deterministic.argtypes = [_vp, i32]
    L.dust_ctx_set_tile.argtypes = [_vp, i32, i32, i32, i32]
    L.dust_ctx_grid_size.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.dust_ctx_status.argtypes = [_vp, ctypes.POINTER(dust_diag_t)]
    L.dust_ctx_set_profile.argtypes = [_vp, i32]
    L.dust_ctx_profile.argtypes = [_vp, ctypes.POINTER(ctypes.c_float), i32,
                                   ctypes.POINTER(ctypes.c_int32)]
    L.dust_bin.argtypes = [_vp, ctypes.POINTER(dust_particles_t), i32, _vp, _vp, ctypes.c_int, _vp]
    L.dust_bin_noalloc.argtypes = L.dust_bin.argtypes
    L.dust_fill_ghosts.argtypes = [_vp, ctypes.POINTER(dust_fields_t),
                                   ctypes.POINTER(dust_forces_t), ctypes.c_double, _vp]
    L.dust_fold_ghosts.argtypes = L.dust_fill_ghosts.argtypes
    L.dust_gather.argtypes = [_vp, ctypes.POINTER(dust_particles_t), ctypes.POINTER(dust_fields_t),
                              _vp, _vp * 3, _vp]
    L.dust_push_expmid.argtypes = [_vp, ctypes.POINTER(dust_particles_t), _vp * 3, ctypes.c_double,
                                   ctypes.POINTER(dust_forces_t), i32, _vp * 4, _vp]
    L.dust_deposit.argtypes = [_vp, ctypes.POINTER(dust_particles_t), _vp * 4,
                               ctypes.POINTER(dust_fields_t), _vp]
    L.dust_apply_feedback.argtypes = [_vp, ctypes.POINTER(dust_fields_t), _vp]
    L.dust_deposit_mass.argtypes = [_vp, ctypes.POINTER(dust_particles_t), _vp, _vp]
    L.dust_drag_source.argtypes = [_vp, ctypes.POINTER(dust_particles_t),
                                   ctypes.POINTER(dust_fields_t), ctypes.c_double,
                                   ctypes.POINTER(dust_forces_t), _vp]
    L.dust_step.argtypes = [_vp, ctypes.POINTER(dust_particles_t), ctypes.POINTER(dust_fields_t),
                            ctypes.c_double, ctypes.POINTER(dust_forces_t), i32, i32, _vp]
    L.dust_ctx_autotune.argtypes = [_vp, ctypes.POINTER(dust_particles_t),
                                    ctypes.POINTER(dust_fields_t), ctypes.c_double,
                                    ctypes.POINTER(dust_forces_t), i32, i32,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float),
                                    _vp]
    for name in EXPORTS:
        if name != "dust_last_error":
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(code: int):
    if code != 0:
        msg = load_library().dust_last_error().decode(errors="replace")
        raise DustError(code, msg)


def _ptr(t, dtype=None, what="array"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{what}: tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what}: dtype {t.dtype}, expected {dtype}")
    return t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


INTEGRATOR = {"em": 0, "si": 1}


def forces_t(kind="none", Omega=0.0, q=0.0, GM=0.0, vertical_gravity=False, g=(0.0, 0.0, 0.0),
             t=0.0, integrator="em") -> dust_forces_t:
    f = dust_forces_t()
    f.kind = FORCE[kind] if isinstance(kind, str) else int(kind)
    f.integrator = INTEGRATOR[integrator] if isinstance(integrator, str) else int(integrator)
    f.vertical_gravity = int(bool(vertical_gravity))
    f.Omega, f.q, f.GM, f.t = float(Omega), float(q), float(GM), float(t)
    for d in range(3):
        f.g[d] = float(g[d])
    return f


class Context:
    """A dust context (dust_ctx_*), holding the boxes and the device workspace.

    boxes: list of dicts with keys geom ('cart'|'cyl'|'sph'), ndim, n (3
    ints), bc_lo, bc_hi (names per axis), shape ('cic'|'tsc' per axis),
    faces (FP64 arrays, n[d]+1 each)."""

    def __init__(self, boxes, prec="f32", drag_mode="tau", species_tau=None, species_mass=None,
                 device=0):
        import numpy as np
        L = load_library()
        self._faces = []
        arr = (dust_box_t * len(boxes))()
        for b, bd in enumerate(boxes):
            nd = int(bd["ndim"])
            arr[b].geom = GEOM[bd["geom"]]
            arr[b].ndim = nd
            for d in range(3):
                arr[b].n[d] = int(bd["n"][d]) if d < nd else 1
                arr[b].bc_lo[d] = BC[bd["bc_lo"][d]] if d < nd else 0
                arr[b].bc_hi[d] = BC[bd["bc_hi"][d]] if d < nd else 0
                arr[b].shape[d] = SHAPE[bd["shape"][d]] if d < nd else 0
                if d < nd:
                    f = np.ascontiguousarray(bd["faces"][d], dtype=np.float64)
                    self._faces.append(f)
                    arr[b].faces[d] = f.ctypes.data_as(_dp)
        self.prec = F64 if prec in ("f64", F64) else F32
        self.ndim = max(int(b["ndim"]) for b in boxes)
        self.nc = max(int(b["ndim"]) if b["geom"] == "cart" else 3 for b in boxes)
        nsp = 0
        tau_p = mass_p = None
        self._tables = []
        if species_tau is not None:
            t = np.ascontiguousarray(species_tau, dtype=np.float64)
            self._tables.append(t)
            tau_p = t.ctypes.data_as(_dp)
            nsp = len(t)
        if species_mass is not None:
            m = np.ascontiguousarray(species_mass, dtype=np.float64)
            self._tables.append(m)
            mass_p = m.ctypes.data_as(_dp)
            nsp = max(nsp, len(m))
        h = _vp()
        _check(L.dust_ctx_create(ctypes.byref(h), int(device), arr, len(boxes), self.prec,
                                 DRAG[drag_mode] if isinstance(drag_mode, str) else int(drag_mode),
                                 tau_p, mass_p, nsp))
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load_library().dust_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def real_dtype(self):
        import torch
        return torch.float64 if self.prec == F64 else torch.float32

    def grid_size(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(load_library().dust_ctx_grid_size(self.handle, ctypes.byref(a), ctypes.byref(b),
                                                 None))
        return a.value, b.value

    def set_arith(self, arith: str):
        """Push arithmetic of an FP32 context: "f32" (default) or "f64"."""
        if arith not in ("f32", "f64"):
            raise ValueError(f"arith must be 'f32' or 'f64', not {arith!r}")
        _check(load_library().dust_ctx_set_arith(self.handle, ARITH_F32 if arith == "f32" else ARITH_F64))

    def set_deterministic(self, on: bool = True):
        """Deterministic mode: the same bits on every run (unfused step,
        sorted deposit without float atomics, fixed-order sums)."""
        _check(load_library().dust_ctx_set_deterministic(self.handle, 1 if on else 0))

    def set_tile(self, tx=0, ty=0, tz=0, slack=0):
        _check(load_library().dust_ctx_set_tile(self.handle, tx, ty, tz, slack))

    def set_profile(self, max_launches: int):
        _check(load_library().dust_ctx_set_profile(self.handle, int(max_launches)))

    def profile(self, max_out: int = 4096):
        buf = (ctypes.c_float * max_out)()
        cnt = ctypes.c_int32()
        _check(load_library().dust_ctx_profile(self.handle, buf, max_out, ctypes.byref(cnt)))
        return [buf[i] for i in range(cnt.value)]

    def status(self) -> dict:
        d = dust_diag_t()
        _check(load_library().dust_ctx_status(self.handle, ctypes.byref(d)))
        return dict(p_part=list(d.p_part), p_grid=list(d.p_grid), e_part=d.e_part,
                    e_grid=d.e_grid, sum_abs_j=d.sum_abs_j,
                    max_cells_per_step=d.max_cells_per_step, n_removed=d.n_removed,
                    n_fallback=d.n_fallback, flags=d.flags, steps=d.steps,
                    flag_names=[v for k, v in FLAG_NAMES.items() if d.flags & k])

    # ------------------------------------------------------------ marshalling
    def particles_t(self, P: dict) -> dust_particles_t:
        import torch
        rd = self.real_dtype
        p = dust_particles_t()
        p.cell = _ptr(P["cell"], torch.int32, "cell")
        n = P["cell"].numel()
        for d in range(3):
            o = P["off"][d] if d < len(P["off"]) else None
            m = P["mom"][d] if d < len(P["mom"]) else None
            p.off[d] = _ptr(o, rd, f"off[{d}]")
            p.mom[d] = _ptr(m, rd, f"mom[{d}]")
        p.drag = _ptr(P.get("drag"), rd, "drag")
        p.mass = _ptr(P.get("mass"), rd, "mass")
        p.species = _ptr(P.get("species"), torch.uint8, "species")
        p.id = _ptr(P.get("id"), torch.int32, "id")
        p.n = n
        return p

    def fields_t(self, F: dict) -> dust_fields_t:
        rd = self.real_dtype
        f = dust_fields_t()
        f.rho = _ptr(F.get("rho"), rd, "rho")
        vel = F.get("vel", [])
        dep = F.get("dep", [])
        for d in range(3):
            f.vel[d] = _ptr(vel[d] if d < len(vel) else None, rd, f"vel[{d}]")
        for d in range(4):
            f.dep[d] = _ptr(dep[d] if d < len(dep) else None, rd, f"dep[{d}]")
        return f

    # ------------------------------------------------------------ entry points
    def bin(self, P, key_mode="cell", perm=None, bin_start=None, apply=False, stream=None):
        import torch
        pt = self.particles_t(P)
        _check(load_library().dust_bin(self.handle, ctypes.byref(pt),
                                       BIN_TILE if key_mode == "tile" else BIN_CELL,
                                       _ptr(perm, torch.int32, "perm"),
                                       _ptr(bin_start, torch.int64, "bin_start"), int(apply),
                                       _stream(stream)))

    def bin_noalloc(self, P, key_mode="cell", perm=None, bin_start=None, apply=False, stream=None):
        """bin() through the allocation-free entry point (at most
        BIN_NOALLOC_MAX particles)."""
        import torch
        pt = self.particles_t(P)
        _check(load_library().dust_bin_noalloc(self.handle, ctypes.byref(pt),
                                               BIN_TILE if key_mode == "tile" else BIN_CELL,
                                               _ptr(perm, torch.int32, "perm"),
                                               _ptr(bin_start, torch.int64, "bin_start"), int(apply),
                                               _stream(stream)))

    def fill_ghosts(self, F, forces: dust_forces_t, t: float, stream=None):
        f = self.fields_t(F)
        _check(load_library().dust_fill_ghosts(self.handle, ctypes.byref(f), ctypes.byref(forces),
                                               float(t), _stream(stream)))

    def fold_ghosts(self, F, forces: dust_forces_t, t: float, stream=None):
        f = self.fields_t(F)
        _check(load_library().dust_fold_ghosts(self.handle, ctypes.byref(f), ctypes.byref(forces),
                                               float(t), _stream(stream)))

    def gather(self, P, F, rho_p, vg_p, stream=None):
        rd = self.real_dtype
        pt, f = self.particles_t(P), self.fields_t(F)
        vg = (_vp * 3)(*[_ptr(vg_p[d] if d < len(vg_p) else None, rd, "vg_p") for d in range(3)])
        _check(load_library().dust_gather(self.handle, ctypes.byref(pt), ctypes.byref(f),
                                          _ptr(rho_p, rd, "rho_p"), vg, _stream(stream)))

    def push_expmid(self, P, vg_p, dt, forces: dust_forces_t, phases, impulse=None, stream=None):
        rd = self.real_dtype
        pt = self.particles_t(P)
        vg_p = vg_p or []
        impulse = impulse or []
        vg = (_vp * 3)(*[_ptr(vg_p[d] if d < len(vg_p) else None, rd, "vg_p") for d in range(3)])
        imp = (_vp * 4)(*[_ptr(impulse[d] if d < len(impulse) else None, rd, "impulse")
                          for d in range(4)])
        _check(load_library().dust_push_expmid(self.handle, ctypes.byref(pt), vg, float(dt),
                                               ctypes.byref(forces), int(phases), imp,
                                               _stream(stream)))

    def deposit(self, P, impulse, F, stream=None):
        rd = self.real_dtype
        pt, f = self.particles_t(P), self.fields_t(F)
        imp = (_vp * 4)(*[_ptr(impulse[d] if d < len(impulse) else None, rd, "impulse")
                          for d in range(4)])
        _check(load_library().dust_deposit(self.handle, ctypes.byref(pt), imp, ctypes.byref(f),
                                           _stream(stream)))

    def drag_source(self, P, F, dt, forces: dust_forces_t, stream=None):
        """dust_drag_source: the predictor's drag force density (Eq. f_D with
        tau <- max(tau, dt)) added to F["dep"]'s momentum channels."""
        pt, f = self.particles_t(P), self.fields_t(F)
        _check(load_library().dust_drag_source(self.handle, ctypes.byref(pt), ctypes.byref(f),
                                               float(dt), ctypes.byref(forces), _stream(stream)))

    def deposit_mass(self, P, rho_d, stream=None):
        """dust_deposit_mass: rho_d (one ghosted array) += m W / dV."""
        if rho_d is not None and rho_d.numel() < self.grid_size()[0]:
            raise ValueError("rho_d: fewer elements than the stored cells")
        pt = self.particles_t(P)
        _check(load_library().dust_deposit_mass(self.handle, ctypes.byref(pt),
                                                _ptr(rho_d, self.real_dtype, "rho_d"),
                                                _stream(stream)))

    def apply_feedback(self, F, stream=None):
        f = self.fields_t(F)
        _check(load_library().dust_apply_feedback(self.handle, ctypes.byref(f), _stream(stream)))

    def step(self, P, F, dt, forces: dust_forces_t, nsteps=1, flags=0, stream=None):
        pt, f = self.particles_t(P), self.fields_t(F)
        _check(load_library().dust_step(self.handle, ctypes.byref(pt), ctypes.byref(f), float(dt),
                                        ctypes.byref(forces), int(nsteps), int(flags),
                                        _stream(stream)))

    def autotune(self, P, F, dt, forces: dust_forces_t, flags=0, steps=12, stream=None):
        """dust_ctx_autotune: returns {"tile": (tx, ty, tz), "rebin_every": k,
        "ms_per_step": t}; the choice stays in the context."""
        pt, f = self.particles_t(P), self.fields_t(F)
        res = (ctypes.c_int32 * 4)()
        ms = ctypes.c_float(0.0)
        _check(load_library().dust_ctx_autotune(self.handle, ctypes.byref(pt), ctypes.byref(f),
                                                float(dt), ctypes.byref(forces), int(flags),
                                                int(steps), res, ctypes.byref(ms),
                                                _stream(stream)))
        return {"tile": (res[0], res[1], res[2]), "rebin_every": res[3],
                "ms_per_step": float(ms.value)}


# ---------------------------------------------------------------- workloads

def upload(w, ctx: "Context", device="cuda", with_id=True):
    """Copy a synthetic workload to the GPU: (particles dict, fields dict)
    of torch tensors in the context's layout (boxes' ghosted fields
    concatenated)."""
    import numpy as np
    import torch
    rd = ctx.real_dtype
    npd = np.float64 if rd == torch.float64 else np.float32
    n = w.n
    P = {"cell": torch.from_numpy(np.ascontiguousarray(w.cell, dtype=np.int32)).to(device)}
    P["off"] = [torch.from_numpy(np.ascontiguousarray(w.off[:, d], dtype=npd)).to(device)
                for d in range(ctx.ndim)]
    P["mom"] = [torch.from_numpy(np.ascontiguousarray(w.mom[:, d], dtype=npd)).to(device)
                for d in range(ctx.nc)]
    if w.drag is not None:
        P["drag"] = torch.from_numpy(np.ascontiguousarray(w.drag, dtype=npd)).to(device)
    if w.mass is not None:
        P["mass"] = torch.from_numpy(np.ascontiguousarray(w.mass, dtype=npd)).to(device)
    if w.species is not None:
        P["species"] = torch.from_numpy(np.ascontiguousarray(w.species, dtype=np.uint8)).to(device)
    if with_id:
        P["id"] = torch.arange(n, dtype=torch.int32, device=device)
    rho = np.concatenate([np.asarray(g["rho"], dtype=npd).ravel() for g in w.gas])
    F = {"rho": torch.from_numpy(rho).to(device)}
    F["vel"] = [torch.from_numpy(np.concatenate([np.asarray(g["vel"][c], dtype=npd).ravel()
                                                 for g in w.gas])).to(device)
                for c in range(ctx.nc)]
    F["dep"] = [torch.zeros_like(F["rho"]) for _ in range(ctx.nc + 1)]
    return P, F


def context_for(w, device=0) -> "Context":
    return Context(w.boxes, prec=w.dtype, drag_mode=w.drag_mode, species_tau=w.species_tau,
                   species_mass=w.species_mass, device=device)


def forces_for(w, t=None) -> dust_forces_t:
    fd = w.forces
    return forces_t(fd.get("kind", "none"), fd.get("Omega", 0.0), fd.get("q", 0.0),
                    fd.get("GM", 0.0), fd.get("vertical_gravity", False),
                    fd.get("g", (0.0, 0.0, 0.0)), w.t0 if t is None else t,
                    fd.get("integrator", "em"))
