// C ABI of the dust hot path (include/dust.h): context, validation,
// workspace, and the orchestration of the per-phase kernels, binning, the
// fused tile kernel and hipGraph capture of multi-step loops.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "dust_fused.h"
#include "dust_launch.h"
#include "dust_types.h"

using namespace dust;

namespace {

thread_local std::string g_err;

dust_status_t fail(dust_status_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(DUST_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct GraphKey {
  std::vector<unsigned char> bytes;
  bool operator==(const GraphKey& o) const { return bytes == o.bytes; }
};

struct Ctx {
  int device = 0;
  int prec = DUST_F32;
  int arith = DUST_ARITH_F32;        // per-particle arithmetic of the step
  int stage_arith = DUST_ARITH_F32;  // of the stage calls (gather, push, deposit, sources)
  int drag_mode = DUST_DRAG_TAU;
  Species species{};
  Species* species_d = nullptr;
  bool have_mass_table = false;
  int geom = 0, ndim = 3;         // shared by every box
  int unif = 0;                   // Cartesian boxes whose axes are all uniform
  int nbox = 0;
  std::vector<Box> boxes;         // host copies (device table pointers inside)
  Box* boxes_d = nullptr;
  std::vector<void*> tables;      // device face / ivol tables
  int64_t n_stored = 0, n_active = 0;
  std::vector<int64_t> store_off;
  DiagDev* diag = nullptr;
  double* grid_part = nullptr;    // per-block partials of the grid sums
  double* xg = nullptr;           // FP64 x-ghost gas layers of shear-periodic boxes
  size_t xg_words = 0;
  double* tdev = nullptr;         // [0] current step start time
  hipStream_t last_stream = nullptr;
  // unfused workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // binning workspace
  BinWork bin{};
  int bin_cur = 0;                // buffer of the last sort's keys / permutation
  size_t bin_bytes = 0;
  void* bin_mem = nullptr;
  // shadow copy of the particle arrays (binned order) read by the fused step
  void* shadow_mem = nullptr;
  size_t shadow_cap = 0;          // bytes
  char* shadow_ptr[12] = {};
  int64_t* bin_start = nullptr;   // nbins+1 (fused path)
  size_t bin_start_cap = 0;
  TileShape tile{{8, 8, 4}};
  int slack = 0;
  int rebin_default = 1;          // rebinning interval when the step flags give none
  // the binned layout that the last fused FP32 uniform-Cartesian run left in
  // the caller's arrays (bin_start and the plan's tile_map describe it);
  // dust_drag_source and dust_deposit_mass use it for those arrays
  bool lay_valid = false;
  int64_t lay_n = 0;
  const void* lay_cell = nullptr;
  FusedPlan plan{};
  // deterministic mode: the unfused step with the sorted (pull) deposit and
  // fixed-order diagnostic sums; det_part holds the kick's block partials
  bool det = false;
  double* det_part = nullptr;
  size_t det_part_words = 0;
  // fused-kernel timing
  std::vector<hipEvent_t> prof_ev;  // 2 per launch
  int prof_max = 0;
  int prof_used = 0;
  // graph cache
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  GraphKey graph_key;
};

size_t real_size(const Ctx* c) { return c->prec == DUST_F64 ? 8 : 4; }
int ncomp(const Box& b) { return b.geom == GEOM_CART ? b.ndim : 3; }
int ctx_nc(const Ctx* c) {
  int nc = 0;
  for (auto& b : c->boxes) nc = std::max(nc, ncomp(b));
  return nc;
}

dust_status_t upload_table(Ctx* c, const std::vector<double>& v, const double** out) {
  void* p = nullptr;
  HIP_TRY(hipMalloc(&p, v.size() * sizeof(double)));
  c->tables.push_back(p);
  HIP_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
  *out = (const double*)p;
  return DUST_OK;
}

dust_status_t build_box(Ctx* c, const dust_box_t& in, int ib, int64_t cell_base, int64_t store_base,
                        Box& B) {
  memset(&B, 0, sizeof(B));
  if (in.geom < DUST_CART || in.geom > DUST_SPH)
    return fail(DUST_EINVAL, "box %d: unknown geometry %d", ib, in.geom);
  if (in.ndim != 2 && in.ndim != 3) return fail(DUST_EINVAL, "box %d: ndim must be 2 or 3", ib);
  if (in.ndim == 2 && in.geom != DUST_CART)
    return fail(DUST_EUNSUPPORTED, "box %d: 2-D boxes must be Cartesian", ib);
  B.geom = in.geom;
  B.ndim = in.ndim;
  int64_t ncell = 1;
  for (int d = 0; d < 3; ++d) {
    Axis& ax = B.ax[d];
    if (d >= in.ndim) {
      ax.n = 1;
      ax.uniform = 1;
      ax.d = 1.0;
      ax.inv_d = 1.0;
      ax.inv_n = 1.0;
      ax.lo = 0.0;
      ax.hi = 1.0;
      ax.L = 1.0;
      continue;
    }
    int n = in.n[d];
    if (n < 1) return fail(DUST_EINVAL, "box %d axis %d: n = %d", ib, d, n);
    if (!in.faces[d]) return fail(DUST_EINVAL, "box %d axis %d: faces is NULL", ib, d);
    const double* f = in.faces[d];
    for (int k = 0; k <= n; ++k)
      if (!std::isfinite(f[k])) return fail(DUST_EINVAL, "box %d axis %d: face %d not finite", ib, d, k);
    for (int k = 0; k < n; ++k)
      if (!(f[k + 1] > f[k])) return fail(DUST_EINVAL, "box %d axis %d: faces not increasing", ib, d);
    if (in.shape[d] != DUST_CIC && in.shape[d] != DUST_TSC && in.shape[d] != DUST_VOL)
      return fail(DUST_EINVAL, "box %d axis %d: unknown shape %d", ib, d, in.shape[d]);
    if (in.shape[d] == DUST_VOL && !(in.geom == DUST_CYL && d == 0))
      return fail(DUST_EUNSUPPORTED, "box %d axis %d: volume weighting is for the cylindrical radius", ib, d);
    for (int s = 0; s < 2; ++s) {
      int bc = s ? in.bc_hi[d] : in.bc_lo[d];
      if (bc < DUST_BC_PERIODIC || bc > DUST_BC_OPEN)
        return fail(DUST_EINVAL, "box %d axis %d: unknown boundary %d", ib, d, bc);
    }
    if ((in.bc_lo[d] == DUST_BC_OPEN) != (in.bc_hi[d] == DUST_BC_OPEN) ||
        (in.bc_lo[d] == DUST_BC_SHEAR) != (in.bc_hi[d] == DUST_BC_SHEAR))
      return fail(DUST_EINVAL, "box %d axis %d: both sides must have the same kind of boundary", ib, d);
    ax.n = n;
    ax.bc_lo = in.bc_lo[d];
    ax.bc_hi = in.bc_hi[d];
    ax.shape = in.shape[d];
    ax.lo = f[0];
    ax.hi = f[n];
    ax.L = f[n] - f[0];
    double w0 = f[1] - f[0], maxdev = 0.0;
    for (int k = 0; k < n; ++k) maxdev = std::max(maxdev, std::fabs((f[k + 1] - f[k]) - w0));
    ax.uniform = maxdev <= 1e-12 * w0 ? 1 : 0;
    ax.d = ax.L / n;
    ax.inv_d = 1.0 / ax.d;
    ax.inv_n = 1.0 / n;
    if (ax.bc_lo != DUST_BC_OPEN && !ax.uniform)
      return fail(DUST_EUNSUPPORTED, "box %d axis %d: periodic axes must be uniform", ib, d);
    ax.kind = AX_PLAIN;
    if (in.geom == DUST_CYL && d == 0) ax.kind = AX_CYL_R;
    if (in.geom == DUST_SPH && d == 0) ax.kind = AX_SPH_R;
    if (in.geom == DUST_SPH && d == 1) ax.kind = AX_THETA;
    // faces with one ghost cell each side of the width of its neighbour
    std::vector<double> ff(n + 3);
    ff[0] = f[0] - (f[1] - f[0]);
    for (int k = 0; k <= n; ++k) ff[k + 1] = f[k];
    ff[n + 2] = f[n] + (f[n] - f[n - 1]);
    if ((ax.kind == AX_CYL_R || ax.kind == AX_SPH_R) && !(ff[0] > 0.0))
      return fail(DUST_EINVAL, "box %d: the inner radial ghost face must be > 0", ib);
    if (ax.kind == AX_THETA && !(ff[0] > 0.0 && ff[n + 2] < M_PI))
      return fail(DUST_EINVAL, "box %d: theta ghost faces must lie in (0, pi)", ib);
    std::vector<double> iv(n + 2);
    for (int k = -1; k <= n; ++k) {
      double a = ff[k + 1], b = ff[k + 2];
      double v;
      switch (ax.kind) {
        case AX_CYL_R: v = 0.5 * (b * b - a * a); break;
        case AX_SPH_R: v = (b * b * b - a * a * a) / 3.0; break;
        case AX_THETA: v = std::cos(a) - std::cos(b); break;
        default: v = b - a;
      }
      iv[k + 1] = 1.0 / v;
    }
    dust_status_t st = upload_table(c, ff, &ax.faces);
    if (st) return st;
    st = upload_table(c, iv, &ax.ivol);
    if (st) return st;
    ax.trig = nullptr;
    if (ax.kind == AX_THETA) {
      std::vector<double> tg(2 * (n + 2));
      for (int k = -1; k <= n; ++k) {
        const double th = 0.5 * (ff[k + 1] + ff[k + 2]);
        tg[2 * (k + 1)] = std::sin(th);
        tg[2 * (k + 1) + 1] = std::cos(th);
      }
      st = upload_table(c, tg, &ax.trig);
      if (st) return st;
    }
    ncell *= n;
  }
  if (B.ax[0].bc_lo == DUST_BC_SHEAR) {
    if (in.geom != DUST_CART || in.ndim != 3)
      return fail(DUST_EUNSUPPORTED, "box %d: shear-periodic needs a 3-D Cartesian box", ib);
    if (B.ax[1].bc_lo != DUST_BC_PERIODIC || !B.ax[0].uniform)
      return fail(DUST_EINVAL, "box %d: shear-periodic x needs uniform x and periodic y", ib);
  }
  for (int d = 1; d < in.ndim; ++d)
    if (B.ax[d].bc_lo == DUST_BC_SHEAR)
      return fail(DUST_EINVAL, "box %d: shear-periodic only on axis 0", ib);
  B.g0 = B.ax[0].n + 2;
  B.g1 = B.ax[1].n + 2;
  B.g2 = in.ndim > 2 ? B.ax[2].n + 2 : 1;
  B.k_off = in.ndim > 2 ? 1 : 0;
  B.cell_base = cell_base;
  B.ncell = ncell;
  B.store_base = store_base;
  B.nstore = (int64_t)B.g0 * B.g1 * B.g2;
  B.xg_base = -1;
  return DUST_OK;
}

template <typename TS> PView<TS> pview(const dust_particles_t* p) {
  PView<TS> v;
  v.cell = p->cell;
  for (int d = 0; d < 3; ++d) {
    v.off[d] = (TS*)p->off[d];
    v.mom[d] = (TS*)p->mom[d];
  }
  v.drag = (TS*)p->drag;
  v.mass = (TS*)p->mass;
  v.species = p->species;
  v.id = p->id;
  v.n = p->n;
  return v;
}

template <typename TS> FView<TS> fview(const dust_fields_t* f) {
  FView<TS> v;
  v.rho = (TS*)f->rho;
  for (int d = 0; d < 3; ++d) v.vel[d] = (TS*)f->vel[d];
  for (int d = 0; d < 4; ++d) v.dep[d] = (TS*)f->dep[d];
  return v;
}

Forces forces_of(const dust_forces_t* f) {
  Forces F{};
  if (!f) return F;
  F.kind = f->kind;
  F.vertical_gravity = f->vertical_gravity;
  F.Omega = f->Omega;
  F.q = f->q;
  F.GM = f->GM;
  for (int d = 0; d < 3; ++d) F.g[d] = f->g[d];
  F.integrator = f->integrator;
  return F;
}

dust_status_t check_ctx(void* ctx) {
  if (!ctx) return fail(DUST_EINVAL, "ctx is NULL");
  return DUST_OK;
}

dust_status_t check_forces(Ctx* c, const dust_forces_t* f) {
  if (!f) return fail(DUST_EINVAL, "forces is NULL");
  if (f->kind < DUST_FORCE_NONE || f->kind > DUST_FORCE_SHEARBOX_FARGO)
    return fail(DUST_EINVAL, "unknown force kind %d", f->kind);
  const bool sb = f->kind == DUST_FORCE_SHEARBOX || f->kind == DUST_FORCE_SHEARBOX_FARGO;
  for (auto& b : c->boxes) {
    if (sb && (b.geom != GEOM_CART || b.ndim != 3))
      return fail(DUST_EUNSUPPORTED, "shearing-box forces need 3-D Cartesian boxes");
    if (f->kind == DUST_FORCE_POINTMASS && b.geom == GEOM_CART)
      return fail(DUST_EUNSUPPORTED, "point-mass gravity is for curvilinear boxes");
    if (b.ax[0].bc_lo == BC_SHEAR && !sb)
      return fail(DUST_EINVAL, "a shear-periodic box needs shearing-box forces");
  }
  if (c->drag_mode == DUST_DRAG_STOKES && !(f->GM > 0))
    return fail(DUST_EINVAL, "Stokes-number drag needs GM > 0");
  if (f->integrator != DUST_INTEGRATOR_EXPMID && f->integrator != DUST_INTEGRATOR_SEMI_IMPLICIT)
    return fail(DUST_EINVAL, "unknown integrator %d", f->integrator);
  if (f->integrator == DUST_INTEGRATOR_SEMI_IMPLICIT && c->geom != GEOM_CART)
    return fail(DUST_EUNSUPPORTED, "the semi-implicit kick is for Cartesian boxes");
  return DUST_OK;
}

dust_status_t check_particles(Ctx* c, const dust_particles_t* p, bool need_mom) {
  if (!p) return fail(DUST_EINVAL, "particles is NULL");
  if (p->n < 0 || p->n > 0x7fffffffLL) return fail(DUST_ESHAPE, "particle count %lld out of range", (long long)p->n);
  if (p->n == 0) return DUST_OK;
  if (!p->cell) return fail(DUST_EINVAL, "particles.cell is NULL");
  int ndim = 0, nc = ctx_nc(c);
  for (auto& b : c->boxes) ndim = std::max(ndim, b.ndim);
  for (int d = 0; d < ndim; ++d)
    if (!p->off[d]) return fail(DUST_EINVAL, "particles.off[%d] is NULL", d);
  if (need_mom)
    for (int d = 0; d < nc; ++d)
      if (!p->mom[d]) return fail(DUST_EINVAL, "particles.mom[%d] is NULL", d);
  return DUST_OK;
}

dust_status_t check_drag(Ctx* c, const dust_particles_t* p) {
  if (p->n == 0) return DUST_OK;
  if (c->drag_mode != DUST_DRAG_SPECIES && !p->drag)
    return fail(DUST_EINVAL, "per-particle drag array required by the drag mode");
  if (!p->mass && !c->have_mass_table)
    return fail(DUST_EINVAL, "no per-particle mass and no species mass table");
  return DUST_OK;
}

dust_status_t check_fields(Ctx* c, const dust_fields_t* f, bool gas, bool dep) {
  if (!f) return fail(DUST_EINVAL, "fields is NULL");
  int nc = ctx_nc(c);
  if (gas) {
    if (!f->rho) return fail(DUST_EINVAL, "fields.rho is NULL");
    for (int d = 0; d < nc; ++d)
      if (!f->vel[d]) return fail(DUST_EINVAL, "fields.vel[%d] is NULL", d);
  }
  if (dep)
    for (int d = 0; d <= nc; ++d)
      if (!f->dep[d]) return fail(DUST_EINVAL, "fields.dep[%d] is NULL", d);
  return DUST_OK;
}

dust_status_t ensure_ws(Ctx* c, int64_t n) {
  size_t need = (size_t)std::max<int64_t>(n, 1) * 8 * 8;
  if (need <= c->ws_bytes) return DUST_OK;
  if (c->ws) HIP_TRY(hipFree(c->ws));
  c->ws = nullptr;
  c->ws_bytes = 0;
  if (hipMalloc(&c->ws, need) != hipSuccess) return fail(DUST_ENOMEM, "workspace of %zu bytes", need);
  c->ws_bytes = need;
  return DUST_OK;
}

dust_status_t ensure_bin(Ctx* c, int64_t n) {
  if ((size_t)n <= c->bin.cap_n && c->bin_mem) return DUST_OK;
  if (c->bin_mem) HIP_TRY(hipFree(c->bin_mem));
  c->bin_mem = nullptr;
  int64_t nn = std::max<int64_t>(n, 1);
  int64_t nblocks = bin_blocks(nn);
  size_t hist = (size_t)256 * nblocks;
  size_t scan = bin_scan_tmp_words((int64_t)hist);
  auto rup = [](size_t b) { return (b + 255) & ~(size_t)255; };
  size_t bytes = 4 * rup((size_t)nn * 4) + rup(hist * 4) + rup(scan * 4) + rup((size_t)nn * 8);
  if (hipMalloc(&c->bin_mem, bytes) != hipSuccess) return fail(DUST_ENOMEM, "bin workspace of %zu bytes", bytes);
  char* q = (char*)c->bin_mem;
  auto take = [&](size_t b) { char* r = q; q += rup(b); return r; };
  c->bin.key[0] = (uint32_t*)take((size_t)nn * 4);
  c->bin.key[1] = (uint32_t*)take((size_t)nn * 4);
  c->bin.val[0] = (uint32_t*)take((size_t)nn * 4);
  c->bin.val[1] = (uint32_t*)take((size_t)nn * 4);
  c->bin.hist = (uint32_t*)take(hist * 4);
  c->bin.scan_tmp = (uint32_t*)take(scan * 4);
  c->bin.gather_tmp = take((size_t)nn * 8);
  c->bin.cap_n = (size_t)nn;
  return DUST_OK;
}

// Forget the captured step graph (its nodes point at context buffers).
void drop_graph(Ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
  c->graph_key = GraphKey{};
}

// Shadow arrays for the particles of p: one per array that p has.
dust_status_t ensure_shadow(Ctx* c, const dust_particles_t* p) {
  size_t rs = real_size(c), n = (size_t)std::max<int64_t>(p->n, 1);
  auto rup = [](size_t b) { return (b + 255) & ~(size_t)255; };
  size_t sizes[12] = {4, rs, rs, rs, rs, rs, rs, rs, rs, 1, 4, 0};
  size_t need = 0;
  for (int k = 0; k < 11; ++k) need += rup(n * sizes[k]);
  if (need > c->shadow_cap) {
    if (c->shadow_mem) HIP_TRY(hipFree(c->shadow_mem));
    c->shadow_mem = nullptr;
    c->shadow_cap = 0;
    if (hipMalloc(&c->shadow_mem, need) != hipSuccess)
      return fail(DUST_ENOMEM, "particle shadow arrays of %zu bytes", need);
    c->shadow_cap = need;
  }
  char* q = (char*)c->shadow_mem;
  for (int k = 0; k < 11; ++k) {
    c->shadow_ptr[k] = q;
    q += rup(n * sizes[k]);
  }
  return DUST_OK;
}

// The shadow arrays as a particle view with the same arrays present as p.
template <typename TS> PView<TS> shadow_view(Ctx* c, const dust_particles_t* p) {
  PView<TS> v = pview<TS>(const_cast<dust_particles_t*>(p));
  v.cell = (int32_t*)c->shadow_ptr[0];
  for (int d = 0; d < 3; ++d) {
    v.off[d] = p->off[d] ? (TS*)c->shadow_ptr[1 + d] : nullptr;
    v.mom[d] = p->mom[d] ? (TS*)c->shadow_ptr[4 + d] : nullptr;
  }
  v.drag = p->drag ? (TS*)c->shadow_ptr[7] : nullptr;
  v.mass = p->mass ? (TS*)c->shadow_ptr[8] : nullptr;
  v.species = p->species ? (uint8_t*)c->shadow_ptr[9] : nullptr;
  v.id = p->id ? (int32_t*)c->shadow_ptr[10] : nullptr;
  return v;
}

dust_status_t ensure_bin_start(Ctx* c) {
  size_t need = (size_t)c->n_active + 1;
  if (need <= c->bin_start_cap) return DUST_OK;
  if (c->bin_start) HIP_TRY(hipFree(c->bin_start));
  if (hipMalloc((void**)&c->bin_start, need * 8) != hipSuccess) return fail(DUST_ENOMEM, "bin starts");
  c->bin_start_cap = need;
  return DUST_OK;
}

// Workspace of the deterministic mode for n particles: the sort's and the
// kick's block partials.
dust_status_t ensure_det(Ctx* c, int64_t n) {
  dust_status_t s;
  if ((s = ensure_bin(c, n)) || (s = ensure_bin_start(c))) return s;
  size_t need = (size_t)kick_partial_words(n);
  if (need <= c->det_part_words) return DUST_OK;
  if (c->det_part) HIP_TRY(hipFree(c->det_part));
  c->det_part = nullptr;
  c->det_part_words = 0;
  if (hipMalloc((void**)&c->det_part, need * 8) != hipSuccess) return fail(DUST_ENOMEM, "kick partials");
  c->det_part_words = need;
  return DUST_OK;
}

// Apply perm (sorted slot -> input index) to every particle array, staging
// each through tmp (8 bytes per particle).
dust_status_t apply_perm(Ctx* c, dust_particles_t* p, const uint32_t* perm, void* tmp, hipStream_t st) {
  int64_t n = p->n;
  int rs = (int)real_size(c);
  auto one = [&](void* a, int bytes) -> dust_status_t {
    if (!a) return DUST_OK;
    launch_permute(a, tmp, perm, n, bytes, st);
    HIP_TRY(hipMemcpyAsync(a, tmp, (size_t)n * bytes, hipMemcpyDeviceToDevice, st));
    return DUST_OK;
  };
  dust_status_t s;
  if ((s = one(p->cell, 4))) return s;
  for (int d = 0; d < 3; ++d) {
    if ((s = one(p->off[d], rs))) return s;
    if ((s = one(p->mom[d], rs))) return s;
  }
  if ((s = one(p->drag, rs))) return s;
  if ((s = one(p->mass, rs))) return s;
  if ((s = one(p->species, 1))) return s;
  if ((s = one(p->id, 4))) return s;
  return DUST_OK;
}

// ------------------------------------------------------------------ allocation-free sort workspace

// Fixed device workspace of dust_bin_noalloc: two key and two value arrays,
// the digit histograms, the scan's block sums and the staging array of the
// permutation, for up to DUST_BIN_NOALLOC_MAX particles (about 24.3 MiB of
// the 25 MiB).  Each GPU the library runs on holds its own copy until the
// process ends.  Host code uses the address taken with hipGetSymbolAddress on
// that device (g_scratch_ptr), never the array's name.
constexpr size_t kScratchBytes = (size_t)25 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Takes the address of the current device's copy of the array, once per
// device (called by dust_ctx_create with `device` current).
dust_status_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(DUST_EUNSUPPORTED, "device %d: at most %d devices", device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return DUST_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(DUST_EDEVICE, "address of the sort scratch array on device %d: %s", device, hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
  return DUST_OK;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

// The sort workspace for n particles carved from a scratch array at base;
// false if it would not fit.
bool scratch_work(void* base, int64_t n, BinWork& w) {
  const int64_t nn = std::max<int64_t>(n, 1);
  const size_t hist = (size_t)256 * bin_blocks(nn);
  const size_t scan = bin_scan_tmp_words((int64_t)hist);
  auto rup = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t bytes = 4 * rup((size_t)nn * 4) + rup(hist * 4) + rup(scan * 4) + rup((size_t)nn * 8);
  if (bytes > kScratchBytes) return false;
  char* q = (char*)base;
  auto take = [&](size_t b) { char* r = q; q += rup(b); return r; };
  w.key[0] = (uint32_t*)take((size_t)nn * 4);
  w.key[1] = (uint32_t*)take((size_t)nn * 4);
  w.val[0] = (uint32_t*)take((size_t)nn * 4);
  w.val[1] = (uint32_t*)take((size_t)nn * 4);
  w.hist = (uint32_t*)take(hist * 4);
  w.scan_tmp = (uint32_t*)take(scan * 4);
  w.gather_tmp = take((size_t)nn * 8);
  w.cap_n = (size_t)nn;
  return true;
}

// ------------------------------------------------------------------ typed drivers

// Deterministic deposit: a stable sort of the particles by cell (into the
// binning workspace and bin starts, which no longer describe a fused
// layout), then every box's cells sum their particles' contributions:
// out.dep[m] += sgn * sum W q[m] / dV for m < nch (the step's deposit: all
// channels, sgn = -1).
template <typename TS, typename A, typename TW>
void deposit_det(Ctx* c, const PView<TS>& pv, const FView<TS>& out, const TW* const q[4], hipStream_t st,
                 int nch = -1, double sgn = -1.0) {
  if (nch < 0) nch = ctx_nc(c) + 1;
  c->bin_cur = launch_bin(pv.cell, pv.n, c->boxes_d, c->nbox, c->n_active, DUST_BIN_CELL, c->tile, c->bin,
                          nullptr, c->bin_start, false, st);
  c->lay_valid = false;
  for (auto& B : c->boxes)
    launch_deposit_pull<TS, A, TW>(pv, B, c->geom, c->ndim, c->unif, out, nch, sgn, q, c->bin.val[c->bin_cur],
                                   c->bin_start, st);
}

// The drag source (mass: the dust density into out.dep[0]) of the
// deterministic mode: per-particle coefficients into the unfused workspace,
// then the sorted deposit.
template <typename TS, typename A>
void source_det(Ctx* c, const PView<TS>& pv, const FView<TS>& fl, const FView<TS>& out, const Forces& F, double dt,
                bool mass, hipStream_t st) {
  const int64_t n = pv.n;
  A* ws = (A*)c->ws;
  A* q[3] = {ws, ws + n, ws + 2 * n};
  launch_source_coeffs<TS, A>(pv, c->boxes_d, c->nbox, c->geom, c->ndim, c->unif, fl, F, c->species_d,
                              c->drag_mode, dt, mass, q, c->diag, st);
  const A* cq[4] = {q[0], q[1], q[2], nullptr};
  deposit_det<TS, A, A>(c, pv, out, cq, st, mass ? 1 : ctx_nc(c), mass ? 1.0 : -1.0);
}

template <typename TS, typename A>
void run_push(Ctx* c, const PView<TS>& pv, const Forces& F, double dt, int phases,
              const TS* const vg[3], TS* const imp[4], DiagDev* dg, hipStream_t st) {
  if (phases & DUST_PHASE_DRIFT1)
    launch_drift<TS, A>(pv, c->boxes_d, c->nbox, c->geom, c->ndim, c->unif, F, 0.5 * dt, c->tdev, 0.5 * dt, 1, dg, st);
  if (phases & DUST_PHASE_KICK)
    launch_kick<TS, A, TS>(pv, c->boxes_d, c->nbox, c->geom, c->ndim, c->unif, F, c->species_d, c->drag_mode, dt,
                           nullptr, vg, imp, dg, c->det ? c->det_part : nullptr, st);
  if (phases & DUST_PHASE_DRIFT2)
    launch_drift<TS, A>(pv, c->boxes_d, c->nbox, c->geom, c->ndim, c->unif, F, 0.5 * dt, c->tdev, dt, 0, dg, st);
}

// One unfused step (time in c->tdev[0] at the start of the step).
template <typename TS, typename A>
void unfused_step(Ctx* c, const PView<TS>& pv, const FView<TS>& fv, const Forces& F, double dt,
                  int flags, hipStream_t st) {
  int nc = ctx_nc(c);
  int64_t n = pv.n;
  A* ws = (A*)c->ws;  // gathered gas and impulses kept in the arithmetic precision
  A* vg[3] = {ws, ws + n, ws + 2 * n};
  A* imp[4] = {ws + 3 * n, ws + 4 * n, ws + 5 * n, ws + 6 * n};
  A* rho_p = c->drag_mode == DUST_DRAG_EPSTEIN ? ws + 7 * n : nullptr;   // Epstein: gathered density
  for (int k = nc; k < 3; ++k) vg[k] = nullptr;
  for (int k = nc + 1; k < 4; ++k) imp[k] = nullptr;
  DiagDev* dg = (flags & DUST_STEP_DIAG) ? c->diag : nullptr;
  DiagDev* dflags = c->diag;  // sticky flags always recorded
  if (!(flags & DUST_STEP_NO_FILL))
    launch_fill<TS>(c->boxes.data(), c->nbox, c->boxes_d, F, c->tdev, 0.5 * dt, fv, c->xg, st);
  launch_clear_deposits<TS>(fv, nc + 1, c->n_stored, st);
  launch_drift<TS, A>(pv, c->boxes_d, c->nbox, c->geom, c->ndim, c->unif, F, 0.5 * dt, c->tdev, 0.5 * dt, 1, dflags, st);
  launch_gather<TS, A, A>(pv, c->boxes_d, c->nbox, c->geom, c->ndim, c->unif, fv,
                          (flags & DUST_STEP_NO_FILL) ? nullptr : c->xg, rho_p, vg, dflags, st);
  const A* cvg[3] = {vg[0], vg[1], vg[2]};
  launch_kick<TS, A, A>(pv, c->boxes_d, c->nbox, c->geom, c->ndim, c->unif, F, c->species_d, c->drag_mode, dt, rho_p,
                        cvg, imp, dg ? dg : dflags, c->det ? c->det_part : nullptr, st);
  const A* cimp[4] = {imp[0], imp[1], imp[2], imp[3]};
  if (c->det)
    deposit_det<TS, A, A>(c, pv, fv, cimp, st);
  else
    launch_deposit<TS, A, A>(pv, c->boxes_d, c->nbox, c->geom, c->ndim, c->unif, fv, cimp, dflags, st);
  launch_drift<TS, A>(pv, c->boxes_d, c->nbox, c->geom, c->ndim, c->unif, F, 0.5 * dt, c->tdev, dt, 0, dflags, st);
  if (dg)
    launch_grid_sums<TS>(c->boxes.data(), c->nbox, c->boxes_d, fv, dg, c->grid_part, st);
  launch_fold<TS>(c->boxes.data(), c->nbox, c->boxes_d, F, c->tdev, 0.5 * dt, fv, st);
  if (flags & DUST_STEP_APPLY_FEEDBACK)
    launch_feedback<TS>(c->boxes.data(), c->nbox, c->boxes_d, fv, st);
}

// How a fused step moves the particles between the caller's arrays and the
// context's shadow copy.
enum StepMove {
  STEP_IN_PLACE,   // stale bins: x is updated where it is
  STEP_REBIN,      // new bins: x is sorted into y (level-major slots)
  STEP_MOVE,       // stale bins, written to y slot for slot
};

// Whether a fused step runs the FP32 uniform-Cartesian tile kernel
// (dust_cart3.hip): 3-D Cartesian boxes with uniform axes, FP32 storage and
// arithmetic, forces none, constant or standard shearing box, masses and
// stopping times from the species table (no per-particle arrays), fewer
// than 2^30 particles (32-bit byte offsets of 4-byte elements).
template <typename TS>
bool use_c3(const Ctx* c, bool f32, const Forces& F, const PView<TS>& x) {
  return f32 && c->geom == GEOM_CART && c->ndim == 3 && c->unif &&
         (F.kind == FORCE_NONE || F.kind == FORCE_CONST || F.kind == FORCE_SHEARBOX) &&
         c->drag_mode == DUST_DRAG_SPECIES && !x.mass && !x.drag && x.n < (int64_t(1) << 30);
}

// Whether the particles are the arrays the last fused FP32 uniform-Cartesian
// run left in their binned layout (same count and cell array).
bool on_layout(const Ctx* c, const PView<float>& p) {
  return c->lay_valid && p.n == c->lay_n && (const void*)p.cell == c->lay_cell;
}

template <typename TS, typename A>
dust_status_t fused_step(Ctx* c, const PView<TS>& x, const PView<TS>& y, const FView<TS>& fv,
                         const Forces& F, double dt, int flags, StepMove mv, hipStream_t st) {
  int nc = ctx_nc(c);
  DiagDev* dg = (flags & DUST_STEP_DIAG) ? c->diag : nullptr;
  constexpr bool f32 = std::is_same<TS, float>::value && std::is_same<A, float>::value;
  const bool c3 = use_c3(c, f32, F, x);
  // Rebinning: keys of the cells the particles kick in, a stable sort, and the
  // source index of every slot in the fused kernel's order, through which
  // the fused kernel reads x while writing y in binned order (the particles
  // without a cell are copied across).
  const uint32_t* src_index = nullptr;
  if (mv == STEP_REBIN) {
    if constexpr (f32) {
      if (c3)
        launch_c3_keys(x, c->boxes_d, c->nbox, dt, c->n_active, c->tile, c->bin.key[0], st);
    }
    if (!c3)
      launch_halfstep_keys<TS, A>(x, c->boxes_d, c->nbox, c->geom, c->ndim, c->unif, F, dt, c->tdev,
                                  c->n_active, c->tile, c->bin.key[0], st);
    c->bin_cur = launch_bin(x.cell, x.n, c->boxes_d, c->nbox, c->n_active, DUST_BIN_TILE, c->tile,
                            c->bin, nullptr, c->bin_start, true, st);
    uint32_t* lm = c->bin.val[1 - c->bin_cur];   // free once the sort is done
    if (c3) {
      launch_c3_level_perm(c->plan, c->bin.val[c->bin_cur], c->bin_start, lm, st);
      launch_copy_tail<TS>(x, y, c->bin_start, c->n_active, st, c->bin.val[c->bin_cur]);
    } else {
      launch_level_perm<TS>(c->plan, x, y, c->bin.val[c->bin_cur], c->bin_start, c->n_active, lm, st);
    }
    src_index = lm;
  } else if (mv == STEP_MOVE) {
    launch_copy_tail<TS>(x, y, c->bin_start, c->n_active, st);
  }
  const PView<TS>& out = mv == STEP_IN_PLACE ? x : y;
  if (!(flags & DUST_STEP_NO_FILL))
    launch_fill<TS>(c->boxes.data(), c->nbox, c->boxes_d, F, c->tdev, 0.5 * dt, fv, c->xg, st);
  launch_clear_deposits<TS>(fv, nc + 1, c->n_stored, st);
  const bool prof = c->prof_used < c->prof_max;
  hipEvent_t ev0 = prof ? c->prof_ev[2 * c->prof_used] : nullptr;
  hipEvent_t ev1 = prof ? c->prof_ev[2 * c->prof_used + 1] : nullptr;
  if constexpr (f32) {
    if (c3)
      launch_c3(c->plan, x, out, mv != STEP_IN_PLACE, c->boxes_d, c->nbox, fv, F, c->species_d, c->drag_mode, dt,
                c->tdev, c->bin_start, (flags & DUST_STEP_NO_FILL) ? nullptr : c->xg, c->diag, dg != nullptr,
                src_index, ev0, ev1, st);
  }
  if (!c3)
    launch_fused<TS, A>(c->plan, x, out, mv != STEP_IN_PLACE, c->boxes_d, c->nbox, c->geom, c->ndim, c->unif,
                        fv, F, c->species_d, c->drag_mode, dt, c->tdev, c->bin_start,
                        (flags & DUST_STEP_NO_FILL) ? nullptr : c->xg, c->diag, dg != nullptr, src_index,
                        ev0, ev1, st);
  HIP_TRY(hipGetLastError());
  if (prof) ++c->prof_used;
  if (dg)
    launch_grid_sums<TS>(c->boxes.data(), c->nbox, c->boxes_d, fv, dg, c->grid_part, st);
  launch_fold<TS>(c->boxes.data(), c->nbox, c->boxes_d, F, c->tdev, 0.5 * dt, fv, st);
  if (flags & DUST_STEP_APPLY_FEEDBACK)
    launch_feedback<TS>(c->boxes.data(), c->nbox, c->boxes_d, fv, st);
  return DUST_OK;
}

template <typename TS, typename A>
dust_status_t run_steps(Ctx* c, dust_particles_t* p, dust_fields_t* f, double dt, const Forces& F,
                        int nsteps, int flags, hipStream_t st) {
  PView<TS> pv = pview<TS>(p);
  FView<TS> fv = fview<TS>(f);
  int rebin_every = (flags >> 8) & 0xff;
  if (rebin_every <= 0) rebin_every = c->rebin_default;
  if (!(flags & DUST_STEP_FUSED)) {
    for (int s = 0; s < nsteps; ++s) {
      // the unfused chain passes gathered velocities and impulses through
      // memory, where FP32 would lose the slip: it computes in FP64
      unfused_step<TS, double>(c, pv, fv, F, dt, flags, st);
      launch_advance_time(c->tdev, dt, (flags & DUST_STEP_DIAG) ? c->diag : nullptr, st);
    }
    return DUST_OK;
  }
  // Every rebinning moves the particles to the other buffer (the caller's
  // arrays or the shadow copy).  With an odd number of rebinnings the last
  // step with stale bins is done out of place instead, so that the call ends
  // in the caller's arrays; with none, a copy at the end.
  PView<TS> sh = shadow_view<TS>(c, p);
  int nrebin = (nsteps + rebin_every - 1) / rebin_every;
  int last_stale = -1;
  for (int s = 0; s < nsteps; ++s)
    if (s % rebin_every) last_stale = s;
  const bool odd = nrebin % 2 == 1;
  bool in_shadow = false;
  for (int s = 0; s < nsteps; ++s) {
    StepMove mv = s % rebin_every == 0 ? STEP_REBIN : (odd && s == last_stale) ? STEP_MOVE : STEP_IN_PLACE;
    const PView<TS>& x = in_shadow ? sh : pv;
    const PView<TS>& y = in_shadow ? pv : sh;
    dust_status_t e = fused_step<TS, A>(c, x, y, fv, F, dt, flags, mv, st);
    if (e) return e;
    if (mv != STEP_IN_PLACE) in_shadow = !in_shadow;
    launch_advance_time(c->tdev, dt, (flags & DUST_STEP_DIAG) ? c->diag : nullptr, st);
  }
  if (in_shadow) launch_copy_particles<TS>(sh, pv, st);
  constexpr bool f32 = std::is_same<TS, float>::value && std::is_same<A, float>::value;
  c->lay_valid = use_c3(c, f32, F, pv);
  c->lay_n = pv.n;
  c->lay_cell = pv.cell;
  return DUST_OK;
}

// Typed dispatch on the storage precision and an arithmetic (DUST_ARITH_*).
template <typename F>
dust_status_t dispatch_arith(Ctx* c, int arith, F&& fn) {
  if (c->prec == DUST_F64) return fn((double)0, (double)0);
  if (arith == DUST_ARITH_F32) return fn((float)0, (float)0);
  return fn((float)0, (double)0);
}

// The stage calls' dispatch.
template <typename F>
dust_status_t dispatch(Ctx* c, F&& fn) {
  return dispatch_arith(c, c->stage_arith, std::forward<F>(fn));
}

}  // namespace

// ============================================================== C ABI

extern "C" {

const char* dust_last_error(void) { return g_err.c_str(); }

dust_status_t dust_ctx_create(void** ctx, int device, const dust_box_t* boxes, int nbox, int32_t prec,
                              int32_t drag_mode, const double* species_tau,
                              const double* species_mass, int nspecies) {
  g_err.clear();
  if (!ctx) return fail(DUST_EINVAL, "ctx out-pointer is NULL");
  *ctx = nullptr;
  if (!boxes || nbox < 1 || nbox > 4096) return fail(DUST_EINVAL, "need 1..4096 boxes");
  if (prec != DUST_F32 && prec != DUST_F64) return fail(DUST_EINVAL, "unknown precision %d", prec);
  if (drag_mode < DUST_DRAG_TAU || drag_mode > DUST_DRAG_EPSTEIN)
    return fail(DUST_EINVAL, "unknown drag mode %d", drag_mode);
  if (nspecies < 0 || nspecies > DUST_MAX_SPECIES)
    return fail(DUST_EINVAL, "nspecies must be 0..%d", DUST_MAX_SPECIES);
  if (drag_mode == DUST_DRAG_SPECIES && (nspecies < 1 || !species_tau))
    return fail(DUST_EINVAL, "species drag needs a tau table");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(DUST_EINVAL, "device %d of %d", device, ndev);
  HIP_TRY(hipSetDevice(device));
  {
    const dust_status_t s = scratch_setup(device);
    if (s) return s;
  }
  Ctx* c = new Ctx();
  c->device = device;
  c->prec = prec;
  c->drag_mode = drag_mode;
  c->species.n = nspecies > 0 ? nspecies : 1;
  for (int s = 0; s < DUST_MAX_SPECIES; ++s) {
    c->species.tau[s] = (species_tau && s < nspecies) ? species_tau[s] : INFINITY;
    c->species.mass[s] = (species_mass && s < nspecies) ? species_mass[s] : 0.0;
    c->species.inv_tau[s] = 1.0 / c->species.tau[s];
  }
  c->have_mass_table = species_mass != nullptr && nspecies > 0;
  if (species_tau)
    for (int s = 0; s < nspecies; ++s)
      if (!(species_tau[s] > 0)) {
        delete c;
        return fail(DUST_EINVAL, "species %d: tau must be > 0 (or +inf)", s);
      }
  int64_t cell_base = 0, store_base = 0;
  c->nbox = nbox;
  c->boxes.resize(nbox);
  c->store_off.resize(nbox + 1);
  for (int b = 0; b < nbox; ++b) {
    dust_status_t s = build_box(c, boxes[b], b, cell_base, store_base, c->boxes[b]);
    if (s) {
      std::string keep = g_err;
      dust_ctx_destroy(c);
      g_err = keep;
      return s;
    }
    c->store_off[b] = store_base;
    cell_base += c->boxes[b].ncell;
    store_base += c->boxes[b].nstore;
  }
  c->store_off[nbox] = store_base;
  // FP64 x-ghost gas layers of the shear-periodic boxes
  c->xg_words = 0;
  for (auto& B : c->boxes)
    if (B.ax[0].bc_lo == DUST_BC_SHEAR) {
      B.xg_base = (int64_t)c->xg_words;
      c->xg_words += (size_t)2 * 3 * B.g1 * B.g2;
    }
  c->geom = c->boxes[0].geom;
  c->ndim = c->boxes[0].ndim;
  for (int b = 1; b < nbox; ++b)
    if (c->boxes[b].geom != c->geom || c->boxes[b].ndim != c->ndim) {
      dust_ctx_destroy(c);
      return fail(DUST_EUNSUPPORTED, "all boxes of a context must share geometry and ndim");
    }
  // FP32 push arithmetic in the step: its slip form keeps the slip accurate
  // (in Cartesian boxes the large velocities come from a smooth background
  // flow that the weights reproduce; in curvilinear boxes the scale factors
  // are two-word FP64 values at the particle and the azimuthal gather sums
  // in FP64).  The stage calls form the slip from a gathered velocity passed
  // through memory, which in curvilinear boxes loses the slip of a particle
  // close to co-rotation in FP32: FP64 there.
  c->arith = DUST_ARITH_F32;
  c->stage_arith = c->geom == GEOM_CART ? DUST_ARITH_F32 : DUST_ARITH_F64;
  c->unif = c->geom == GEOM_CART ? 1 : 0;
  for (int b = 0; b < nbox; ++b)
    for (int d = 0; d < c->ndim; ++d)
      if (!c->boxes[b].ax[d].uniform) c->unif = 0;
  c->n_active = cell_base;
  c->n_stored = store_base;
  if (cell_base >= 0x7fffffffLL) {
    dust_ctx_destroy(c);
    return fail(DUST_ESHAPE, "more than 2^31-1 active cells");
  }
  if (hipMalloc((void**)&c->species_d, sizeof(Species)) != hipSuccess ||
      hipMemcpy(c->species_d, &c->species, sizeof(Species), hipMemcpyHostToDevice) != hipSuccess ||
      hipMalloc((void**)&c->boxes_d, sizeof(Box) * nbox) != hipSuccess ||
      hipMalloc((void**)&c->diag, sizeof(DiagDev)) != hipSuccess ||
      hipMalloc((void**)&c->grid_part, sizeof(double) * 4 * GRID_SUM_PARTS) != hipSuccess ||
      (c->xg_words && hipMalloc((void**)&c->xg, sizeof(double) * c->xg_words) != hipSuccess) ||
      hipMalloc((void**)&c->tdev, 64) != hipSuccess) {
    dust_ctx_destroy(c);
    return fail(DUST_ENOMEM, "context tables");
  }
  if (hipMemcpy(c->boxes_d, c->boxes.data(), sizeof(Box) * nbox, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(c->diag, 0, sizeof(DiagDev)) != hipSuccess || hipMemset(c->tdev, 0, 64) != hipSuccess) {
    dust_ctx_destroy(c);
    return fail(DUST_EDEVICE, "context upload");
  }
  if (c->ndim == 2) c->tile = TileShape{{16, 16, 1}};
  fused_plan_init(c->plan, c->boxes.data(), nbox, c->tile, c->slack);
  *ctx = c;
  return DUST_OK;
}

dust_status_t dust_ctx_destroy(void* ctx) {
  if (!ctx) return DUST_OK;
  Ctx* c = (Ctx*)ctx;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
  if (c->graph) hipGraphDestroy(c->graph);
  for (auto e : c->prof_ev) hipEventDestroy(e);
  for (void* p : c->tables) hipFree(p);
  if (c->boxes_d) hipFree(c->boxes_d);
  if (c->species_d) hipFree(c->species_d);
  if (c->diag) hipFree(c->diag);
  if (c->grid_part) hipFree(c->grid_part);
  if (c->xg) hipFree(c->xg);
  if (c->tdev) hipFree(c->tdev);
  if (c->ws) hipFree(c->ws);
  if (c->bin_mem) hipFree(c->bin_mem);
  if (c->shadow_mem) hipFree(c->shadow_mem);
  if (c->bin_start) hipFree(c->bin_start);
  if (c->det_part) hipFree(c->det_part);
  fused_plan_free(c->plan);
  delete c;
  return DUST_OK;
}

dust_status_t dust_ctx_set_arith(void* ctx, int32_t arith) {
  if (check_ctx(ctx)) return DUST_EINVAL;
  if (arith != DUST_ARITH_F64 && arith != DUST_ARITH_F32) return fail(DUST_EINVAL, "unknown arith %d", arith);
  ((Ctx*)ctx)->arith = arith;
  ((Ctx*)ctx)->stage_arith = arith;
  return DUST_OK;
}

dust_status_t dust_ctx_set_deterministic(void* ctx, int32_t on) {
  if (check_ctx(ctx)) return DUST_EINVAL;
  if (on != 0 && on != 1) return fail(DUST_EINVAL, "deterministic: 0 or 1, not %d", on);
  Ctx* c = (Ctx*)ctx;
  c->det = on != 0;
  drop_graph(c);
  return DUST_OK;
}

dust_status_t dust_ctx_set_tile(void* ctx, int32_t tx, int32_t ty, int32_t tz, int32_t slack) {
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  int32_t t[3] = {tx, ty, tz};
  TileShape want = c->tile;
  for (int d = 0; d < 3; ++d) {
    if (t[d] < 0 || t[d] > 64) return fail(DUST_EINVAL, "tile extent %d out of 0..64", t[d]);
    if (t[d] > 0) want.t[d] = t[d];
  }
  if (slack < 0 || slack > 4) return fail(DUST_EINVAL, "slack %d out of 0..4", slack);
  drop_graph(c);
  c->lay_valid = false;
  dust_status_t s = fused_plan_init(c->plan, c->boxes.data(), c->nbox, want, slack);
  if (s) {
    // keep the previous shape (and a valid plan)
    (void)fused_plan_init(c->plan, c->boxes.data(), c->nbox, c->tile, c->slack);
    return fail(s, "tile %dx%dx%d is not one of the compiled fused tile shapes", want.t[0], want.t[1],
                want.t[2]);
  }
  c->tile = want;
  c->slack = slack;
  return DUST_OK;
}

dust_status_t dust_ctx_set_profile(void* ctx, int32_t max_launches) {
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  if (max_launches < 0 || max_launches > 100000) return fail(DUST_EINVAL, "max_launches out of range");
  HIP_TRY(hipSetDevice(c->device));
  for (auto e : c->prof_ev) hipEventDestroy(e);
  c->prof_ev.clear();
  c->prof_max = 0;
  c->prof_used = 0;
  for (int i = 0; i < 2 * max_launches; ++i) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    c->prof_ev.push_back(e);
  }
  c->prof_max = max_launches;
  drop_graph(c);  // graphs captured before carry no event nodes
  return DUST_OK;
}

dust_status_t dust_ctx_profile(void* ctx, float* ms_out, int32_t max_out, int32_t* count_out) {
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->last_stream));
  int n = std::min(c->prof_used, max_out);
  for (int i = 0; i < n; ++i) HIP_TRY(hipEventElapsedTime(&ms_out[i], c->prof_ev[2 * i], c->prof_ev[2 * i + 1]));
  if (count_out) *count_out = n;
  return DUST_OK;
}

dust_status_t dust_ctx_grid_size(void* ctx, int64_t* n_stored, int64_t* n_active, int64_t* box_store_offset) {
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  if (n_stored) *n_stored = c->n_stored;
  if (n_active) *n_active = c->n_active;
  if (box_store_offset)
    for (int b = 0; b <= c->nbox; ++b) box_store_offset[b] = c->store_off[b];
  return DUST_OK;
}

dust_status_t dust_ctx_status(void* ctx, dust_diag_t* out) {
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->last_stream));
  DiagDev d;
  HIP_TRY(hipMemcpy(&d, c->diag, sizeof(d), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(c->diag, 0, sizeof(DiagDev)));
  if (out) {
    memset(out, 0, sizeof(*out));
    for (int k = 0; k < 3; ++k) {
      out->p_part[k] = d.p_part[k];
      out->p_grid[k] = d.p_grid[k];
    }
    out->e_part = d.e_part;
    out->e_grid = d.e_grid;
    out->sum_abs_j = d.sum_abs_j;
    double m;
    memcpy(&m, &d.max_cells_bits, 8);
    out->max_cells_per_step = m;
    out->n_removed = (int64_t)d.n_removed;
    out->n_fallback = (int64_t)d.n_fallback;
    out->flags = (int32_t)d.flags;
    out->steps = (int32_t)d.steps;
  }
  return DUST_OK;
}

dust_status_t dust_bin(void* ctx, dust_particles_t* p, int32_t key_mode, int32_t* perm_out,
                       int64_t* bin_start_out, int apply_permutation, void* stream) {
  g_err.clear();
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  if (key_mode != DUST_BIN_CELL && key_mode != DUST_BIN_TILE) return fail(DUST_EINVAL, "unknown key mode");
  if (!p) return fail(DUST_EINVAL, "particles is NULL");
  if (p->n < 0 || p->n > 0x7fffffffLL) return fail(DUST_ESHAPE, "particle count out of range");
  if (p->n > 0 && !p->cell) return fail(DUST_EINVAL, "particles.cell is NULL");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(c->device));
  dust_status_t s = ensure_bin(c, p->n);
  if (s) return s;
  c->last_stream = st;
  if (apply_permutation) c->lay_valid = false;
  c->bin_cur = launch_bin(p->cell, p->n, c->boxes_d, c->nbox, c->n_active, key_mode, c->tile,
                          c->bin, perm_out, bin_start_out, false, st);
  if (apply_permutation && p->n > 0) return apply_perm(c, p, c->bin.val[c->bin_cur], c->bin.gather_tmp, st);
  HIP_TRY(hipGetLastError());
  return DUST_OK;
}

dust_status_t dust_bin_noalloc(void* ctx, dust_particles_t* p, int32_t key_mode, int32_t* perm_out,
                               int64_t* bin_start_out, int apply_permutation, void* stream) {
  g_err.clear();
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  if (key_mode != DUST_BIN_CELL && key_mode != DUST_BIN_TILE) return fail(DUST_EINVAL, "unknown key mode");
  if (!p) return fail(DUST_EINVAL, "particles is NULL");
  if (p->n < 0 || p->n > DUST_BIN_NOALLOC_MAX)
    return fail(DUST_ESHAPE, "dust_bin_noalloc: %lld particles, at most %d", (long long)p->n,
                DUST_BIN_NOALLOC_MAX);
  if (p->n > 0 && !p->cell) return fail(DUST_EINVAL, "particles.cell is NULL");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(c->device));
  void* base = scratch_of(c->device);
  if (!base) return fail(DUST_EDEVICE, "no scratch array address for device %d", c->device);
  BinWork w;
  if (!scratch_work(base, p->n, w)) return fail(DUST_ESHAPE, "sort workspace exceeds the scratch array");
  c->last_stream = st;
  if (apply_permutation) c->lay_valid = false;
  // every workspace word the sort reads is written before in the same call
  // (keys, histograms, scans), so nothing is cleared
  const int cur = launch_bin(p->cell, p->n, c->boxes_d, c->nbox, c->n_active, key_mode, c->tile, w,
                             perm_out, bin_start_out, false, st);
  if (apply_permutation && p->n > 0) {
    dust_status_t s = apply_perm(c, p, w.val[cur], w.gather_tmp, st);
    if (s) return s;
  }
  HIP_TRY(hipGetLastError());
  return DUST_OK;
}

dust_status_t dust_fill_ghosts(void* ctx, dust_fields_t* f, const dust_forces_t* frc, double t, void* stream) {
  g_err.clear();
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  dust_status_t s;
  if ((s = check_fields(c, f, true, false)) || (s = check_forces(c, frc))) return s;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(c->device));
  c->last_stream = st;
  launch_set_time(c->tdev, t, st);
  Forces F = forces_of(frc);
  return dispatch(c, [&](auto ts, auto) -> dust_status_t {
    using TS = decltype(ts);
    FView<TS> fv = fview<TS>(f);
    launch_fill<TS>(c->boxes.data(), c->nbox, c->boxes_d, F, c->tdev, 0.0, fv, c->xg, st);
    HIP_TRY(hipGetLastError());
    return DUST_OK;
  });
}

dust_status_t dust_fold_ghosts(void* ctx, dust_fields_t* f, const dust_forces_t* frc, double t, void* stream) {
  g_err.clear();
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  dust_status_t s;
  if ((s = check_fields(c, f, false, true)) || (s = check_forces(c, frc))) return s;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(c->device));
  c->last_stream = st;
  launch_set_time(c->tdev, t, st);
  Forces F = forces_of(frc);
  return dispatch(c, [&](auto ts, auto) -> dust_status_t {
    using TS = decltype(ts);
    FView<TS> fv = fview<TS>(f);
    launch_fold<TS>(c->boxes.data(), c->nbox, c->boxes_d, F, c->tdev, 0.0, fv, st);
    HIP_TRY(hipGetLastError());
    return DUST_OK;
  });
}

dust_status_t dust_gather(void* ctx, const dust_particles_t* p, const dust_fields_t* f, void* rho_p,
                          void* vg_p[3], void* stream) {
  g_err.clear();
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  dust_status_t s;
  if ((s = check_particles(c, p, false)) || (s = check_fields(c, f, true, false))) return s;
  int nc = ctx_nc(c);
  if (!vg_p) return fail(DUST_EINVAL, "vg_p is NULL");
  for (int k = 0; k < nc; ++k)
    if (p->n > 0 && !vg_p[k]) return fail(DUST_EINVAL, "vg_p[%d] is NULL", k);
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(c->device));
  c->last_stream = st;
  return dispatch(c, [&](auto ts, auto ta) -> dust_status_t {
    using TS = decltype(ts);
    using A = decltype(ta);
    TS* vg[3] = {nullptr, nullptr, nullptr};
    for (int k = 0; k < nc; ++k) vg[k] = (TS*)vg_p[k];
    launch_gather<TS, A, TS>(pview<TS>(p), c->boxes_d, c->nbox, c->geom, c->ndim, c->unif, fview<TS>(f),
                             nullptr, (TS*)rho_p, vg, c->diag, st);
    HIP_TRY(hipGetLastError());
    return DUST_OK;
  });
}

dust_status_t dust_push_expmid(void* ctx, dust_particles_t* p, const void* const vg_p[3], double dt,
                               const dust_forces_t* frc, int32_t phases, void* impulse[4], void* stream) {
  g_err.clear();
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  dust_status_t s;
  if ((s = check_particles(c, p, true)) || (s = check_forces(c, frc))) return s;
  if (!std::isfinite(dt)) return fail(DUST_EINVAL, "dt not finite");
  if (phases & ~(DUST_PHASE_DRIFT1 | DUST_PHASE_KICK | DUST_PHASE_DRIFT2))
    return fail(DUST_EINVAL, "unknown phase bits");
  int nc = ctx_nc(c);
  if (phases & DUST_PHASE_KICK) {
    if ((s = check_drag(c, p))) return s;
    if (c->drag_mode == DUST_DRAG_EPSTEIN)
      return fail(DUST_EUNSUPPORTED, "Epstein drag needs the gathered density: use the unfused dust_step");
    if (!vg_p) return fail(DUST_EINVAL, "vg_p is NULL");
    for (int k = 0; k < nc; ++k)
      if (p->n > 0 && !vg_p[k]) return fail(DUST_EINVAL, "vg_p[%d] is NULL", k);
  }
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(c->device));
  c->last_stream = st;
  if (c->det && (phases & DUST_PHASE_KICK) && (s = ensure_det(c, p->n))) return s;
  launch_set_time(c->tdev, frc->t, st);
  Forces F = forces_of(frc);
  return dispatch(c, [&](auto ts, auto ta) -> dust_status_t {
    using TS = decltype(ts);
    using A = decltype(ta);
    const TS* vg[3] = {nullptr, nullptr, nullptr};
    TS* imp[4] = {nullptr, nullptr, nullptr, nullptr};
    if (vg_p)
      for (int k = 0; k < nc; ++k) vg[k] = (const TS*)vg_p[k];
    if (impulse)
      for (int k = 0; k <= nc; ++k) imp[k] = (TS*)impulse[k];
    run_push<TS, A>(c, pview<TS>(p), F, dt, phases, vg, imp, c->diag, st);
    HIP_TRY(hipGetLastError());
    return DUST_OK;
  });
}

dust_status_t dust_deposit(void* ctx, const dust_particles_t* p, const void* const impulse[4],
                           dust_fields_t* f, void* stream) {
  g_err.clear();
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  dust_status_t s;
  if ((s = check_particles(c, p, false)) || (s = check_fields(c, f, false, true))) return s;
  int nc = ctx_nc(c);
  if (!impulse) return fail(DUST_EINVAL, "impulse is NULL");
  for (int k = 0; k <= nc; ++k)
    if (p->n > 0 && !impulse[k]) return fail(DUST_EINVAL, "impulse[%d] is NULL", k);
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(c->device));
  c->last_stream = st;
  if (c->det && (s = ensure_det(c, p->n))) return s;
  return dispatch(c, [&](auto ts, auto ta) -> dust_status_t {
    using TS = decltype(ts);
    using A = decltype(ta);
    const TS* imp[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k <= nc; ++k) imp[k] = (const TS*)impulse[k];
    if (c->det)
      deposit_det<TS, A, TS>(c, pview<TS>(p), fview<TS>(f), imp, st);
    else
      launch_deposit<TS, A, TS>(pview<TS>(p), c->boxes_d, c->nbox, c->geom, c->ndim, c->unif, fview<TS>(f), imp,
                                c->diag, st);
    HIP_TRY(hipGetLastError());
    return DUST_OK;
  });
}

dust_status_t dust_drag_source(void* ctx, const dust_particles_t* p, dust_fields_t* f, double dt,
                               const dust_forces_t* frc, void* stream) {
  g_err.clear();
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  dust_status_t s;
  if ((s = check_particles(c, p, true)) || (s = check_fields(c, f, true, true)) ||
      (s = check_forces(c, frc)) || (s = check_drag(c, p)))
    return s;
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(DUST_EINVAL, "dt must be finite and positive");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(c->device));
  c->last_stream = st;
  Forces F = forces_of(frc);
  if (c->det && ((s = ensure_det(c, p->n)) || (s = ensure_ws(c, p->n)))) return s;
  return dispatch(c, [&](auto ts, auto ta) -> dust_status_t {
    using TS = decltype(ts);
    using A = decltype(ta);
    if (c->det) {
      source_det<TS, A>(c, pview<TS>(p), fview<TS>(f), fview<TS>(f), F, dt, false, st);
      HIP_TRY(hipGetLastError());
      return DUST_OK;
    }
    if constexpr (std::is_same<TS, float>::value && std::is_same<A, float>::value) {
      const PView<float> pv = pview<float>(p);
      if (on_layout(c, pv) && use_c3(c, true, F, pv)) {
        const FView<float> fv = fview<float>(f);
        float* const out[3] = {fv.dep[0], fv.dep[1], fv.dep[2]};
        launch_c3_aux(c->plan, pv, c->boxes_d, c->nbox, fv, out, false, F, c->species_d, dt, c->bin_start,
                      c->n_active, c->diag, st);
        HIP_TRY(hipGetLastError());
        return DUST_OK;
      }
    }
    launch_drag_source<TS, A>(pview<TS>(p), c->boxes_d, c->nbox, c->geom, c->ndim, c->unif, fview<TS>(f), F,
                              c->species_d, c->drag_mode, dt, c->diag, st);
    HIP_TRY(hipGetLastError());
    return DUST_OK;
  });
}

dust_status_t dust_deposit_mass(void* ctx, const dust_particles_t* p, void* rho_d, void* stream) {
  g_err.clear();
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  dust_status_t s;
  if ((s = check_particles(c, p, false))) return s;
  if (p->n > 0 && !p->mass && !c->have_mass_table)
    return fail(DUST_EINVAL, "no per-particle mass and no species mass table");
  if (!rho_d) return fail(DUST_EINVAL, "rho_d is NULL");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(c->device));
  c->last_stream = st;
  if (c->det && ((s = ensure_det(c, p->n)) || (s = ensure_ws(c, p->n)))) return s;
  return dispatch(c, [&](auto ts, auto ta) -> dust_status_t {
    using TS = decltype(ts);
    using A = decltype(ta);
    if (c->det) {
      FView<TS> out{};
      out.dep[0] = (TS*)rho_d;
      source_det<TS, A>(c, pview<TS>(p), FView<TS>{}, out, Forces{}, 1.0, true, st);
      HIP_TRY(hipGetLastError());
      return DUST_OK;
    }
    if constexpr (std::is_same<TS, float>::value && std::is_same<A, float>::value) {
      const PView<float> pv = pview<float>(p);
      const Forces none{};
      if (on_layout(c, pv) && use_c3(c, true, none, pv)) {
        float* const out[3] = {(float*)rho_d, nullptr, nullptr};
        launch_c3_aux(c->plan, pv, c->boxes_d, c->nbox, FView<float>{}, out, true, none, c->species_d, 1.0,
                      c->bin_start, c->n_active, c->diag, st);
        HIP_TRY(hipGetLastError());
        return DUST_OK;
      }
    }
    launch_mass_density<TS, A>(pview<TS>(p), c->boxes_d, c->nbox, c->geom, c->ndim, c->unif, (TS*)rho_d,
                               c->species_d, c->diag, st);
    HIP_TRY(hipGetLastError());
    return DUST_OK;
  });
}

dust_status_t dust_apply_feedback(void* ctx, dust_fields_t* f, void* stream) {
  g_err.clear();
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  dust_status_t s;
  if ((s = check_fields(c, f, true, true))) return s;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(c->device));
  c->last_stream = st;
  return dispatch(c, [&](auto ts, auto) -> dust_status_t {
    using TS = decltype(ts);
    launch_feedback<TS>(c->boxes.data(), c->nbox, c->boxes_d, fview<TS>(f), st);
    HIP_TRY(hipGetLastError());
    return DUST_OK;
  });
}

dust_status_t dust_step(void* ctx, dust_particles_t* p, dust_fields_t* f, double dt,
                        const dust_forces_t* frc, int32_t nsteps, int32_t flags, void* stream) {
  g_err.clear();
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  dust_status_t s;
  if ((s = check_particles(c, p, true)) || (s = check_fields(c, f, true, true)) ||
      (s = check_forces(c, frc)) || (s = check_drag(c, p)))
    return s;
  if (!std::isfinite(dt)) return fail(DUST_EINVAL, "dt not finite");
  if (nsteps < 0) return fail(DUST_EINVAL, "nsteps < 0");
  if (flags & ~0xff1f) return fail(DUST_EINVAL, "unknown step flag bits");
  if (nsteps == 0) return DUST_OK;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(c->device));
  c->last_stream = st;
  // the deterministic mode runs the unfused chain
  if (c->det) {
    flags &= ~DUST_STEP_FUSED;
    if ((s = ensure_det(c, p->n))) return s;
  }
  if (!(flags & DUST_STEP_FUSED) && (s = ensure_ws(c, p->n))) return s;
  if (flags & DUST_STEP_FUSED) {
    if (frc->integrator != DUST_INTEGRATOR_EXPMID)
      return fail(DUST_EUNSUPPORTED, "the fused step takes the exponential midpoint kick only");
    if (c->drag_mode == DUST_DRAG_EPSTEIN)
      return fail(DUST_EUNSUPPORTED, "the fused step has no Epstein drag (unfused step only)");
    if ((s = ensure_bin(c, p->n)) || (s = ensure_bin_start(c)) || (s = ensure_shadow(c, p))) return s;
    if (!c->plan.ok) return fail(DUST_EUNSUPPORTED, "no fused plan for these boxes");
    if (fused_plan_reserve(c->plan, p->n) != DUST_OK) return fail(DUST_ENOMEM, "deferred-particle list");
    if (fused_lds_bytes(c->plan, ctx_nc(c), c->prec == DUST_F64 ? 8 : 4) + FUSED_STATIC_LDS > 160 * 1024 ||
        c3_lds_bytes(c->plan) + FUSED_STATIC_LDS > 160 * 1024)
      return fail(DUST_EUNSUPPORTED, "fused tile window needs more than 160 KiB of LDS");
  }
  Forces F = forces_of(frc);
  launch_set_time(c->tdev, frc->t, st);
  auto body = [&]() -> dust_status_t {
    c->prof_used = 0;
    return dispatch_arith(c, c->arith, [&](auto ts, auto ta) -> dust_status_t {
      using TS = decltype(ts);
      using A = decltype(ta);
      return run_steps<TS, A>(c, p, f, dt, F, nsteps, flags, st);
    });
  };
  if (!(flags & DUST_STEP_GRAPH)) {
    s = body();
    if (s) return s;
    HIP_TRY(hipGetLastError());
    return DUST_OK;
  }
  // graph: keyed by every argument except the start time (read on device)
  GraphKey key;
  auto put = [&](const void* ptr, size_t n) {
    const unsigned char* b = (const unsigned char*)ptr;
    key.bytes.insert(key.bytes.end(), b, b + n);
  };
  put(p, sizeof(*p));
  put(f, sizeof(*f));
  put(&dt, sizeof(dt));
  put(&F, sizeof(F));
  put(&nsteps, sizeof(nsteps));
  put(&flags, sizeof(flags));
  put(&st, sizeof(st));
  put(&c->arith, sizeof(c->arith));
  put(&c->stage_arith, sizeof(c->stage_arith));
  put(&c->tile, sizeof(c->tile));
  put(&c->rebin_default, sizeof(c->rebin_default));
  put(&c->plan.tiles_d, sizeof(c->plan.tiles_d));
  put(&c->plan.defer_list, sizeof(c->plan.defer_list));
  put(&c->shadow_mem, sizeof(c->shadow_mem));
  put(&c->bin_mem, sizeof(c->bin_mem));
  put(&c->bin_start, sizeof(c->bin_start));
  put(&c->ws, sizeof(c->ws));
  put(&c->prof_max, sizeof(c->prof_max));
  put(&c->det, sizeof(c->det));
  put(&c->det_part, sizeof(c->det_part));
  if (!(c->graph_exec && key == c->graph_key)) {
    if (c->graph_exec) {
      hipGraphExecDestroy(c->graph_exec);
      c->graph_exec = nullptr;
    }
    if (c->graph) {
      hipGraphDestroy(c->graph);
      c->graph = nullptr;
    }
    hipStream_t cap = st;
    bool own = false;
    if (cap == nullptr) {
      HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      own = true;
      HIP_TRY(hipStreamSynchronize(nullptr));
    }
    HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    hipStream_t saved = st;
    st = cap;
    s = body();
    st = saved;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cap, &g);
    if (s) {
      if (g) hipGraphDestroy(g);
      if (own) hipStreamDestroy(cap);
      return s;
    }
    if (e != hipSuccess) {
      if (own) hipStreamDestroy(cap);
      return fail(DUST_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    }
    c->graph = g;
    e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
    if (own) hipStreamDestroy(cap);
    if (e != hipSuccess) return fail(DUST_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
    c->graph_key = key;
  }
  HIP_TRY(hipGraphLaunch(c->graph_exec, st));
  return DUST_OK;
}


// Autotuner: times the fused step for every compiled tile shape and
// rebinning intervals 1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64 on copies of the caller's particles and fields,
// then keeps the fastest shape and interval in the context.
dust_status_t dust_ctx_autotune(void* ctx, const dust_particles_t* p, const dust_fields_t* f,
                                double dt, const dust_forces_t* frc, int32_t flags, int32_t steps,
                                int32_t* result, float* ms_per_step, void* stream) {
  g_err.clear();
  if (check_ctx(ctx)) return DUST_EINVAL;
  Ctx* c = (Ctx*)ctx;
  dust_status_t s;
  if ((s = check_particles(c, p, true)) || (s = check_fields(c, f, true, true)) ||
      (s = check_forces(c, frc)) || (s = check_drag(c, p)))
    return s;
  if (!std::isfinite(dt)) return fail(DUST_EINVAL, "dt not finite");
  if (steps < 1 || steps > 1000) return fail(DUST_EINVAL, "steps out of 1..1000");
  if (frc && frc->integrator != DUST_INTEGRATOR_EXPMID)
    return fail(DUST_EUNSUPPORTED, "the autotuner times the fused step (exponential midpoint kick)");
  if (c->drag_mode == DUST_DRAG_EPSTEIN)
    return fail(DUST_EUNSUPPORTED, "the autotuner times the fused step (no Epstein drag)");
  if (c->det)
    return fail(DUST_EUNSUPPORTED, "the autotuner times the fused step, which the deterministic mode does not run");
  if (flags & ~(DUST_STEP_APPLY_FEEDBACK | DUST_STEP_DIAG | DUST_STEP_NO_FILL))
    return fail(DUST_EINVAL, "autotune flags: only APPLY_FEEDBACK, DIAG, NO_FILL");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(c->device));
  const size_t n = (size_t)p->n, rs = real_size(c), ns = (size_t)c->n_stored;
  // scratch copies: particle arrays, then fields
  struct Arr { const void* src; void** dst; size_t bytes; };
  dust_particles_t pc = *p;
  dust_fields_t fc = *f;
  std::vector<Arr> arrs;
  auto add = [&](const void* src, void** dst, size_t bytes) {
    if (src) arrs.push_back({src, dst, bytes});
  };
  add(p->cell, (void**)&pc.cell, n * 4);
  for (int d = 0; d < 3; ++d) {
    add(p->off[d], &pc.off[d], n * rs);
    add(p->mom[d], &pc.mom[d], n * rs);
  }
  add(p->drag, (void**)&pc.drag, n * rs);
  add(p->mass, (void**)&pc.mass, n * rs);
  add(p->species, (void**)&pc.species, n);
  add(p->id, (void**)&pc.id, n * 4);
  add(f->rho, &fc.rho, ns * rs);
  for (int d = 0; d < 3; ++d) add(f->vel[d], &fc.vel[d], ns * rs);
  for (int d = 0; d < 4; ++d) add(f->dep[d], &fc.dep[d], ns * rs);
  size_t total = 0;
  for (auto& a : arrs) total += (a.bytes + 255) & ~(size_t)255;
  void* mem = nullptr;
  if (total && hipMalloc(&mem, total) != hipSuccess) return fail(DUST_ENOMEM, "autotune copies of %zu bytes", total);
  {
    char* q = (char*)mem;
    for (auto& a : arrs) {
      *a.dst = q;
      q += (a.bytes + 255) & ~(size_t)255;
    }
  }
  auto restore = [&]() -> dust_status_t {
    for (auto& a : arrs)
      HIP_TRY(hipMemcpyAsync(*a.dst, a.src, a.bytes, hipMemcpyDeviceToDevice, st));
    return DUST_OK;
  };
  // keep the caller's diagnostics and profiling state
  DiagDev saved{};
  HIP_TRY(hipMemcpy(&saved, c->diag, sizeof(DiagDev), hipMemcpyDeviceToHost));
  const int prof_max = c->prof_max;
  c->prof_max = 0;
  const TileShape keep_tile = c->tile;
  std::vector<TileShape> shapes;
  if (c->ndim > 2) {
    const int t3[6][3] = {{8, 8, 4}, {16, 4, 4}, {4, 16, 4}, {4, 4, 16}, {8, 4, 8}, {4, 8, 8}};
    for (auto& t : t3) shapes.push_back(TileShape{{t[0], t[1], t[2]}});
  } else {
    const int t2[3][2] = {{16, 16}, {32, 8}, {8, 32}};
    for (auto& t : t2) shapes.push_back(TileShape{{t[0], t[1], 1}});
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best = 1e30f;
  TileShape best_tile = keep_tile;
  int best_k = 1;
  s = DUST_OK;
  for (const TileShape& t : shapes) {
    c->tile = t;
    drop_graph(c);
    if (fused_plan_init(c->plan, c->boxes.data(), c->nbox, c->tile, c->slack) != DUST_OK) continue;
    if (fused_lds_bytes(c->plan, ctx_nc(c), (int)rs) + FUSED_STATIC_LDS > 160 * 1024) continue;
    static const int kIntervals[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};
    for (int ki = 0; ki < 12 && !s; ++ki) {
      const int k = kIntervals[ki];
      // whole intervals, so that every candidate pays its share of rebinning
      const int n = k * ((steps + k - 1) / k);
      if ((s = restore())) break;
      const int32_t fl = flags | DUST_STEP_FUSED | DUST_STEP_REBIN_EVERY(k);
      if ((s = dust_step(c, &pc, &fc, dt, frc, 1, fl, st))) break;  // warm-up
      if (hipEventRecord(e0, st) != hipSuccess) { s = fail(DUST_EDEVICE, "event record"); break; }
      if ((s = dust_step(c, &pc, &fc, dt, frc, n, fl, st))) break;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        s = fail(DUST_EDEVICE, "event sync");
        break;
      }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { s = fail(DUST_EDEVICE, "event time"); break; }
      ms /= (float)n;
      if (ms < best) {
        best = ms;
        best_tile = t;
        best_k = k;
      }
    }
    if (s) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  if (mem) (void)hipFree(mem);
  c->prof_max = prof_max;
  c->tile = s ? keep_tile : best_tile;
  drop_graph(c);
  c->lay_valid = false;
  dust_status_t s2 = fused_plan_init(c->plan, c->boxes.data(), c->nbox, c->tile, c->slack);
  HIP_TRY(hipMemcpy(c->diag, &saved, sizeof(DiagDev), hipMemcpyHostToDevice));
  if (s) return s;
  if (s2) return fail(s2, "fused plan");
  c->rebin_default = best_k;
  if (result) {
    result[0] = best_tile.t[0];
    result[1] = best_tile.t[1];
    result[2] = best_tile.t[2];
    result[3] = best_k;
  }
  if (ms_per_step) *ms_per_step = best;
  return DUST_OK;
}

}  // extern "C"
