// Fused tile step: plan (tile table), the dispatcher over geometries and the
// partial reduction, and the rebinning kernels (half-step keys, level-major
// permutation, particle copies).  The kernels themselves are in
// dust_fused_kern.h.
#include <algorithm>
#include <vector>

#include "dust_fused_kern.h"

namespace dust {

// Supported tile shapes (cells per axis, 256 cells each).
struct Shape3 { int x, y, z; };
static const Shape3 kShapes3[] = {{8, 8, 4}, {16, 4, 4}, {4, 16, 4}, {4, 4, 16}, {8, 4, 8}, {4, 8, 8}};
static const Shape3 kShapes2[] = {{16, 16, 1}, {32, 8, 1}, {8, 32, 1}};

static int shape_id(int ndim, TileShape t) {
  if (ndim > 2) {
    for (int s = 0; s < 6; ++s)
      if (kShapes3[s].x == t.t[0] && kShapes3[s].y == t.t[1] && kShapes3[s].z == t.t[2]) return s;
  } else {
    for (int s = 0; s < 3; ++s)
      if (kShapes2[s].x == t.t[0] && kShapes2[s].y == t.t[1]) return s;
  }
  return -1;
}

dust_status_t fused_plan_init(FusedPlan& plan, const Box* boxes, int nbox, TileShape tile, int slack) {
  (void)slack;
  fused_plan_free(plan);
  plan.tile = tile;
  plan.halo = FUSED_HALO;
  if (nbox < 1) return DUST_EINVAL;
  int ndim = boxes[0].ndim;
  if (ndim == 2) plan.tile.t[2] = 1;
  plan.shape = shape_id(ndim, plan.tile);
  if (plan.shape < 0) return DUST_EUNSUPPORTED;
  std::vector<TileDesc> tiles;
  plan.small = true;
  for (int b = 0; b < nbox; ++b) {
    const Box& B = boxes[b];
    if (B.ncell >= (1 << 24)) plan.small = false;
    int n[3] = {B.ax[0].n, B.ax[1].n, B.ndim > 2 ? B.ax[2].n : 1};
    int t[3] = {plan.tile.t[0], plan.tile.t[1], B.ndim > 2 ? plan.tile.t[2] : 1};
    int nt[3];
    for (int d = 0; d < 3; ++d) nt[d] = (n[d] + t[d] - 1) / t[d];
    int64_t key = B.cell_base;
    for (int tk = 0; tk < nt[2]; ++tk)
      for (int tj = 0; tj < nt[1]; ++tj)
        for (int ti = 0; ti < nt[0]; ++ti) {
          TileDesc d{};
          d.box = b;
          d.i0 = ti * t[0];
          d.j0 = tj * t[1];
          d.k0 = tk * t[2];
          d.ex = std::min(t[0], n[0] - d.i0);
          d.ey = std::min(t[1], n[1] - d.j0);
          d.ez = std::min(t[2], n[2] - d.k0);
          d.key0 = key;
          key += (int64_t)d.ex * d.ey * d.ez;
          tiles.push_back(d);
        }
  }
  int h2 = 2 * FUSED_HALO;
  plan.rmax[0] = plan.tile.t[0] + h2;
  plan.rmax[1] = plan.tile.t[1] + h2;
  plan.rmax[2] = ndim > 2 ? plan.tile.t[2] + h2 : 1;
  plan.lds_cells = (size_t)plan.rmax[0] * plan.rmax[1] * plan.rmax[2];
  plan.ntiles = (int)tiles.size();
  if (hipMalloc((void**)&plan.tiles_d, sizeof(TileDesc) * tiles.size()) != hipSuccess)
    return DUST_ENOMEM;
  if (hipMemcpy(plan.tiles_d, tiles.data(), sizeof(TileDesc) * tiles.size(), hipMemcpyHostToDevice) !=
      hipSuccess)
    return DUST_EDEVICE;
  if (hipMalloc((void**)&plan.part_d, sizeof(double) * PART_WORDS * (tiles.size() + DEFER_BLOCKS)) !=
          hipSuccess ||
      hipMalloc((void**)&plan.tile_map, 256 * tiles.size()) != hipSuccess ||
      hipMalloc((void**)&plan.defer_count, 256) != hipSuccess)
    return DUST_ENOMEM;
  if (hipMemset(plan.defer_count, 0, 256) != hipSuccess) return DUST_EDEVICE;
  plan.ok = true;
  return DUST_OK;
}

void fused_plan_free(FusedPlan& plan) {
  if (plan.tiles_d) (void)hipFree(plan.tiles_d);
  if (plan.part_d) (void)hipFree(plan.part_d);
  if (plan.defer_count) (void)hipFree(plan.defer_count);
  if (plan.defer_list) (void)hipFree(plan.defer_list);
  if (plan.tile_map) (void)hipFree(plan.tile_map);
  plan.tile_map = nullptr;
  plan.tiles_d = nullptr;
  plan.part_d = nullptr;
  plan.defer_count = nullptr;
  plan.defer_list = nullptr;
  plan.defer_cap = 0;
  plan.ok = false;
  plan.ntiles = 0;
}

// LDS of one workgroup: the FP64 deposit window ((nc+1) channels, padded to
// 32 bytes), then the gas window as one 4-vector of the storage type per cell
// (a single 16- or 32-byte LDS read gives every component of a cell).
static size_t fused_dep_doubles(size_t cells, int nc) { return (cells * (nc + 1) + 3) & ~(size_t)3; }

dust_status_t fused_plan_reserve(FusedPlan& plan, int64_t n) {
  if ((size_t)n <= plan.defer_cap && plan.defer_list) return DUST_OK;
  if (plan.defer_list) (void)hipFree(plan.defer_list);
  plan.defer_list = nullptr;
  plan.defer_cap = 0;
  size_t cap = (size_t)std::max<int64_t>(n, 1);
  // (slot written, particle read) pairs
  if (hipMalloc((void**)&plan.defer_list, 2 * cap * sizeof(uint32_t)) != hipSuccess) return DUST_ENOMEM;
  plan.defer_cap = cap;
  return DUST_OK;
}

size_t fused_lds_bytes(const FusedPlan& plan, int nc, int ts_bytes) {
  return fused_dep_doubles(plan.lds_cells, nc) * sizeof(double) + plan.lds_cells * 4 * (size_t)ts_bytes;
}

// Adds the per-workgroup partials of one fused launch to the diagnostics
// block, in a fixed order (one workgroup).
static constexpr int REDUCE_THREADS = 1024;
__global__ void __launch_bounds__(REDUCE_THREADS)
    k_reduce_fused_partials(const double* __restrict__ part, int n, DiagDev* dg, int sums,
                            uint32_t* defer_count) {
  constexpr int NW = REDUCE_THREADS / 64;
  static_assert(REDUCE_THREADS % PART_WORDS == 0 && 64 % PART_WORDS == 0, "word per lane");
  __shared__ double wred[NW][PART_WORDS];
  __shared__ double red[1][PART_WORDS];
  // the partials read as one flat array (coalesced): every element a thread
  // reads is word k = threadIdx.x % PART_WORDS of some slot; fixed order
  const int k = threadIdx.x % PART_WORDS;
  const bool is_max = k == 5;
  const int64_t total = (int64_t)n * PART_WORDS;
  double acc = 0.0;
#pragma unroll 8
  for (int64_t e = threadIdx.x; e < total; e += REDUCE_THREADS) {
    const double v = part[e];
    acc = is_max ? fmax(acc, v) : acc + v;
  }
  // lanes of the wave with the same word, in a fixed butterfly
  for (int off = PART_WORDS; off < 64; off <<= 1) {
    const double o = __shfl_xor(acc, off);
    acc = is_max ? fmax(acc, o) : acc + o;
  }
  if ((threadIdx.x & 63) < PART_WORDS) wred[threadIdx.x >> 6][k] = acc;
  __syncthreads();
  if (threadIdx.x < PART_WORDS) {
    double v = wred[0][k];
    for (int w = 1; w < NW; ++w) v = is_max ? fmax(v, wred[w][k]) : v + wred[w][k];
    red[0][k] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (dg && sums) {
      for (int k = 0; k < 3; ++k) dg->p_part[k] += red[0][k];
      dg->e_part += red[0][3];
      dg->sum_abs_j += red[0][4];
      atomic_max_nonneg(&dg->max_cells_bits, red[0][5]);
      if (red[0][5] > 1.8) atomicOr(&dg->flags, (unsigned)DUST_FLAG_CFL);
    }
    const unsigned long long fb = (unsigned long long)red[0][6];
    if (dg && fb) {
      dg->n_fallback += fb;
      atomicOr(&dg->flags, (unsigned)DUST_FLAG_TILE_OVERFLOW);
    }
    *defer_count = 0u;   // ready for the next launch (zeroed at set-up too)
  }
}


DUST_FUSED_G_ALL(extern, float, double)
DUST_FUSED_G_ALL(extern, float, float)
DUST_FUSED_G_ALL(extern, double, double)

template <typename TS, typename A>
void launch_fused(const FusedPlan& plan, const PView<TS>& p, const PView<TS>& q, bool copy_attrs,
                  const Box* boxes_d, int nbox, int geom, int ndim, int unif, const FView<TS>& fl,
                  const Forces& f, const Species* sp, int drag_mode, double dt, const double* tdev,
                  const int64_t* bin_start, const double* xg, DiagDev* dg, bool sums,
                  const uint32_t* src_index, hipEvent_t ev0, hipEvent_t ev1, hipStream_t st) {
  if (plan.ntiles == 0) return;
  double* part = plan.part_d;
  // (the deferred-particle count is zero here: set at set-up, and reset by
  // the partial reduction that ends every launch)
#define DUST_G(G, D, UU)                                                                          \
  launch_fused_g<TS, A, G, D, UU>(plan, p, q, copy_attrs, boxes_d, fl, f, sp, drag_mode, dt, tdev, \
                                  bin_start, xg, dg, part, sums, plan.defer_list,                  \
                                  plan.defer_count, src_index, nbox, ev0, ev1, st)
  if (geom == GEOM_CART && ndim == 2 && unif) DUST_G(GEOM_CART, 2, true);
  else if (geom == GEOM_CART && ndim == 2) DUST_G(GEOM_CART, 2, false);
  else if (geom == GEOM_CART && unif) DUST_G(GEOM_CART, 3, true);
  else if (geom == GEOM_CART) DUST_G(GEOM_CART, 3, false);
  else if (geom == GEOM_CYL) DUST_G(GEOM_CYL, 3, false);
  else DUST_G(GEOM_SPH, 3, false);
#undef DUST_G
  launch_reduce_fused(plan, dg, sums, st);
}

void launch_reduce_fused(const FusedPlan& plan, DiagDev* dg, bool sums, hipStream_t st) {
  if (plan.ntiles == 0) return;
  hipLaunchKernelGGL(k_reduce_fused_partials, dim3(1), dim3(REDUCE_THREADS), 0, st, (const double*)plan.part_d,
                     plan.ntiles + DEFER_BLOCKS, dg, (int)sums, plan.defer_count);
}

// ---------------------------------------------------------------- rebinning by half-step cell

// Tile-major key of the cell each particle reaches in the first half drift
// (the same drift the fused kernel does, so a particle is normally processed
// by the thread of the cell it kicks in).  A particle that leaves through an
// open face keeps the key of its current cell (the fused kernel removes it);
// a particle without a valid cell gets key nbins.  (The sort takes the
// particle indices as values.)
template <typename TS, typename A, int GEOM, int NDIM, bool U>
__global__ void __launch_bounds__(256)
    k_halfstep_keys(PView<TS> p, const Box* __restrict__ boxes, int nbox, Forces f, A dt,
                    const double* __restrict__ tdev, uint32_t nbins, TileShape ts,
                    uint32_t* __restrict__ key) {
  constexpr int nc = GEOM == GEOM_CART ? NDIM : 3;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  // every load issued before the cell is examined (one memory latency)
  const int64_t c = p.cell[i];
  A off[3], mom[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    off[d] = d < NDIM ? A(p.off[d][i]) : A(0);
    mom[d] = d < nc ? A(p.mom[d][i]) : A(0);
  }
  uint32_t k = nbins;
  auto key_in = [&](const Box& B) {
    int idx[3];
    unravel(B, c - B.cell_base, idx);
    const A h = A(0.5) * dt;
    int here[3] = {idx[0], idx[1], idx[2]};
    return drift_any<A, GEOM, NDIM, U>(B, f, true, h, *tdev + double(h), idx, off, mom)
               ? tile_key_idx(B, idx, ts) : tile_key_idx(B, here, ts);
  };
  if (c >= 0 && c < (int64_t)nbins) {
    // one box (the common case): its descriptor is uniform, read with
    // scalar loads; several boxes: the particle's box per lane
    if (nbox == 1)
      k = key_in(boxes[0]);
    else
      k = key_in(boxes[find_box(boxes, nbox, c)]);
  }
  // a key beyond the bins would break the sort's bin starts
  key[i] = k < nbins ? k : nbins;
}

template <typename TS, typename A>
void launch_halfstep_keys(const PView<TS>& p, const Box* boxes_d, int nbox, int geom, int ndim,
                          int unif, const Forces& f, double dt, const double* tdev, int64_t nbins,
                          TileShape ts, uint32_t* key, hipStream_t st) {
  if (p.n == 0) return;
  unsigned g = (unsigned)((p.n + 255) / 256);
#define DUST_K(G, D, UU)                                                                          \
  hipLaunchKernelGGL((k_halfstep_keys<TS, A, G, D, UU>), dim3(g), dim3(256), 0, st, p, boxes_d,     \
                     nbox, f, A(dt), tdev, (uint32_t)nbins, ts, key)
  if (geom == GEOM_CART && ndim == 2 && unif) DUST_K(GEOM_CART, 2, true);
  else if (geom == GEOM_CART && ndim == 2) DUST_K(GEOM_CART, 2, false);
  else if (geom == GEOM_CART && unif) DUST_K(GEOM_CART, 3, true);
  else if (geom == GEOM_CART) DUST_K(GEOM_CART, 3, false);
  else if (geom == GEOM_CYL) DUST_K(GEOM_CYL, 3, false);
  else DUST_K(GEOM_SPH, 3, false);
#undef DUST_K
}

// Copy particle `from` of src to slot `to` of dst (every array src has).
template <typename TS>
__device__ __forceinline__ void copy_particle(const PView<TS>& src, int64_t from, const PView<TS>& dst,
                                              int64_t to) {
  dst.cell[to] = src.cell[from];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (src.off[d]) dst.off[d][to] = src.off[d][from];
    if (src.mom[d]) dst.mom[d][to] = src.mom[d][from];
  }
  if (src.drag) dst.drag[to] = src.drag[from];
  if (src.mass) dst.mass[to] = src.mass[from];
  if (src.species) dst.species[to] = src.species[from];
  if (src.id) dst.id[to] = src.id[from];
}

// The level-major order of each tile's binned particles as a permutation:
// lm[slot] = perm[ps + j] for the j-th particle of a cell whose sorted range
// starts at ps (one workgroup per tile, one thread per cell: the fused
// kernel's mapping).
__global__ void __launch_bounds__(256)
    k_level_perm(const TileDesc* __restrict__ tiles, TileShape ts, const uint32_t* __restrict__ perm,
                 const int64_t* __restrict__ bin_start, uint32_t* __restrict__ lm) {
  const TileDesc td = tiles[blockIdx.x];
  const int TX = ts.t[0], TY = ts.t[1];
  const int lx = threadIdx.x % TX, ly = (threadIdx.x / TX) % TY, lz = threadIdx.x / (TX * TY);
  const bool own = lx < td.ex && ly < td.ey && lz < td.ez;
  int64_t ps = 0, pe = 0;
  if (own) {
    const int64_t key = td.key0 + lx + (int64_t)td.ex * (ly + (int64_t)td.ey * lz);
    ps = bin_start[key];
    pe = bin_start[key + 1];
  }
  const WaveLevels wl = wave_levels(own ? (int)(pe - ps) : 0, ps);
  uint32_t lvl = wl.base;
  for (int j = 0; j < wl.nlev; ++j) {
    const uint32_t to = level_slot(wl, j, lvl);
    if (wl.cnt > j) lm[to] = perm[ps + j];
  }
}

// Particles without a cell (sorted last, from slot bin_start[nbins] on), which
// no tile visits: dst[s] = src[perm[s]], or src[s] when perm is null (src and
// dst distinct).
template <typename TS>
__global__ void __launch_bounds__(256)
    k_copy_tail(PView<TS> src, PView<TS> dst, const uint32_t* __restrict__ perm,
                const int64_t* __restrict__ bin_start, int64_t nbins) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = bin_start[nbins] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < src.n;
       s += stride)
    copy_particle(src, perm ? (int64_t)perm[s] : s, dst, s);
}

// dst = src, every array.
template <typename TS>
__global__ void __launch_bounds__(256) k_copy_particles(PView<TS> src, PView<TS> dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < src.n; s += stride)
    copy_particle(src, s, dst, s);
}

template <typename TS>
void launch_level_perm(const FusedPlan& plan, const PView<TS>& src, const PView<TS>& dst,
                       const uint32_t* perm, const int64_t* bin_start, int64_t nbins, uint32_t* lm,
                       hipStream_t st) {
  if (src.n == 0) return;
  if (plan.ntiles > 0)
    hipLaunchKernelGGL(k_level_perm, dim3(plan.ntiles), dim3(256), 0, st, plan.tiles_d, plan.tile, perm,
                       bin_start, lm);
  // the tail is usually empty: a grid-stride loop
  unsigned g = (unsigned)std::min<int64_t>((src.n + 255) / 256, 512);
  hipLaunchKernelGGL(k_copy_tail<TS>, dim3(g), dim3(256), 0, st, src, dst, perm, bin_start, nbins);
}

template <typename TS>
void launch_copy_tail(const PView<TS>& src, const PView<TS>& dst, const int64_t* bin_start, int64_t nbins,
                      hipStream_t st, const uint32_t* perm) {
  if (src.n == 0) return;
  unsigned g = (unsigned)std::min<int64_t>((src.n + 255) / 256, 512);
  hipLaunchKernelGGL(k_copy_tail<TS>, dim3(g), dim3(256), 0, st, src, dst, perm, bin_start, nbins);
}

template <typename TS>
void launch_copy_particles(const PView<TS>& src, const PView<TS>& dst, hipStream_t st) {
  if (src.n == 0) return;
  unsigned g = (unsigned)std::min<int64_t>((src.n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_copy_particles<TS>, dim3(g), dim3(256), 0, st, src, dst);
}

#define DUST_FUSED_INST(TS, A)                                                                    \
  template void launch_fused<TS, A>(const FusedPlan&, const PView<TS>&, const PView<TS>&, bool,     \
                                    const Box*, int, int, int, int, const FView<TS>&,              \
                                    const Forces&, const Species*, int, double, const double*,     \
                                    const int64_t*, const double*, DiagDev*, bool, const uint32_t*, \
                                    hipEvent_t, hipEvent_t, hipStream_t);                          \
  template void launch_halfstep_keys<TS, A>(const PView<TS>&, const Box*, int, int, int, int,       \
                                            const Forces&, double, const double*, int64_t,         \
                                            TileShape, uint32_t*, hipStream_t);

DUST_FUSED_INST(float, double)
DUST_FUSED_INST(float, float)
DUST_FUSED_INST(double, double)

template void launch_level_perm<float>(const FusedPlan&, const PView<float>&, const PView<float>&,
                                       const uint32_t*, const int64_t*, int64_t, uint32_t*,
                                       hipStream_t);
template void launch_level_perm<double>(const FusedPlan&, const PView<double>&, const PView<double>&,
                                        const uint32_t*, const int64_t*, int64_t, uint32_t*,
                                        hipStream_t);
template void launch_copy_tail<float>(const PView<float>&, const PView<float>&, const int64_t*, int64_t,
                                      hipStream_t, const uint32_t*);
template void launch_copy_tail<double>(const PView<double>&, const PView<double>&, const int64_t*,
                                       int64_t, hipStream_t, const uint32_t*);
template void launch_copy_particles<float>(const PView<float>&, const PView<float>&, hipStream_t);
template void launch_copy_particles<double>(const PView<double>&, const PView<double>&, hipStream_t);

}  // namespace dust
