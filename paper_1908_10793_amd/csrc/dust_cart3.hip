// Fused tile step for uniform 3-D Cartesian boxes in FP32: the rebinning
// kernels (half-step keys with this path's drift; the ranking of each tile's
// cells by particle count and the source index of every slot) and the
// dispatcher over tile shapes.  The kernel is in dust_cart3_kern.h.
#include "dust_cart3_aux.h"

namespace dust {

DUST_C3_SHAPES(extern)
DUST_C3_AUX_SHAPES(extern)

// Rebinning: order the cells of every tile for the tile kernel's threads
// into tmap, and write lm[slot] = perm[ps + j], the source of every slot of
// the level-major layout that c3_layout describes.
//
// A wave runs as many levels as its fullest cell, so its cells should have
// similar counts; and its 64 lanes read the gas window at their cells'
// stencils, where lanes whose float4 fall in the same LDS bank group
// (window index mod 16) serialise.  The cells are therefore ranked by count
// (descending, ties by tile-local index) within each bank group, and ordered
// by (rank, group): a wave of a full tile takes 4 ranks of every group, and
// every 16 consecutive lanes hold one cell of each group.  (rx, ry: x and y
// extents of the tile kernel's gas window.)
__global__ void __launch_bounds__(256)
    k_c3_level_perm(const TileDesc* __restrict__ tiles, const uint32_t* __restrict__ perm,
                    const int64_t* __restrict__ bin_start, uint8_t* __restrict__ tmap,
                    uint32_t* __restrict__ lm, int rx, int ry) {
  __shared__ int cnt_s[256];
  __shared__ int grp_s[256];
  __shared__ int gsize[16];
  __shared__ uint8_t map_s[256];
  const TileDesc td = tiles[blockIdx.x];
  const int nct = td.ex * td.ey * td.ez;
  const int t = threadIdx.x;
  const int c = t < nct ? (int)(bin_start[td.key0 + t + 1] - bin_start[td.key0 + t]) : -1;
  int g = -1;
  if (t < nct) {
    const int lx = t % td.ex, ly = (t / td.ex) % td.ey, lz = t / (td.ex * td.ey);
    g = ((lx + FUSED_HALO) + rx * ((ly + FUSED_HALO) + ry * (lz + FUSED_HALO))) & 15;
  }
  cnt_s[t] = c;
  grp_s[t] = g;
  if (t < 16) gsize[t] = 0;
  __syncthreads();
  if (t < nct) atomicAdd(&gsize[g], 1);
  __syncthreads();
  if (t < nct) {
    int rank = 0;
    for (int u = 0; u < nct; ++u) {
      const int cu = cnt_s[u];
      rank += (grp_s[u] == g && (cu > c || (cu == c && u < t))) ? 1 : 0;
    }
    // position in (rank, group) order
    int pos = 0;
    for (int k = 0; k < 16; ++k) {
      const int sz = gsize[k];
      pos += min(sz, rank) + ((k < g && sz > rank) ? 1 : 0);
    }
    map_s[pos] = (uint8_t)t;
  }
  __syncthreads();
  const int lc = t < nct ? (int)map_s[t] : -1;
  tmap[(size_t)blockIdx.x * 256 + t] = (uint8_t)(lc < 0 ? 0 : lc);
  int64_t ps;
  const WaveLevels wl = c3_layout(td, lc, bin_start, ps);
  uint32_t lvl = wl.base;
  // four levels at a time: a lane's four sources share a cache line, and
  // their loads issue together
  for (int j0 = 0; j0 < wl.nlev; j0 += 4) {
    uint32_t src[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) src[q] = wl.cnt > j0 + q ? perm[ps + j0 + q] : 0u;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (j0 + q >= wl.nlev) break;   // (wave-uniform)
      const uint32_t to = level_slot(wl, j0 + q, lvl);
      if (wl.cnt > j0 + q) lm[to] = src[q];
    }
  }
}

// Half-step tile keys with the drift of the fast path (a particle is then
// normally processed by the thread of the cell it kicks in).
__global__ void __launch_bounds__(256)
    k_c3_keys(PView<float> p, const Box* __restrict__ boxes, int nbox, float dt,
              uint32_t nbins, TileShape ts, uint32_t* __restrict__ key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const int32_t c = p.cell[i];
  float off[3], mom[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    off[d] = p.off[d][i];
    mom[d] = p.mom[d][i];
  }
  uint32_t k = nbins;
  if (c >= 0 && c < (int32_t)nbins) {
    const Box& B = nbox == 1 ? boxes[0] : boxes[find_box(boxes, nbox, c)];
    const C3Box cb = c3_box(B, dt);
    int idx[3];
    c3_unravel(c - cb.cell_base, cb.n[0], cb.n[1], B.ax[0].inv_n, B.ax[1].inv_n, idx);
    int nx[3];
    bool in = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      nx[d] = c3_move(idx[d], off[d], mom[d], cb.hinv[d]);
      if (nx[d] < 0 || nx[d] >= cb.n[d]) {
        if (cb.per[d]) nx[d] = c3_wrap(nx[d], cb.n[d]);
        else in = false;
      }
    }
    k = tile_key_idx(B, in ? nx : idx, ts);
  }
  // a key beyond the bins would break the sort's bin starts
  key[i] = k < nbins ? k : nbins;
}

size_t c3_lds_bytes(const FusedPlan& plan) {
  return (size_t)plan.lds_cells * (4 * sizeof(double) + sizeof(float4));
}

void launch_c3(const FusedPlan& plan, const PView<float>& p, const PView<float>& q, bool copy_attrs,
               const Box* boxes_d, int nbox, const FView<float>& fl, const Forces& f, const Species* sp,
               int drag_mode, double dt, const double* tdev, const int64_t* bin_start, const double* xg,
               DiagDev* dg, bool sums, const uint32_t* src_index, hipEvent_t ev0, hipEvent_t ev1,
               hipStream_t st) {
  if (plan.ntiles == 0) return;
  if (ev0) (void)hipEventRecord(ev0, st);
#define DUST_C3(TX, TY, TZ)                                                                             \
  launch_c3_shape<TX, TY, TZ>(plan, p, q, copy_attrs, boxes_d, fl, f, sp, drag_mode, dt, tdev, bin_start,  \
                              xg, dg, sums, src_index, st)
  switch (plan.shape) {
    case 0: DUST_C3(8, 8, 4); break;
    case 1: DUST_C3(16, 4, 4); break;
    case 2: DUST_C3(4, 16, 4); break;
    case 3: DUST_C3(4, 4, 16); break;
    case 4: DUST_C3(8, 4, 8); break;
    default: DUST_C3(4, 8, 8); break;
  }
#undef DUST_C3
  if (ev1) (void)hipEventRecord(ev1, st);
  hipLaunchKernelGGL((k_fused_deferred<float, float, GEOM_CART, 3, true>), dim3(DEFER_BLOCKS), dim3(256), 0, st,
                     p, q, (int)copy_attrs, boxes_d, nbox, fl, f, sp, drag_mode, float(dt), tdev, xg,
                     (const uint32_t*)plan.defer_list, (const uint32_t*)plan.defer_count, plan.part_d,
                     plan.ntiles, (int)sums, dg);
  launch_reduce_fused(plan, dg, sums, st);
}

void launch_c3_aux(const FusedPlan& plan, const PView<float>& p, const Box* boxes_d, int nbox,
                   const FView<float>& fl, float* const out[3], bool mass, const Forces& f, const Species* sp,
                   double dt, const int64_t* bin_start, int64_t nbins, DiagDev* dg, hipStream_t st) {
  if (plan.ntiles == 0 && p.n == 0) return;
#define DUST_C3A(TX, TY, TZ) \
  launch_c3_aux_shape<TX, TY, TZ>(plan, p, boxes_d, nbox, fl, out, mass, f, sp, dt, bin_start, nbins, dg, st)
  switch (plan.shape) {
    case 0: DUST_C3A(8, 8, 4); break;
    case 1: DUST_C3A(16, 4, 4); break;
    case 2: DUST_C3A(4, 16, 4); break;
    case 3: DUST_C3A(4, 4, 16); break;
    case 4: DUST_C3A(8, 4, 8); break;
    default: DUST_C3A(4, 8, 8); break;
  }
#undef DUST_C3A
}

void launch_c3_keys(const PView<float>& p, const Box* boxes_d, int nbox, double dt, int64_t nbins,
                    TileShape ts, uint32_t* key, hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_c3_keys, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, st, p, boxes_d, nbox,
                     float(dt), (uint32_t)nbins, ts, key);
}

void launch_c3_level_perm(const FusedPlan& plan, const uint32_t* perm, const int64_t* bin_start,
                          uint32_t* lm, hipStream_t st) {
  if (plan.ntiles > 0)
    hipLaunchKernelGGL(k_c3_level_perm, dim3(plan.ntiles), dim3(256), 0, st, plan.tiles_d, perm, bin_start,
                       plan.tile_map, lm, plan.tile.t[0] + 2 * FUSED_HALO, plan.tile.t[1] + 2 * FUSED_HALO);
}

}  // namespace dust
