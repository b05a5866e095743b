// Fused gather - exponential-midpoint push - deposit kernel (gfx950).
//
// One workgroup per grid tile.  Particles are binned tile by tile (tile-major
// keys), so a tile's particles are one contiguous range.  The workgroup
// stages the gas velocity of the tile plus a halo in LDS, then each thread
// takes particles: half drift, weights at x^{n+1/2}, gather from LDS, kick,
// drag impulse and energy accumulated into an LDS copy of the deposit window
// (the same weights as the gather), second half drift, store.  The window is
// finally added to the global deposit arrays (scaled by the inverse cell
// volume) with one atomic per touched cell and channel.  A particle whose
// stencil at x^{n+1/2} leaves the window (it moved too far since the last
// binning, or wrapped across a periodic face) takes the same arithmetic
// against global memory instead.
//
// Lanes of a wave are spread across the tile's particle range (stride of a
// few cells) so that the LDS atomics of one instruction rarely hit the same
// cell.
#include <algorithm>
#include <vector>

#include "dust_device.h"
#include "dust_fused.h"
#include "dust_launch.h"
#include "dust_particle.h"

namespace dust {

static constexpr int FUSED_THREADS = 256;
static constexpr int FUSED_K = 2;  // particles per thread per chunk
static constexpr int FUSED_CHUNK = FUSED_THREADS * FUSED_K;

dust_status_t fused_plan_init(FusedPlan& plan, const Box* boxes, int nbox, TileShape tile, int slack) {
  fused_plan_free(plan);
  plan.tile = tile;
  plan.halo = 2 + slack;
  std::vector<TileDesc> tiles;
  int rmax[3] = {1, 1, 1};
  for (int b = 0; b < nbox; ++b) {
    const Box& B = boxes[b];
    int n[3] = {B.ax[0].n, B.ax[1].n, B.ndim > 2 ? B.ax[2].n : 1};
    int t[3] = {tile.t[0], tile.t[1], B.ndim > 2 ? tile.t[2] : 1};
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
          rmax[0] = std::max(rmax[0], d.ex + 2 * plan.halo);
          rmax[1] = std::max(rmax[1], d.ey + 2 * plan.halo);
          rmax[2] = std::max(rmax[2], B.ndim > 2 ? d.ez + 2 * plan.halo : 1);
        }
  }
  for (int d = 0; d < 3; ++d) plan.rmax[d] = rmax[d];
  plan.lds_cells = (size_t)rmax[0] * rmax[1] * rmax[2];
  // 3 gas components + 4 deposit channels, at most 8 bytes each
  if (plan.lds_cells * 7 * 8 > 160 * 1024 && plan.lds_cells * 7 * 4 > 160 * 1024) return DUST_EUNSUPPORTED;
  plan.ntiles = (int)tiles.size();
  if (hipMalloc((void**)&plan.tiles_d, sizeof(TileDesc) * tiles.size()) != hipSuccess)
    return DUST_ENOMEM;
  if (hipMemcpy(plan.tiles_d, tiles.data(), sizeof(TileDesc) * tiles.size(), hipMemcpyHostToDevice) !=
      hipSuccess)
    return DUST_EDEVICE;
  plan.ok = true;
  return DUST_OK;
}

void fused_plan_free(FusedPlan& plan) {
  if (plan.tiles_d) hipFree(plan.tiles_d);
  plan.tiles_d = nullptr;
  plan.ok = false;
  plan.ntiles = 0;
}

template <typename TS, typename A, int GEOM, int NDIM>
__global__ void __launch_bounds__(FUSED_THREADS)
    k_fused(const TileDesc* tiles, PView<TS> p, const Box* boxes, FView<TS> fl, Forces f,
            const Species* sp, int drag_mode, A dt, const double* tdev, const int64_t* bin_start,
            int halo, DiagDev* dg, int sums) {
  constexpr int nc = GEOM == GEOM_CART ? NDIM : 3;
  constexpr int c2 = NDIM > 2 ? 1 : 0;
  extern __shared__ unsigned char smem_raw[];
  TS* smem = reinterpret_cast<TS*>(smem_raw);
  const TileDesc td = tiles[blockIdx.x];
  const Box& B = boxes[td.box];
  const int hz = NDIM > 2 ? halo : 0;
  const int rx = td.ex + 2 * halo, ry = td.ey + 2 * halo, rz = td.ez + 2 * hz;
  const int rcells = rx * ry * rz;
  const int ox = td.i0 - halo, oy = td.j0 - halo, oz = td.k0 - hz;  // region origin
  TS* gas = smem;                       // nc * rcells
  TS* dep = smem + (size_t)nc * rcells; // (nc+1) * rcells
  const double t0 = *tdev;
  const A h = A(0.5) * dt;
  const int n0 = B.ax[0].n, n1 = B.ax[1].n, n2 = NDIM > 2 ? B.ax[2].n : 1;

  // stage gas, clear deposit window
  for (int r = threadIdx.x; r < rcells; r += FUSED_THREADS) {
    int a = r % rx, bq = (r / rx) % ry, cq = r / (rx * ry);
    int i = ox + a, j = oy + bq, k = oz + cq;
    bool in = i >= -1 && i <= n0 && j >= -1 && j <= n1 && (NDIM < 3 || (k >= -1 && k <= n2));
    int64_t id = in ? stored_index(B, i, j, k) : 0;
#pragma unroll
    for (int m = 0; m < nc; ++m) gas[m * rcells + r] = in ? fl.vel[m][id] : TS(0);
#pragma unroll
    for (int m = 0; m <= nc; ++m) dep[m * rcells + r] = TS(0);
  }
  __syncthreads();

  const int64_t ps = bin_start[td.key0];
  const int64_t pe = bin_start[td.key0 + (int64_t)td.ex * td.ey * td.ez];
  double s_j[3] = {0, 0, 0}, s_e = 0, s_abs = 0, s_cells = 0;
  unsigned long long n_fb = 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

  for (int64_t cs = ps; cs < pe; cs += FUSED_CHUNK) {
#pragma unroll 1
    for (int r = 0; r < FUSED_K; ++r) {
      // lanes spread FUSED_K*4 particles apart inside the chunk
      int64_t i = cs + (int64_t)lane * (4 * FUSED_K) + wv * FUSED_K + r;
      if (i >= pe) continue;
      int idx[3];
      A off[3], mom[3];
      int32_t cid = p.cell[i];
      if (cid < 0 || cid < B.cell_base || cid >= B.cell_base + B.ncell) {
        if (cid >= 0) flag(dg, DUST_FLAG_BAD_CELL);
        continue;
      }
      unravel(B, cid - B.cell_base, idx);
      bool bad = false;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        off[d] = d < NDIM ? A(p.off[d][i]) : A(0);
        mom[d] = d < nc ? A(p.mom[d][i]) : A(0);
        bad |= !(off[d] >= A(-0.5) && off[d] < A(0.5));
      }
      if (bad) flag(dg, DUST_FLAG_OFFSET_RANGE);
      // half drift to x^{n+1/2}
      if (!drift<A, GEOM, NDIM>(B, f, true, h, t0 + double(h), idx, off, mom)) {
        store_particle<TS, A, GEOM, NDIM>(p, B, f, t0 + double(h), i, false, idx, off, mom, dg);
        continue;
      }
      // weights at x^{n+1/2}
      Stencil<A> s;
      stencil_weights<A, NDIM>(B, idx, off, s);
      const int la = idx[0] - ox, lb = idx[1] - oy, lc = idx[2] - oz;
      const bool inside = la >= 1 && la <= rx - 2 && lb >= 1 && lb <= ry - 2 &&
                          (c2 == 0 || (lc >= 1 && lc <= rz - 2));
      // gather (Eq. Delta_vp)
      A v[3] = {A(0), A(0), A(0)};
      if (inside) {
        const int base = la + rx * (lb + ry * lc);
#pragma unroll
        for (int c = -c2; c <= c2; ++c)
#pragma unroll
          for (int bb = -1; bb <= 1; ++bb) {
            A wbc = s.w[1][bb + 1] * s.w[2][c + 1];
#pragma unroll
            for (int a = -1; a <= 1; ++a) {
              A w = s.w[0][a + 1] * wbc;
              int r0 = base + a + rx * (bb + ry * c);
#pragma unroll
              for (int m = 0; m < nc; ++m) v[m] += w * A(gas[m * rcells + r0]);
            }
          }
      } else {
#pragma unroll
        for (int c = -c2; c <= c2; ++c)
#pragma unroll
          for (int bb = -1; bb <= 1; ++bb) {
            A wbc = s.w[1][bb + 1] * s.w[2][c + 1];
#pragma unroll
            for (int a = -1; a <= 1; ++a) {
              A w = s.w[0][a + 1] * wbc;
              int64_t id = stored_index(B, idx[0] + a, idx[1] + bb, idx[2] + c);
#pragma unroll
              for (int m = 0; m < nc; ++m) v[m] += w * A(fl.vel[m][id]);
            }
          }
      }
      // kick
      Where<A> wh;
      where<A, GEOM, NDIM>(B, idx, off, wh);
      A pg[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) pg[m] = m < nc ? v[m] * wh.sc[m] : A(0);
      int spc = p.species ? p.species[i] : 0;
      if (spc >= sp->n) {
        flag(dg, DUST_FLAG_BAD_CELL);
        spc = 0;
      }
      A dval = drag_mode == DRAG_SPECIES ? A(sp->tau[spc]) : A(p.drag[i]);
      A m = p.mass ? A(p.mass[i]) : A(sp->mass[spc]);
      A it = inverse_tau<A, GEOM>(f, drag_mode, dval, wh);
      KickOut<A> o;
      kick<A, GEOM, NDIM>(B, f, dt, it, wh, mom, pg, o);
      A q[4] = {A(0), A(0), A(0), A(0)};
#pragma unroll
      for (int k = 0; k < nc; ++k) {
        q[k] = m * o.j[k];
        if (sums) {
          A vbar = (mom[k] + A(0.5) * o.dp[k]) / wh.sc[k];
          A dl = cell_width<A>(B.ax[k], idx[k]) * (GEOM == GEOM_CART || k == 0 ? A(1) : wh.sc[k]);
          double cps = fabs(double(vbar * dt / dl));
          s_cells = cps > s_cells ? cps : s_cells;
          s_j[k] += double(q[k]);
          s_abs += fabs(double(q[k]));
        }
        mom[k] += o.dp[k];
      }
      q[nc] = m * o.e;
      if (sums) s_e += double(q[nc]);
      // deposit (Eq. dust_feedback_final), same weights and cells as the gather
      if (inside) {
        const int base = la + rx * (lb + ry * lc);
        TS qs[4];
#pragma unroll
        for (int k = 0; k <= nc; ++k) qs[k] = TS(-q[k]);
#pragma unroll
        for (int c = -c2; c <= c2; ++c)
#pragma unroll
          for (int bb = -1; bb <= 1; ++bb) {
            A wbc = s.w[1][bb + 1] * s.w[2][c + 1];
#pragma unroll
            for (int a = -1; a <= 1; ++a) {
              TS w = TS(s.w[0][a + 1] * wbc);
              int r0 = base + a + rx * (bb + ry * c);
#pragma unroll
              for (int k = 0; k <= nc; ++k) atomicAdd(&dep[k * rcells + r0], w * qs[k]);
            }
          }
      } else {
        ++n_fb;
#pragma unroll
        for (int c = -c2; c <= c2; ++c)
#pragma unroll
          for (int bb = -1; bb <= 1; ++bb) {
            A wbc = s.w[1][bb + 1] * s.w[2][c + 1];
#pragma unroll
            for (int a = -1; a <= 1; ++a) {
              int ii = idx[0] + a, jj = idx[1] + bb, kk = idx[2] + c;
              A w = s.w[0][a + 1] * wbc * A(inv_volume(B, ii, jj, kk));
              int64_t id = stored_index(B, ii, jj, kk);
#pragma unroll
              for (int k = 0; k <= nc; ++k) unsafeAtomicAdd(&fl.dep[k][id], TS(-w * q[k]));
            }
          }
      }
      // second half drift to x^{n+1}
      bool alive = drift<A, GEOM, NDIM>(B, f, false, h, t0 + double(dt), idx, off, mom);
      store_particle<TS, A, GEOM, NDIM>(p, B, f, t0 + double(dt), i, alive, idx, off, mom, dg);
    }
  }
  __syncthreads();

  // add the deposit window to the grid
  for (int r = threadIdx.x; r < rcells; r += FUSED_THREADS) {
    int a = r % rx, bq = (r / rx) % ry, cq = r / (rx * ry);
    int i = ox + a, j = oy + bq, k = oz + cq;
    bool in = i >= -1 && i <= n0 && j >= -1 && j <= n1 && (NDIM < 3 || (k >= -1 && k <= n2));
    if (!in) continue;
    int64_t id = stored_index(B, i, j, k);
    double iv = inv_volume(B, i, j, k);
#pragma unroll
    for (int m = 0; m <= nc; ++m) {
      TS x = dep[m * rcells + r];
      if (x != TS(0)) unsafeAtomicAdd(&fl.dep[m][id], TS(double(x) * iv));
    }
  }

  if (dg) {
    if (sums) {
      for (int k = 0; k < 3; ++k) s_j[k] = wave_sum(s_j[k]);
      s_e = wave_sum(s_e);
      s_abs = wave_sum(s_abs);
      s_cells = wave_max(s_cells);
    }
    unsigned long long fb = wave_sum(n_fb);
    if (lane == 0) {
      if (sums) {
        for (int k = 0; k < 3; ++k) unsafeAtomicAdd(&dg->p_part[k], s_j[k]);
        unsafeAtomicAdd(&dg->e_part, s_e);
        unsafeAtomicAdd(&dg->sum_abs_j, s_abs);
        atomic_max_nonneg(&dg->max_cells_bits, s_cells);
        if (s_cells > 1.8) atomicOr(&dg->flags, (unsigned)DUST_FLAG_CFL);
      }
      if (fb) {
        atomicAdd(&dg->n_fallback, fb);
        atomicOr(&dg->flags, (unsigned)DUST_FLAG_TILE_OVERFLOW);
      }
    }
  }
}

template <typename TS, typename A, int GEOM, int NDIM>
static void launch_fused_g(const FusedPlan& plan, const PView<TS>& p, const Box* boxes_d,
                           const FView<TS>& fl, const Forces& f, const Species* sp, int drag_mode,
                           double dt, const double* tdev, const int64_t* bin_start, DiagDev* dg,
                           bool sums, hipStream_t st) {
  size_t lds = plan.lds_cells * 7 * sizeof(TS);
  if (lds > 160 * 1024) return;  // rejected on the host before any launch
  if (lds > 64 * 1024) {
    static bool raised = false;
    if (!raised) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused<TS, A, GEOM, NDIM>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      raised = true;
    }
  }
  hipLaunchKernelGGL((k_fused<TS, A, GEOM, NDIM>), dim3(plan.ntiles), dim3(FUSED_THREADS), lds, st,
                     plan.tiles_d, p, boxes_d, fl, f, sp, drag_mode, A(dt), tdev, bin_start,
                     plan.halo, dg, (int)sums);
}

template <typename TS, typename A>
void launch_fused(const FusedPlan& plan, const PView<TS>& p, const Box* boxes_d, int nbox, int geom,
                  int ndim, const FView<TS>& fl, const Forces& f, const Species* sp, int drag_mode,
                  double dt, const double* tdev, const int64_t* bin_start, DiagDev* dg, bool sums,
                  hipStream_t st) {
  (void)nbox;
  if (plan.ntiles == 0) return;
  if (geom == GEOM_CART && ndim == 2)
    launch_fused_g<TS, A, GEOM_CART, 2>(plan, p, boxes_d, fl, f, sp, drag_mode, dt, tdev, bin_start,
                                        dg, sums, st);
  else if (geom == GEOM_CART)
    launch_fused_g<TS, A, GEOM_CART, 3>(plan, p, boxes_d, fl, f, sp, drag_mode, dt, tdev, bin_start,
                                        dg, sums, st);
  else if (geom == GEOM_CYL)
    launch_fused_g<TS, A, GEOM_CYL, 3>(plan, p, boxes_d, fl, f, sp, drag_mode, dt, tdev, bin_start,
                                       dg, sums, st);
  else
    launch_fused_g<TS, A, GEOM_SPH, 3>(plan, p, boxes_d, fl, f, sp, drag_mode, dt, tdev, bin_start,
                                       dg, sums, st);
}

#define DUST_FUSED_INST(TS, A)                                                                    \
  template void launch_fused<TS, A>(const FusedPlan&, const PView<TS>&, const Box*, int, int, int,  \
                                    const FView<TS>&, const Forces&, const Species*, int, double,  \
                                    const double*, const int64_t*, DiagDev*, bool, hipStream_t);

DUST_FUSED_INST(float, double)
DUST_FUSED_INST(float, float)
DUST_FUSED_INST(double, double)

}  // namespace dust
