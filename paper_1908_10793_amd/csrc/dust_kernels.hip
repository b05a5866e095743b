// Unfused per-phase kernels of the dust hot path (gfx950): drift, gather,
// exponential-midpoint kick, deposit, ghost fill / fold, feedback and FP64
// conservation sums.  One thread per particle (or per grid cell); all the
// per-particle arithmetic lives in dust_device.h and is shared with the
// fused kernel.
#include "dust_device.h"
#include "dust_fused.h"
#include "dust_launch.h"
#include "dust_particle.h"

namespace dust {

// ---------------------------------------------------------------- particle kernels
// Templated on the geometry and dimension of the context's boxes so that the
// stencil and component loops unroll into registers.

template <typename TS, typename A, int GEOM, int NDIM, bool U>
__global__ void __launch_bounds__(256) k_drift(PView<TS> p, const Box* boxes, int nbox, Forces f,
                                               A h, const double* tdev, double toff, int first,
                                               DiagDev* dg) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const double t_after = *tdev + toff;
  int idx[3];
  A off[3], mom[3];
  int b = load_particle<TS, A, GEOM, NDIM>(p, boxes, nbox, i, idx, off, mom, dg);
  if (b < 0) return;
  const Box& B = boxes[b];
  bool alive = drift_any<A, GEOM, NDIM, U>(B, f, first != 0, h, t_after, idx, off, mom);
  store_particle_any<TS, A, GEOM, NDIM>(p, B, f, t_after, i, alive, idx, off, mom, dg);
}

template <typename TS, typename A, typename TW, int GEOM, int NDIM, bool U>
__global__ void __launch_bounds__(256) k_gather(PView<TS> p, const Box* boxes, int nbox,
                                                FView<TS> fl, const double* xg, TW* rho_p,
                                                TW* vg0, TW* vg1, TW* vg2, DiagDev* dg) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  int idx[3];
  A off[3], mom[3];
  int b = load_particle<TS, A, GEOM, NDIM>(p, boxes, nbox, i, idx, off, mom, dg);
  if (b < 0) return;
  const Box& B = boxes[b];
  Stencil<A> s;
  stencil_weights<A, GEOM, NDIM, U>(B, idx, off, s);
  constexpr int nc = GEOM == GEOM_CART ? NDIM : 3;
  constexpr int c2 = NDIM > 2 ? 1 : 0;
  A r = A(0), v[3] = {A(0), A(0), A(0)};
#pragma unroll
  for (int c = -c2; c <= c2; ++c)
#pragma unroll
    for (int bb = -1; bb <= 1; ++bb) {
      A wbc = s.w[1][bb + 1] * s.w[2][c + 1];
#pragma unroll
      for (int a = -1; a <= 1; ++a) {
        A w = s.w[0][a + 1] * wbc;
        int64_t id = stored_index(B, idx[0] + a, idx[1] + bb, idx[2] + c);
        if (rho_p) r += w * A(fl.rho[id]);
#pragma unroll
        for (int m = 0; m < nc; ++m) v[m] += w * A(gas_comp(B, fl, xg, m, idx[0] + a, idx[1] + bb, idx[2] + c));
      }
    }
  if (rho_p) rho_p[i] = TW(r);
  if (vg0) vg0[i] = TW(v[0]);
  if (vg1) vg1[i] = TW(v[1]);
  if (nc > 2 && vg2) vg2[i] = TW(v[2]);
}

template <typename TS, typename A, typename TW, int GEOM, int NDIM, bool U>
__global__ void __launch_bounds__(256) k_kick(PView<TS> p, const Box* boxes, int nbox, Forces f,
                                              const Species* sp, int drag_mode, A dt, const TW* rho_p,
                                              const TW* vg0,
                                              const TW* vg1, const TW* vg2, TW* imp0, TW* imp1,
                                              TW* imp2, TW* imp3, DiagDev* dg, double* part) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int nc = GEOM == GEOM_CART ? NDIM : 3;
  double sums[5] = {0, 0, 0, 0, 0};
  double cells = 0.0;
  if (i < p.n) {
    int idx[3];
    A off[3], mom[3];
    int b = load_particle<TS, A, GEOM, NDIM>(p, boxes, nbox, i, idx, off, mom, dg);
    if (b >= 0) {
      const Box& B = boxes[b];
      Where<A> w;
      where<A, GEOM, NDIM, U>(B, idx, off, w);
      // slip: canonical gas momentum at the particle minus p
      A sl[3] = {A(vg0[i]) * w.sc[0] - mom[0], A(vg1[i]) * w.sc[1] - mom[1],
                 nc > 2 ? A(vg2[i]) * w.sc[2] - mom[2] : A(0)};
      int s = p.species ? p.species[i] : 0;
      if (s >= sp->n) {
        flag(dg, DUST_FLAG_BAD_CELL);
        s = 0;
      }
      A dval = drag_mode == DRAG_SPECIES ? A(1) : A(p.drag[i]);
      A m = p.mass ? A(p.mass[i]) : A(sp->mass[s]);
      // Epstein: tau = C / rho_g with the density gathered at x^{n+1/2}
      A it = drag_mode == DRAG_EPSTEIN ? A(rho_p[i]) / dval
                                       : inverse_tau<A, GEOM>(f, drag_mode, dval, A(sp->inv_tau[s]), w);
      A c, psi;
      propagator<A>(dt * it, c, psi);
      KickOut<A> o;
      kick_any<A, GEOM, NDIM>(B, f, dt, it, c, psi, w, mom, sl, o);
      TW* imp[4] = {imp0, imp1, imp2, imp3};
      bool fin = isfinite(double(o.e));
#pragma unroll
      for (int k = 0; k < nc; ++k) {
        A vbar = (mom[k] + A(0.5) * o.dp[k]) / w.sc[k];
        A dl = cell_width<A, U>(B.ax[k], idx[k]) * (GEOM == GEOM_CART || k == 0 ? A(1) : w.sc[k]);
        double cps = fabs(double(vbar * dt / dl));
        cells = cps > cells ? cps : cells;
        mom[k] += o.dp[k];
        fin &= isfinite(double(mom[k]));
        p.mom[k][i] = TS(mom[k]);
        if (imp[k]) imp[k][i] = TW(m * o.j[k]);
        sums[k] = double(m * o.j[k]);
        sums[4] += fabs(double(m * o.j[k]));
      }
      if (imp[nc]) imp[nc][i] = TW(m * o.e);
      sums[3] = double(m * o.e);
      if (!fin) flag(dg, DUST_FLAG_NONFINITE);
    }
  }
  if (dg) {
#pragma unroll
    for (int k = 0; k < 5; ++k) sums[k] = wave_sum(sums[k]);
    cells = wave_max(cells);
    if (part) {
      // deterministic: the block's sums in a fixed order into its slot of
      // part (added up by k_reduce_kick_partials)
      __shared__ double red[4][5];
      if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 5; ++k) red[threadIdx.x >> 6][k] = sums[k];
      __syncthreads();
      if (threadIdx.x < 5)
        part[(size_t)blockIdx.x * 5 + threadIdx.x] =
            ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
    }
    if ((threadIdx.x & 63) == 0) {
      if (!part) {
        for (int k = 0; k < 3; ++k) unsafeAtomicAdd(&dg->p_part[k], sums[k]);
        unsafeAtomicAdd(&dg->e_part, sums[3]);
        unsafeAtomicAdd(&dg->sum_abs_j, sums[4]);
      }
      atomic_max_nonneg(&dg->max_cells_bits, cells);
      if (cells > 1.8) atomicOr(&dg->flags, (unsigned)DUST_FLAG_CFL);
    }
  }
}

// Sum of the kick's per-block partials (5 per block) in a fixed order, added
// to the diagnostics.
__global__ void __launch_bounds__(256)
    k_reduce_kick_partials(const double* __restrict__ part, int64_t nblocks, DiagDev* dg) {
  __shared__ double red[256][5];
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
    for (int k = 0; k < 5; ++k) acc[k] += part[(size_t)b * 5 + k];
#pragma unroll
  for (int k = 0; k < 5; ++k) red[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int k = 0; k < 5; ++k) red[threadIdx.x][k] += red[threadIdx.x + h][k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) dg->p_part[k] += red[0][k];
    dg->e_part += red[0][3];
    dg->sum_abs_j += red[0][4];
  }
}

template <typename TS, typename A, typename TW, int GEOM, int NDIM, bool U>
__global__ void __launch_bounds__(256) k_deposit(PView<TS> p, const Box* boxes, int nbox,
                                                 FView<TS> fl, const TW* imp0, const TW* imp1,
                                                 const TW* imp2, const TW* imp3, DiagDev* dg) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  int idx[3];
  A off[3], mom[3];
  int b = load_particle<TS, A, GEOM, NDIM>(p, boxes, nbox, i, idx, off, mom, dg);
  if (b < 0) return;
  const Box& B = boxes[b];
  constexpr int nc = GEOM == GEOM_CART ? NDIM : 3;
  A q[4] = {A(imp0[i]), A(imp1[i]), A(imp2[i]), A(0)};
  if (nc > 2) q[3] = A(imp3[i]);
  Stencil<A> s;
  stencil_weights<A, GEOM, NDIM, U>(B, idx, off, s);
  constexpr int c2 = NDIM > 2 ? 1 : 0;
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

// Deposit without float atomics, for the deterministic mode (the step's
// Eq. dust_feedback_final, the predictor's drag source, the dust density):
// one thread per stored cell (active or ghost) of box B sums W q / dV of
// the particles whose stencil covers the cell -- those of the 3^d active
// cells around it, the offsets in a fixed order and each cell's particles
// in the order of a stable sort by cell (perm, bin_start over the global
// cell ids) -- in FP64, for the nch channels q0.. (per particle), and adds
// sgn times the sums to out.dep[0..nch).  Every word has one writer and a
// fixed summation order, so the result is the same bits on every run.
template <typename TS, typename A, typename TW, int GEOM, int NDIM, bool U>
__global__ void __launch_bounds__(256)
    k_deposit_pull(PView<TS> p, Box B, FView<TS> fl, int nch, double sgn, const TW* imp0, const TW* imp1,
                   const TW* imp2, const TW* imp3, const uint32_t* __restrict__ perm,
                   const int64_t* __restrict__ bin_start) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B.nstore) return;
  constexpr int c2 = NDIM > 2 ? 1 : 0;
  const int i = (int)(t % B.g0) - 1;
  const int j = (int)((t / B.g0) % B.g1) - 1;
  const int k = (int)(t / ((int64_t)B.g0 * B.g1)) - B.k_off;
  const int n0 = B.ax[0].n, n1 = B.ax[1].n, n2 = NDIM > 2 ? B.ax[2].n : 1;
  const TW* imp[4] = {imp0, imp1, imp2, imp3};
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // this cell is the particle's host cell shifted by (a, bb, c)
  for (int c = -c2; c <= c2; ++c) {
    const int sk = k - c;
    if (sk < 0 || sk >= n2) continue;
    for (int bb = -1; bb <= 1; ++bb) {
      const int sj = j - bb;
      if (sj < 0 || sj >= n1) continue;
      for (int a = -1; a <= 1; ++a) {
        const int si = i - a;
        if (si < 0 || si >= n0) continue;
        int src[3] = {si, sj, sk};
        const int64_t cid = B.cell_base + ravel(B, src);
        const int64_t e = bin_start[cid + 1];
        for (int64_t s = bin_start[cid]; s < e; ++s) {
          const int64_t ip = perm[s];
          A off[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) off[d] = d < NDIM ? A(p.off[d][ip]) : A(0);
          Stencil<A> sw;
          stencil_weights<A, GEOM, NDIM, U>(B, src, off, sw);
          const double w = double(sw.w[0][a + 1] * sw.w[1][bb + 1] * sw.w[2][c + 1]);
#pragma unroll
          for (int m = 0; m < 4; ++m)
            if (m < nch) acc[m] += w * double(imp[m][ip]);
        }
      }
    }
  }
  const double iv = inv_volume(B, i, j, k);
  const int64_t id = B.store_base + t;
#pragma unroll
  for (int m = 0; m < 4; ++m)
    if (m < nch) fl.dep[m][id] = TS(double(fl.dep[m][id]) + sgn * (acc[m] * iv));
}

// Per-particle coefficients for the deterministic drag source and dust
// density (deposited by k_deposit_pull): q_m = m min(1/tau, 1/dt) times the
// slip sum_i W_i (s_m v_i - p_m), as ds_particles forms them (Epstein: tau
// from the gathered gas density), or the particle mass (MASS); zero for a
// particle without a cell (which no bin holds).
template <typename TS, typename A, int GEOM, int NDIM, bool U, bool MASS>
__global__ void __launch_bounds__(256)
    k_source_coeffs(PView<TS> p, const Box* boxes, int nbox, FView<TS> fl, Forces f, const Species* sp,
                    int drag_mode, A inv_dt, A* q0, A* q1, A* q2, DiagDev* dg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  constexpr int nc = MASS ? 1 : (GEOM == GEOM_CART ? NDIM : 3);
  constexpr int c2 = NDIM > 2 ? 1 : 0;
  A* q[3] = {q0, q1, q2};
  int idx[3];
  A off[3], mom[3] = {A(0), A(0), A(0)};
  const int b = MASS ? load_position<TS, A, NDIM>(p, boxes, nbox, i, idx, off, dg)
                     : load_particle<TS, A, GEOM, NDIM>(p, boxes, nbox, i, idx, off, mom, dg);
  A out[3] = {A(0), A(0), A(0)};
  if (b >= 0) {
    const Box& B = boxes[b];
    int sidx = p.species ? p.species[i] : 0;
    if (sidx >= sp->n) {
      flag(dg, DUST_FLAG_BAD_CELL);
      sidx = 0;
    }
    const A m = p.mass ? A(p.mass[i]) : A(sp->mass[sidx]);
    if constexpr (MASS) {
      out[0] = m;
    } else {
      Stencil<A> s;
      stencil_weights<A, GEOM, NDIM, U>(B, idx, off, s);
      Where<A> w;
      where<A, GEOM, NDIM, U>(B, idx, off, w);
      A sl[3] = {A(0), A(0), A(0)};
      A rg = A(0);
#pragma unroll
      for (int cc = -c2; cc <= c2; ++cc)
#pragma unroll
        for (int bb = -1; bb <= 1; ++bb) {
          const A wbc = s.w[1][bb + 1] * s.w[2][cc + 1];
#pragma unroll
          for (int a = -1; a <= 1; ++a) {
            const A wt = s.w[0][a + 1] * wbc;
            if (drag_mode == DRAG_EPSTEIN)
              rg += wt * A(fl.rho[stored_index(B, idx[0] + a, idx[1] + bb, idx[2] + cc)]);
#pragma unroll
            for (int mm = 0; mm < nc; ++mm)
              sl[mm] += wt * (A(gas_comp(B, fl, nullptr, mm, idx[0] + a, idx[1] + bb, idx[2] + cc)) * w.sc[mm] -
                              mom[mm]);
          }
        }
      const A dval = drag_mode == DRAG_SPECIES ? A(1) : A(p.drag[i]);
      const A it = drag_mode == DRAG_EPSTEIN ? rg / dval
                                             : inverse_tau<A, GEOM>(f, drag_mode, dval, A(sp->inv_tau[sidx]), w);
      const A k = m * (it < inv_dt ? it : inv_dt);
#pragma unroll
      for (int mm = 0; mm < nc; ++mm) out[mm] = k * sl[mm];
    }
  }
#pragma unroll
  for (int mm = 0; mm < nc; ++mm) q[mm][i] = out[mm];
}

// Drag source of the gas predictor (Sec. 3.1, Eq. Delta_vp and f_D): at the
// particle's current position, the canonical slip between the weighted gas
// velocity and the particle, times m / max(tau, dt) (the stiffness limiter
// of Bai & Stone 2010), subtracted from the momentum channels with the
// gather's weights over the cell volume.  inv_dt = 1/dt.
// Each thread takes DS_PPT particles 64 slots apart (a workgroup covers
// 256 * DS_PPT consecutive slots) and sums the contributions of consecutive
// ones with the same host cell in registers (the particles of a cell sit 64
// slots apart in the level-major layout of the fused step), so a cell's
// stencil is deposited once per run instead of once per particle.  Where
// the workgroup's particles share a box and their stencils fit a window of
// ds_win_cells<TS>() cells, the box is workgroup-uniform, the window's gas
// velocity is staged in LDS, the gathers read it there, the deposits go to
// an FP64 LDS window (FP64 LDS atomics run ~20x faster than FP32 ones on
// gfx950) and that window is added to HBM once; otherwise gathers and
// deposits go to HBM.  Correct for any particle order.
static constexpr int DS_PPT = 4;
// window capacity in cells: 3 FP64 deposit channels + 3 gas components in
// storage precision within 64 KiB of LDS
template <typename TS> constexpr int ds_win_cells() { return sizeof(TS) == 4 ? 1600 : 1300; }

struct DsWindow {
  int o[3], ext[3];
  int64_t cells;
};

// Host cell and offsets of particle i (the dust density needs no momenta):
// the box index, or -1 without a cell (flags as load_particle).
template <typename TS, typename A, int NDIM>
__device__ __forceinline__ int load_position(const PView<TS>& p, const Box* boxes, int nbox, int64_t i,
                                             int idx[3], A off[3], DiagDev* dg) {
  const int64_t c = p.cell[i];
  if (c < 0) return -1;
  const int b = find_box(boxes, nbox, c);
  const Box& B = boxes[b];
  if (c >= B.cell_base + B.ncell) {
    flag(dg, DUST_FLAG_BAD_CELL);
    return -1;
  }
  unravel(B, c - B.cell_base, idx);
  bool bad = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    off[d] = d < NDIM ? A(p.off[d][i]) : A(0);
    bad |= !(off[d] >= A(-0.5) && off[d] < A(0.5));
  }
  if (bad) flag(dg, DUST_FLAG_OFFSET_RANGE);
  return b;
}

// The particles of one thread (see k_drag_source).  WIN: every particle
// with a cell lies in box ub (workgroup-uniform) inside window wd.
// MASS: the dust density instead (one channel, the particle mass, no gas).
// EPS: Epstein drag (stopping time from the gathered gas density).
template <typename TS, typename A, int GEOM, int NDIM, bool U, bool WIN, bool MASS, bool EPS>
__device__ __forceinline__ void ds_particles(const PView<TS>& p, const Box* boxes, int nbox, int ub,
                                             const FView<TS>& fl, const Forces& f, const Species* sp,
                                             int drag_mode, A inv_dt, DiagDev* dg, int64_t base,
                                             double* win, const TS* gwin, const DsWindow& wd) {
  constexpr int nc = MASS ? 1 : (GEOM == GEOM_CART ? NDIM : 3);
  constexpr int c2 = NDIM > 2 ? 1 : 0;
  constexpr int NT = NDIM > 2 ? 27 : 9;
  // register sums of the current run of particles with host cell `cur`
  A acc[NT][3];
  int64_t cur = -1;
  int cb = 0, cidx[3] = {0, 0, 0};
  auto flush = [&]() {
    const Box& B = WIN ? boxes[ub] : boxes[cb];
    double iv[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int a = 0; a < 3; ++a) iv[d][a] = d < NDIM ? B.ax[d].ivol[cidx[d] + a] : 1.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int a = t % 3, bb = (t / 3) % 3, cc = NDIM > 2 ? t / 9 : 1;
      const int ii = cidx[0] + a - 1, jj = cidx[1] + bb - 1, kk = cidx[2] + cc - 1;
      const A v = A(iv[0][a] * iv[1][bb] * iv[2][cc]);
      constexpr A sgn = MASS ? A(1) : A(-1);   // the drag source is subtracted
      if constexpr (WIN) {
        const int64_t e = (ii - wd.o[0]) + (int64_t)wd.ext[0] * ((jj - wd.o[1]) + (int64_t)wd.ext[1] * (kk - wd.o[2]));
#pragma unroll
        for (int m = 0; m < nc; ++m) atomicAdd(&win[m * wd.cells + e], double(sgn * acc[t][m] * v));
      } else {
        const int64_t id = stored_index(B, ii, jj, kk);
#pragma unroll
        for (int m = 0; m < nc; ++m) unsafeAtomicAdd(&fl.dep[m][id], TS(sgn * acc[t][m] * v));
      }
    }
  };
  for (int j = 0; j < DS_PPT; ++j) {
    const int64_t i = base + 64 * j;
    if (i >= p.n) break;
    int idx[3];
    A off[3], mom[3];
    int b;
    if constexpr (WIN) {
      // every particle with a valid cell is in box ub (the window test)
      const Box& B = boxes[ub];
      const int64_t c = p.cell[i];
      if (c < 0) continue;
      if (c < B.cell_base || c >= B.cell_base + B.ncell) {
        flag(dg, DUST_FLAG_BAD_CELL);
        continue;
      }
      unravel(B, c - B.cell_base, idx);
      constexpr int nm = MASS ? 0 : nc;
      bool bad = false, nonfinite = false;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        off[d] = d < NDIM ? A(p.off[d][i]) : A(0);
        mom[d] = d < nm ? A(p.mom[d][i]) : A(0);
        bad |= !(off[d] >= A(-0.5) && off[d] < A(0.5));
        nonfinite |= !isfinite(double(mom[d]));
      }
      if (bad) flag(dg, DUST_FLAG_OFFSET_RANGE);
      if (nonfinite) flag(dg, DUST_FLAG_NONFINITE);
      b = ub;
    } else if constexpr (MASS) {
      b = load_position<TS, A, NDIM>(p, boxes, nbox, i, idx, off, dg);
      if (b < 0) continue;
    } else {
      b = load_particle<TS, A, GEOM, NDIM>(p, boxes, nbox, i, idx, off, mom, dg);
      if (b < 0) continue;
    }
    const Box& B = WIN ? boxes[ub] : boxes[b];
    const int64_t c = p.cell[i];
    if (c != cur) {
      if (cur >= 0) flush();
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int m = 0; m < 3; ++m) acc[t][m] = A(0);
      cur = c;
      cb = b;
      cidx[0] = idx[0];
      cidx[1] = idx[1];
      cidx[2] = idx[2];
    }
    Stencil<A> s;
    stencil_weights<A, GEOM, NDIM, U>(B, idx, off, s);
    A q[3] = {A(0), A(0), A(0)};
    if constexpr (MASS) {
      int sidx = p.species ? p.species[i] : 0;
      if (sidx >= sp->n) {
        flag(dg, DUST_FLAG_BAD_CELL);
        sidx = 0;
      }
      q[0] = p.mass ? A(p.mass[i]) : A(sp->mass[sidx]);
    } else {
      Where<A> w;
      where<A, GEOM, NDIM, U>(B, idx, off, w);
      // slip s_c v_g,c - p_c as a weighted sum of per-cell differences (keeps
      // its relative accuracy where the velocities are much larger than it)
      A sl[3] = {A(0), A(0), A(0)};
      A rg = A(0);   // gas density at the particle (Epstein drag)
      int64_t e0 = 0;
      if constexpr (WIN)
        e0 = (idx[0] - wd.o[0]) + (int64_t)wd.ext[0] * ((idx[1] - wd.o[1]) + (int64_t)wd.ext[1] * (idx[2] - wd.o[2]));
#pragma unroll
      for (int cc = -c2; cc <= c2; ++cc)
#pragma unroll
        for (int bb = -1; bb <= 1; ++bb) {
          A wbc = s.w[1][bb + 1] * s.w[2][cc + 1];
#pragma unroll
          for (int a = -1; a <= 1; ++a) {
            A wt = s.w[0][a + 1] * wbc;
            if constexpr (EPS) rg += wt * A(fl.rho[stored_index(B, idx[0] + a, idx[1] + bb, idx[2] + cc)]);
#pragma unroll
            for (int m = 0; m < nc; ++m) {
              A g;
              if constexpr (WIN)
                g = A(gwin[m * wd.cells + e0 + a + (int64_t)wd.ext[0] * (bb + (int64_t)wd.ext[1] * cc)]);
              else
                g = A(gas_comp(B, fl, nullptr, m, idx[0] + a, idx[1] + bb, idx[2] + cc));
              sl[m] += wt * (g * w.sc[m] - mom[m]);
            }
          }
        }
      int sidx = p.species ? p.species[i] : 0;
      if (sidx >= sp->n) {
        flag(dg, DUST_FLAG_BAD_CELL);
        sidx = 0;
      }
      A dval = drag_mode == DRAG_SPECIES ? A(1) : A(p.drag[i]);
      A m = p.mass ? A(p.mass[i]) : A(sp->mass[sidx]);
      A it;
      if constexpr (EPS)
        it = rg / dval;
      else
        it = inverse_tau<A, GEOM>(f, drag_mode, dval, A(sp->inv_tau[sidx]), w);
      A k = m * (it < inv_dt ? it : inv_dt);
#pragma unroll
      for (int mm = 0; mm < nc; ++mm) q[mm] = k * sl[mm];
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      A wt = s.w[0][t % 3] * s.w[1][(t / 3) % 3] * s.w[2][NDIM > 2 ? t / 9 : 1];
#pragma unroll
      for (int mm = 0; mm < nc; ++mm) acc[t][mm] += wt * q[mm];
    }
  }
  if (cur >= 0) flush();
}

// Window over the host cells [lo, hi] (plus one cell on each side) if it
// holds at most cap cells.
template <int NDIM>
__device__ __forceinline__ bool ds_window(const int lo[3], const int hi[3], int64_t cap, DsWindow& wd) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    wd.o[d] = d < NDIM ? lo[d] - 1 : 0;
    wd.ext[d] = d < NDIM ? hi[d] - lo[d] + 3 : 1;
  }
  wd.cells = (int64_t)wd.ext[0] * wd.ext[1] * wd.ext[2];
  return wd.cells <= cap;
}

template <typename TS, int NC, bool GAS>
__device__ __forceinline__ void ds_stage(const Box& B, const FView<TS>& fl, const DsWindow& wd, double* win,
                                         TS* gwin, int lane, int nlanes) {
  for (int64_t e = lane; e < wd.cells; e += nlanes) {
    int ii = wd.o[0] + (int)(e % wd.ext[0]);
    int jj = wd.o[1] + (int)((e / wd.ext[0]) % wd.ext[1]);
    int kk = wd.o[2] + (int)(e / ((int64_t)wd.ext[0] * wd.ext[1]));
    int64_t id = stored_index(B, ii, jj, kk);
#pragma unroll
    for (int m = 0; m < NC; ++m) {
      win[m * wd.cells + e] = 0.0;
      if constexpr (GAS) gwin[m * wd.cells + e] = fl.vel[m][id];
    }
  }
}

template <typename TS, int NC>
__device__ __forceinline__ void ds_add_window(const Box& B, const FView<TS>& fl, const DsWindow& wd,
                                              const double* win, int lane, int nlanes) {
  for (int64_t e = lane; e < wd.cells; e += nlanes) {
    int ii = wd.o[0] + (int)(e % wd.ext[0]);
    int jj = wd.o[1] + (int)((e / wd.ext[0]) % wd.ext[1]);
    int kk = wd.o[2] + (int)(e / ((int64_t)wd.ext[0] * wd.ext[1]));
    int64_t id = stored_index(B, ii, jj, kk);
#pragma unroll
    for (int m = 0; m < NC; ++m) {
      double v = win[m * wd.cells + e];
      if (v != 0.0) unsafeAtomicAdd(&fl.dep[m][id], TS(v));
    }
  }
}

// Windows: one for the workgroup when its particles' window fits the LDS
// capacity, else one per wave (a quarter of the capacity each) for the waves
// whose particles' window fits that; the other waves go to HBM.
template <typename TS, typename A, int GEOM, int NDIM, bool U, bool MASS, bool EPS>
__device__ __forceinline__ void ds_body(const PView<TS>& p, const Box* boxes, int nbox, const FView<TS>& fl,
                                        const Forces& f, const Species* sp, int drag_mode, A inv_dt,
                                        DiagDev* dg) {
  constexpr int nc = MASS ? 1 : (GEOM == GEOM_CART ? NDIM : 3);
  constexpr int CAP = ds_win_cells<TS>();
  __shared__ double win[3 * CAP];
  __shared__ TS gwin[3 * CAP];
  __shared__ int s_lo[4][3], s_hi[4][3], s_blo[4], s_bhi[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    for (int d = 0; d < 3; ++d) {
      s_lo[wave][d] = 0x7fffffff;
      s_hi[wave][d] = -0x7fffffff;
    }
    s_blo[wave] = 0x7fffffff;
    s_bhi[wave] = -1;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * (256 * DS_PPT) + (int64_t)wave * (64 * DS_PPT) + lane;
  // bounding box of each wave's host cells
  {
    int lo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, hi[3] = {-0x7fffffff, -0x7fffffff, -0x7fffffff};
    int blo = 0x7fffffff, bhi = -1;
    auto add = [&](const Box& B, int b, int64_t c) {
      if (c >= B.cell_base + B.ncell) return;
      int idx[3];
      unravel(B, c - B.cell_base, idx);
#pragma unroll
      for (int d = 0; d < NDIM; ++d) {
        lo[d] = idx[d] < lo[d] ? idx[d] : lo[d];
        hi[d] = idx[d] > hi[d] ? idx[d] : hi[d];
      }
      blo = b < blo ? b : blo;
      bhi = b > bhi ? b : bhi;
    };
    for (int j = 0; j < DS_PPT; ++j) {
      int64_t i = base + 64 * j;
      if (i >= p.n) break;
      int64_t c = p.cell[i];
      if (c < 0) continue;
      // one box: a uniform descriptor (scalar loads)
      if (nbox == 1)
        add(boxes[0], 0, c);
      else {
        const int b = find_box(boxes, nbox, c);
        add(boxes[b], b, c);
      }
    }
    if (bhi >= 0) {
#pragma unroll
      for (int d = 0; d < NDIM; ++d) {
        atomicMin(&s_lo[wave][d], lo[d]);
        atomicMax(&s_hi[wave][d], hi[d]);
      }
      atomicMin(&s_blo[wave], blo);
      atomicMax(&s_bhi[wave], bhi);
    }
  }
  __syncthreads();
  // workgroup window (uniform decision)
  int glo[3], ghi[3], gblo = 0x7fffffff, gbhi = -1;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    glo[d] = 0x7fffffff;
    ghi[d] = -0x7fffffff;
  }
  for (int w = 0; w < 4; ++w) {
    if (s_bhi[w] < 0) continue;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      glo[d] = s_lo[w][d] < glo[d] ? s_lo[w][d] : glo[d];
      ghi[d] = s_hi[w][d] > ghi[d] ? s_hi[w][d] : ghi[d];
    }
    gblo = s_blo[w] < gblo ? s_blo[w] : gblo;
    gbhi = s_bhi[w] > gbhi ? s_bhi[w] : gbhi;
  }
  DsWindow wd;
  const bool wg_win = gbhi >= 0 && gblo == gbhi && ds_window<NDIM>(glo, ghi, CAP * 3 / nc, wd);
  if (wg_win) {
    const int ub = __builtin_amdgcn_readfirstlane(gblo);
    const Box& B = boxes[ub];
    ds_stage<TS, nc, !MASS>(B, fl, wd, win, gwin, threadIdx.x, blockDim.x);
    __syncthreads();
    ds_particles<TS, A, GEOM, NDIM, U, true, MASS, EPS>(p, boxes, nbox, ub, fl, f, sp, drag_mode, inv_dt, dg, base,
                                             win, gwin, wd);
    __syncthreads();
    ds_add_window<TS, nc>(B, fl, wd, win, threadIdx.x, blockDim.x);
    return;   // uniform: the whole workgroup leaves here
  }
  // per-wave windows (each wave decides for itself; barriers stay uniform)
  int wlo[3], whi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    wlo[d] = s_lo[wave][d];
    whi[d] = s_hi[wave][d];
  }
  const int qcap = CAP / 4;
  double* wwin = win + wave * 3 * qcap;
  TS* wgwin = gwin + wave * 3 * qcap;
  const bool w_win = s_bhi[wave] >= 0 && s_blo[wave] == s_bhi[wave] &&
                     ds_window<NDIM>(wlo, whi, qcap * 3 / nc, wd);
  const int ub = __builtin_amdgcn_readfirstlane(s_blo[wave]);
  if (w_win) ds_stage<TS, nc, !MASS>(boxes[ub], fl, wd, wwin, wgwin, lane, 64);
  __syncthreads();
  if (w_win)
    ds_particles<TS, A, GEOM, NDIM, U, true, MASS, EPS>(p, boxes, nbox, ub, fl, f, sp, drag_mode, inv_dt, dg, base,
                                             wwin, wgwin, wd);
  else
    ds_particles<TS, A, GEOM, NDIM, U, false, MASS, EPS>(p, boxes, nbox, 0, fl, f, sp, drag_mode, inv_dt, dg, base,
                                              wwin, wgwin, wd);
  __syncthreads();
  if (w_win) ds_add_window<TS, nc>(boxes[ub], fl, wd, wwin, lane, 64);
}

template <typename TS, typename A, int GEOM, int NDIM, bool U, bool EPS>
__global__ void __launch_bounds__(256) k_drag_source(PView<TS> p, const Box* boxes, int nbox,
                                                     FView<TS> fl, Forces f, const Species* sp,
                                                     int drag_mode, A inv_dt, DiagDev* dg) {
  ds_body<TS, A, GEOM, NDIM, U, false, EPS>(p, boxes, nbox, fl, f, sp, drag_mode, inv_dt, dg);
}

// Dust density: rho_d (fl.dep[0]) += m W / dV with the gather's weights.
template <typename TS, typename A, int GEOM, int NDIM, bool U>
__global__ void __launch_bounds__(256) k_mass_density(PView<TS> p, const Box* boxes, int nbox,
                                                      FView<TS> fl, const Species* sp, DiagDev* dg) {
  ds_body<TS, A, GEOM, NDIM, U, true, false>(p, boxes, nbox, fl, Forces{}, sp, DRAG_TAU, A(0), dg);
}

// Dispatch on the (geometry, dimension) shared by the context's boxes.
#define DUST_GEOM_SWITCH(geom, ndim, unif, CALL)                      \
  do {                                                                \
    if ((geom) == GEOM_CART && (ndim) == 2 && (unif)) {               \
      constexpr int G_ = GEOM_CART, D_ = 2;                           \
      constexpr bool U_ = true;                                       \
      CALL;                                                           \
    } else if ((geom) == GEOM_CART && (ndim) == 2) {                  \
      constexpr int G_ = GEOM_CART, D_ = 2;                           \
      constexpr bool U_ = false;                                      \
      CALL;                                                           \
    } else if ((geom) == GEOM_CART && (unif)) {                       \
      constexpr int G_ = GEOM_CART, D_ = 3;                           \
      constexpr bool U_ = true;                                       \
      CALL;                                                           \
    } else if ((geom) == GEOM_CART) {                                 \
      constexpr int G_ = GEOM_CART, D_ = 3;                           \
      constexpr bool U_ = false;                                      \
      CALL;                                                           \
    } else if ((geom) == GEOM_CYL) {                                  \
      constexpr int G_ = GEOM_CYL, D_ = 3;                            \
      constexpr bool U_ = false;                                      \
      CALL;                                                           \
    } else {                                                          \
      constexpr int G_ = GEOM_SPH, D_ = 3;                            \
      constexpr bool U_ = false;                                      \
      CALL;                                                           \
    }                                                                 \
  } while (0)

// ---------------------------------------------------------------- grid kernels
// Each ghost kernel treats several arrays of one box in one launch: the
// array is blockIdx.y.

template <typename TS> struct Arr4 {
  TS* a[4];
};

// One launch of a per-box kernel over several boxes: box[e] takes blocks
// [blk0[e], blk0[e+1]) of the grid (up to MB_BOXES boxes per launch); a
// block finds its entry by a scan of blk0 and reads its box descriptor from
// the device table (a block-uniform address).
static constexpr int MB_BOXES = 16;
static_assert(GRID_SUM_PARTS >= GRID_SUM_BLOCKS + MB_BOXES, "grid-sum partials");
struct BoxGrid {
  int n;
  int box[MB_BOXES];
  uint32_t blk0[MB_BOXES + 1];
};
__device__ __forceinline__ int grid_entry(const BoxGrid& g) {
  int e = 0;
  while (e + 1 < g.n && blockIdx.x >= g.blk0[e + 1]) ++e;
  return e;
}
// thread index within the box's range
__device__ __forceinline__ int64_t grid_thread(const BoxGrid& g, int e) {
  return (int64_t)(blockIdx.x - g.blk0[e]) * blockDim.x + threadIdx.x;
}

// x ghosts of one box: shear-periodic (interpolated in y) or periodic.
template <typename TS>
__global__ void k_fill_x(const Box* boxes, BoxGrid bg, Arr4<TS> arrs, int boost, double qOmega,
                         const double* tdev, double toff) {
  const int e = grid_entry(bg);
  const Box& B = boxes[bg.box[e]];
  const int shear = B.ax[0].bc_lo == BC_SHEAR;
  const int vy_slot = B.geom == GEOM_CART && boost ? 2 : -1;
  TS* a = arrs.a[blockIdx.y];
  const int comp_vy = (int)blockIdx.y == vy_slot;
  int n0 = B.ax[0].n, n1 = B.ax[1].n, n2 = B.ndim > 2 ? B.ax[2].n : 1;
  int64_t t = grid_thread(bg, e);
  if (t >= (int64_t)n1 * n2) return;
  const Shift sh = make_shift(B, qOmega, *tdev + toff);
  int j = (int)(t % n1), k = (int)(t / n1);
  if (shear) {
    // right ghost (x_0 + L, y_j) = (x_0, y_j + s); left ghost = (x_{n-1}, y_j - s)
    int jl = j + sh.si;
    double fr = sh.sf;
    int j0 = ((jl % n1) + n1) % n1, j1 = ((jl + 1) % n1 + n1) % n1;
    double v = (1.0 - fr) * double(a[stored_index(B, 0, j0, k)]) +
               fr * double(a[stored_index(B, 0, j1, k)]);
    a[stored_index(B, n0, j, k)] = TS(v - (comp_vy ? sh.u : 0.0));
    double pos_fl = -sh.si - (sh.sf > 0 ? 1 : 0);
    int jm = j + (int)pos_fl;
    double frm = sh.sf > 0 ? 1.0 - sh.sf : 0.0;
    j0 = ((jm % n1) + n1) % n1;
    j1 = ((jm + 1) % n1 + n1) % n1;
    v = (1.0 - frm) * double(a[stored_index(B, n0 - 1, j0, k)]) +
        frm * double(a[stored_index(B, n0 - 1, j1, k)]);
    a[stored_index(B, -1, j, k)] = TS(v + (comp_vy ? sh.u : 0.0));
  } else {
    a[stored_index(B, -1, j, k)] = a[stored_index(B, n0 - 1, j, k)];
    a[stored_index(B, n0, j, k)] = a[stored_index(B, 0, j, k)];
  }
}

// FP64 copy of the shear-periodic x-ghost gas of velocity component m, with
// the y and z ghost rows of the layer (periodic images): the interpolated and
// boosted ghost values keep their FP64 rounding, so that a particle next to
// the shear boundary sees the gas at the accuracy of the interior values.
template <typename TS>
__global__ void k_fill_xghost(const Box* boxes, BoxGrid bg, Arr4<TS> vel, double* xg, double qOmega,
                              const double* tdev, double toff, int boost) {
  const int ge = grid_entry(bg);
  const Box& B = boxes[bg.box[ge]];
  const int m = blockIdx.y, comp_vy = boost && m == 1;
  const TS* a = vel.a[m];
  const int n0 = B.ax[0].n, n1 = B.ax[1].n, n2 = B.ax[2].n;
  const int g1 = n1 + 2, g2 = n2 + 2;
  const int64_t t = grid_thread(bg, ge);
  if (t >= (int64_t)g1 * g2) return;
  const Shift sh = make_shift(B, qOmega, *tdev + toff);
  const int jg = (int)(t % g1), kg = (int)(t / g1);
  const int j = ((jg - 1) % n1 + n1) % n1, k = ((kg - 1) % n2 + n2) % n2;
  int jl = j + sh.si;
  int j0 = ((jl % n1) + n1) % n1, j1 = ((jl + 1) % n1 + n1) % n1;
  double right = (1.0 - sh.sf) * double(a[stored_index(B, 0, j0, k)]) +
                 sh.sf * double(a[stored_index(B, 0, j1, k)]) - (comp_vy ? sh.u : 0.0);
  int jm = j - sh.si - (sh.sf > 0 ? 1 : 0);
  double frm = sh.sf > 0 ? 1.0 - sh.sf : 0.0;
  j0 = ((jm % n1) + n1) % n1;
  j1 = ((jm + 1) % n1 + n1) % n1;
  double left = (1.0 - frm) * double(a[stored_index(B, n0 - 1, j0, k)]) +
                frm * double(a[stored_index(B, n0 - 1, j1, k)]) + (comp_vy ? sh.u : 0.0);
  const int64_t layer = (int64_t)g1 * g2;
  xg[B.xg_base + (0 * 3 + m) * layer + t] = left;
  xg[B.xg_base + (1 * 3 + m) * layer + t] = right;
}

template <typename TS> __global__ void k_fill_y(const Box* boxes, BoxGrid bg, Arr4<TS> arrs) {
  const int e = grid_entry(bg);
  const Box& B = boxes[bg.box[e]];
  TS* a = arrs.a[blockIdx.y];
  int n0 = B.ax[0].n, n1 = B.ax[1].n, n2 = B.ndim > 2 ? B.ax[2].n : 1;
  int64_t t = grid_thread(bg, e);
  if (t >= (int64_t)(n0 + 2) * n2) return;
  int i = (int)(t % (n0 + 2)) - 1, k = (int)(t / (n0 + 2));
  a[stored_index(B, i, -1, k)] = a[stored_index(B, i, n1 - 1, k)];
  a[stored_index(B, i, n1, k)] = a[stored_index(B, i, 0, k)];
}

template <typename TS> __global__ void k_fill_z(const Box* boxes, BoxGrid bg, Arr4<TS> arrs) {
  const int e = grid_entry(bg);
  const Box& B = boxes[bg.box[e]];
  TS* a = arrs.a[blockIdx.y];
  int n0 = B.ax[0].n, n1 = B.ax[1].n, n2 = B.ax[2].n;
  int64_t t = grid_thread(bg, e);
  if (t >= (int64_t)(n0 + 2) * (n1 + 2)) return;
  int i = (int)(t % (n0 + 2)) - 1, j = (int)(t / (n0 + 2)) - 1;
  a[stored_index(B, i, j, -1)] = a[stored_index(B, i, j, n2 - 1)];
  a[stored_index(B, i, j, n2)] = a[stored_index(B, i, j, 0)];
}

template <typename TS> __global__ void k_fold_z(const Box* boxes, BoxGrid bg, Arr4<TS> arrs) {
  const int e = grid_entry(bg);
  const Box& B = boxes[bg.box[e]];
  TS* a = arrs.a[blockIdx.y];
  int n0 = B.ax[0].n, n1 = B.ax[1].n, n2 = B.ax[2].n;
  int64_t t = grid_thread(bg, e);
  if (t >= (int64_t)(n0 + 2) * (n1 + 2)) return;
  int i = (int)(t % (n0 + 2)) - 1, j = (int)(t / (n0 + 2)) - 1;
  int64_t gl = stored_index(B, i, j, -1), gh = stored_index(B, i, j, n2);
  a[stored_index(B, i, j, n2 - 1)] += a[gl];
  a[stored_index(B, i, j, 0)] += a[gh];
  a[gl] = TS(0);
  a[gh] = TS(0);
}

template <typename TS> __global__ void k_fold_y(const Box* boxes, BoxGrid bg, Arr4<TS> arrs) {
  const int e = grid_entry(bg);
  const Box& B = boxes[bg.box[e]];
  TS* a = arrs.a[blockIdx.y];
  int n0 = B.ax[0].n, n1 = B.ax[1].n, n2 = B.ndim > 2 ? B.ax[2].n : 1;
  int64_t t = grid_thread(bg, e);
  if (t >= (int64_t)(n0 + 2) * n2) return;
  int i = (int)(t % (n0 + 2)) - 1, k = (int)(t / (n0 + 2));
  int64_t gl = stored_index(B, i, -1, k), gh = stored_index(B, i, n1, k);
  a[stored_index(B, i, n1 - 1, k)] += a[gl];
  a[stored_index(B, i, 0, k)] += a[gh];
  a[gl] = TS(0);
  a[gh] = TS(0);
}

// x fold, written as a gather over the ghost rows that feed each partner
// cell (no atomics).  The energy channel (e != NULL) gains +/- u D_y.
template <typename TS>
__global__ void k_fold_x(const Box* boxes, BoxGrid bg, Arr4<TS> arrs, const TS* dy, int boost_energy,
                         double qOmega, const double* tdev, double toff) {
  const int ge = grid_entry(bg);
  const Box& B = boxes[bg.box[ge]];
  const int shear = B.ax[0].bc_lo == BC_SHEAR;
  const int nch = B.geom == GEOM_CART ? B.ndim : 3;
  const int energy_slot = shear && boost_energy ? nch : -1;
  TS* a = arrs.a[blockIdx.y];
  const int is_energy = (int)blockIdx.y == energy_slot;
  int n0 = B.ax[0].n, n1 = B.ax[1].n, n2 = B.ndim > 2 ? B.ax[2].n : 1;
  int64_t t = grid_thread(bg, ge);
  if (t >= (int64_t)n1 * n2) return;
  const Shift sh = make_shift(B, qOmega, *tdev + toff);
  int jt = (int)(t % n1), k = (int)(t / n1);
  auto wrapj = [n1](int j) { return ((j % n1) + n1) % n1; };
  if (!shear) {
    a[stored_index(B, n0 - 1, jt, k)] += a[stored_index(B, -1, jt, k)];
    a[stored_index(B, 0, jt, k)] += a[stored_index(B, n0, jt, k)];
    return;
  }
  auto gr = [&](int j) {  // right ghost value, energy frame-shifted
    double v = double(a[stored_index(B, n0, j, k)]);
    if (is_energy) v += sh.u * double(dy[stored_index(B, n0, j, k)]);
    return v;
  };
  auto gl = [&](int j) {
    double v = double(a[stored_index(B, -1, j, k)]);
    if (is_energy) v -= sh.u * double(dy[stored_index(B, -1, j, k)]);
    return v;
  };
  // right ghost row j lands on floor(j + s) (1 - sf) and floor(j + s) + 1 (sf)
  double add0 = (1.0 - sh.sf) * gr(wrapj(jt - sh.si));
  if (sh.sf > 0) add0 += sh.sf * gr(wrapj(jt - sh.si - 1));
  // left ghost row j lands on floor(j - s) and floor(j - s) + 1
  double addn;
  if (sh.sf > 0) {
    int c = sh.si + 1;  // ceil(s)
    addn = sh.sf * gl(wrapj(jt + c)) + (1.0 - sh.sf) * gl(wrapj(jt + c - 1));
  } else {
    addn = gl(wrapj(jt + sh.si));
  }
  a[stored_index(B, 0, jt, k)] += TS(add0);
  a[stored_index(B, n0 - 1, jt, k)] += TS(addn);
}

template <typename TS> __global__ void k_clear_x_ghosts(const Box* boxes, BoxGrid bg, Arr4<TS> arrs) {
  const int e = grid_entry(bg);
  const Box& B = boxes[bg.box[e]];
  TS* a = arrs.a[blockIdx.y];
  int n0 = B.ax[0].n, n1 = B.ax[1].n, n2 = B.ndim > 2 ? B.ax[2].n : 1;
  int64_t t = grid_thread(bg, e);
  if (t >= (int64_t)n1 * n2) return;
  int j = (int)(t % n1), k = (int)(t / n1);
  a[stored_index(B, -1, j, k)] = TS(0);
  a[stored_index(B, n0, j, k)] = TS(0);
}

// Step start time (set, or advanced by dt), and the diagnostics' step count
// when dg is given (one launch per step).
__global__ void k_set_time(double* t, double v, double add, DiagDev* dg) {
  t[0] = add != 0.0 ? t[0] + add : v;
  if (dg) dg->steps += 1;
}

void launch_set_time(double* tdev, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_time, dim3(1), dim3(1), 0, st, tdev, v, 0.0, (DiagDev*)nullptr);
}
void launch_advance_time(double* tdev, double dt, DiagDev* count, hipStream_t st) {
  hipLaunchKernelGGL(k_set_time, dim3(1), dim3(1), 0, st, tdev, 0.0, dt, count);
}

template <typename TS> __global__ void k_fill_values(Arr4<TS> arrs, int64_t n, TS v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) arrs.a[blockIdx.y][i] = v;
}

template <typename TS> __global__ void k_fill_value(TS* a, int64_t n, TS v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// v_c += D_c / (rho s_c) on the active cells of the boxes.
template <typename TS> __global__ void k_feedback(const Box* boxes, BoxGrid bg, FView<TS> fl) {
  const int e = grid_entry(bg);
  const Box& B = boxes[bg.box[e]];
  int n0 = B.ax[0].n, n1 = B.ax[1].n, n2 = B.ndim > 2 ? B.ax[2].n : 1;
  int64_t t = grid_thread(bg, e);
  if (t >= (int64_t)n0 * n1 * n2) return;
  int idx[3];
  unravel(B, t, idx);   // (active cell counts are below 2^31)
  const int i = idx[0], j = idx[1], k = idx[2];
  int64_t id = stored_index(B, i, j, k);
  const int nc = B.geom == GEOM_CART ? B.ndim : 3;
  double sc[3] = {1.0, 1.0, 1.0};
  if (B.geom != GEOM_CART) {
    double x0 = cell_centre<double, false>(B.ax[0], i);
    sc[1] = x0;
    if (B.geom == GEOM_SPH) sc[2] = x0 * sin(cell_centre<double, false>(B.ax[1], j));
  }
  const double irho = 1.0 / double(fl.rho[id]);   // one division per cell
  for (int c = 0; c < nc; ++c) {
    const double q = double(fl.dep[c][id]) * irho;
    fl.vel[c][id] = TS(double(fl.vel[c][id]) + (c == 0 ? q : q / sc[c]));
  }
}

// FP64 sums of dV D over every stored cell of the boxes: a grid-stride loop
// over each box's blocks, a block reduction into the block's slot of
// `part`, then one workgroup adds the slots in a fixed order (no contended
// atomics, deterministic).
template <typename TS>
__global__ void __launch_bounds__(256) k_grid_sums(const Box* boxes, BoxGrid bg, FView<TS> fl,
                                                   double* __restrict__ part) {
  __shared__ double red[4][4];
  const int ge = grid_entry(bg);
  const Box& B = boxes[bg.box[ge]];
  const int nc = B.geom == GEOM_CART ? B.ndim : 3;
  const double inv_g0 = 1.0 / B.g0, inv_g1 = 1.0 / B.g1;
  double s[4] = {0, 0, 0, 0};
  const int64_t stride = (int64_t)(bg.blk0[ge + 1] - bg.blk0[ge]) * blockDim.x;
  for (int64_t t = grid_thread(bg, ge); t < B.nstore; t += stride) {
    int i, j, k;
    if (B.nstore < 0x7fffffffLL) {
      int r = div_small((int)t, B.g0, inv_g0);
      i = (int)t - r * B.g0;
      int q = div_small(r, B.g1, inv_g1);
      j = r - q * B.g1;
      k = q;
    } else {
      i = (int)(t % B.g0);
      j = (int)((t / B.g0) % B.g1);
      k = (int)(t / ((int64_t)B.g0 * B.g1));
    }
    double dv = 1.0 / inv_volume(B, i - 1, j - 1, k - B.k_off);
    int64_t id = B.store_base + t;
    for (int c = 0; c <= nc; ++c) s[c] += dv * double(fl.dep[c][id]);
  }
  for (int c = 0; c < 4; ++c) s[c] = wave_sum(s[c]);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int c = 0; c < 4; ++c) red[wave][c] = s[c];
  __syncthreads();
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    part[(size_t)blockIdx.x * 4 + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
  }
}

__global__ void __launch_bounds__(256)
    k_reduce_grid_partials(const double* __restrict__ part, int n, int nc, DiagDev* dg) {
  __shared__ double red[256][4];
  double acc[4] = {0, 0, 0, 0};
#pragma unroll 4
  for (int b = threadIdx.x; b < n; b += 256)
    for (int c = 0; c < 4; ++c) acc[c] += part[(size_t)b * 4 + c];
  for (int c = 0; c < 4; ++c) red[threadIdx.x][c] = acc[c];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int c = 0; c < 4; ++c) red[threadIdx.x][c] += red[threadIdx.x + h][c];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int c = 0; c < nc; ++c) dg->p_grid[c] += red[0][c];
    dg->e_grid += red[0][nc];
  }
}

// ---------------------------------------------------------------- launchers

static inline unsigned blocks_for(int64_t n, int bs = 256) {
  return (unsigned)((n + bs - 1) / bs);
}

template <typename TS, typename A>
void launch_drift(const PView<TS>& p, const Box* boxes, int nbox, int geom, int ndim, int unif,
                  const Forces& f, double h, const double* tdev, double toff, int first,
                  DiagDev* dg, hipStream_t st) {
  if (p.n == 0) return;
  DUST_GEOM_SWITCH(geom, ndim, unif,
                   hipLaunchKernelGGL((k_drift<TS, A, G_, D_, U_>), dim3(blocks_for(p.n)), dim3(256), 0,
                                      st, p, boxes, nbox, f, A(h), tdev, toff, first, dg));
}

template <typename TS, typename A, typename TW>
void launch_gather(const PView<TS>& p, const Box* boxes, int nbox, int geom, int ndim, int unif,
                   const FView<TS>& fl, const double* xg, TW* rho_p, TW* const vg[3], DiagDev* dg,
                   hipStream_t st) {
  if (p.n == 0) return;
  DUST_GEOM_SWITCH(geom, ndim, unif,
                   hipLaunchKernelGGL((k_gather<TS, A, TW, G_, D_, U_>), dim3(blocks_for(p.n)), dim3(256),
                                      0, st, p, boxes, nbox, fl, xg, rho_p, vg[0], vg[1], vg[2], dg));
}

template <typename TS, typename A, typename TW>
void launch_kick(const PView<TS>& p, const Box* boxes, int nbox, int geom, int ndim, int unif,
                 const Forces& f, const Species* sp, int drag_mode, double dt, const TW* rho_p,
                 const TW* const vg[3], TW* const imp[4], DiagDev* dg, double* part, hipStream_t st) {
  if (p.n == 0) return;
  if (!dg) part = nullptr;
  DUST_GEOM_SWITCH(geom, ndim, unif,
                   hipLaunchKernelGGL((k_kick<TS, A, TW, G_, D_, U_>), dim3(blocks_for(p.n)), dim3(256),
                                      0, st, p, boxes, nbox, f, sp, drag_mode, A(dt), rho_p, vg[0], vg[1],
                                      vg[2], imp[0], imp[1], imp[2], imp[3], dg, part));
  if (part)
    hipLaunchKernelGGL(k_reduce_kick_partials, dim3(1), dim3(256), 0, st, (const double*)part,
                       (int64_t)blocks_for(p.n), dg);
}

int64_t kick_partial_words(int64_t n) { return 5 * (int64_t)blocks_for(std::max<int64_t>(n, 1)); }

template <typename TS, typename A, typename TW>
void launch_deposit(const PView<TS>& p, const Box* boxes, int nbox, int geom, int ndim, int unif,
                    const FView<TS>& fl, const TW* const imp[4], DiagDev* dg, hipStream_t st) {
  if (p.n == 0) return;
  DUST_GEOM_SWITCH(geom, ndim, unif,
                   hipLaunchKernelGGL((k_deposit<TS, A, TW, G_, D_, U_>), dim3(blocks_for(p.n)), dim3(256),
                                      0, st, p, boxes, nbox, fl, imp[0], imp[1], imp[2], imp[3], dg));
}

template <typename TS, typename A, typename TW>
void launch_deposit_pull(const PView<TS>& p, const Box& B, int geom, int ndim, int unif, const FView<TS>& fl,
                         int nch, double sgn, const TW* const imp[4], const uint32_t* perm,
                         const int64_t* bin_start, hipStream_t st) {
  if (B.nstore == 0) return;
  DUST_GEOM_SWITCH(geom, ndim, unif,
                   hipLaunchKernelGGL((k_deposit_pull<TS, A, TW, G_, D_, U_>), dim3(blocks_for(B.nstore)),
                                      dim3(256), 0, st, p, B, fl, nch, sgn, imp[0], imp[1], imp[2], imp[3],
                                      perm, bin_start));
}

template <typename TS, typename A>
void launch_source_coeffs(const PView<TS>& p, const Box* boxes, int nbox, int geom, int ndim, int unif,
                          const FView<TS>& fl, const Forces& f, const Species* sp, int drag_mode, double dt,
                          bool mass, A* const q[3], DiagDev* dg, hipStream_t st) {
  if (p.n == 0) return;
  if (mass)
    DUST_GEOM_SWITCH(geom, ndim, unif,
                     hipLaunchKernelGGL((k_source_coeffs<TS, A, G_, D_, U_, true>), dim3(blocks_for(p.n)),
                                        dim3(256), 0, st, p, boxes, nbox, fl, f, sp, drag_mode, A(1.0 / dt),
                                        q[0], q[1], q[2], dg));
  else
    DUST_GEOM_SWITCH(geom, ndim, unif,
                     hipLaunchKernelGGL((k_source_coeffs<TS, A, G_, D_, U_, false>), dim3(blocks_for(p.n)),
                                        dim3(256), 0, st, p, boxes, nbox, fl, f, sp, drag_mode, A(1.0 / dt),
                                        q[0], q[1], q[2], dg));
}

template <typename TS, typename A>
void launch_drag_source(const PView<TS>& p, const Box* boxes, int nbox, int geom, int ndim, int unif,
                        const FView<TS>& fl, const Forces& f, const Species* sp, int drag_mode,
                        double dt, DiagDev* dg, hipStream_t st) {
  if (p.n == 0) return;
  if (drag_mode == DRAG_EPSTEIN)
    DUST_GEOM_SWITCH(geom, ndim, unif,
                     hipLaunchKernelGGL((k_drag_source<TS, A, G_, D_, U_, true>),
                                        dim3(blocks_for(p.n, 256 * DS_PPT)), dim3(256), 0, st, p, boxes,
                                        nbox, fl, f, sp, drag_mode, A(1.0 / dt), dg));
  else
    DUST_GEOM_SWITCH(geom, ndim, unif,
                     hipLaunchKernelGGL((k_drag_source<TS, A, G_, D_, U_, false>),
                                        dim3(blocks_for(p.n, 256 * DS_PPT)), dim3(256), 0, st, p, boxes,
                                        nbox, fl, f, sp, drag_mode, A(1.0 / dt), dg));
}

template <typename TS, typename A>
void launch_mass_density(const PView<TS>& p, const Box* boxes, int nbox, int geom, int ndim, int unif,
                         TS* rho_d, const Species* sp, DiagDev* dg, hipStream_t st) {
  if (p.n == 0) return;
  FView<TS> fl{};
  fl.dep[0] = rho_d;
  DUST_GEOM_SWITCH(geom, ndim, unif,
                   hipLaunchKernelGGL((k_mass_density<TS, A, G_, D_, U_>), dim3(blocks_for(p.n, 256 * DS_PPT)),
                                      dim3(256), 0, st, p, boxes, nbox, fl, sp, dg));
}

// Launches `launch(grid, blocks)` over the boxes b with want(b), each with
// blocks(b) blocks, MB_BOXES boxes per launch.
template <typename Want, typename Blocks, typename Launch>
static void for_box_grids(const Box* hb, int nbox, Want want, Blocks blocks, Launch launch) {
  BoxGrid g{};
  uint32_t nb = 0;
  auto flush = [&]() {
    if (g.n) {
      g.blk0[g.n] = nb;
      launch(g, nb);
    }
    g = BoxGrid{};
    nb = 0;
  };
  for (int b = 0; b < nbox; ++b) {
    if (!want(hb[b])) continue;
    const uint32_t k = blocks(hb[b]);
    if (k == 0) continue;
    g.box[g.n] = b;
    g.blk0[g.n] = nb;
    nb += k;
    if (++g.n == MB_BOXES) flush();
  }
  flush();
}

static inline int box_nc(const Box& B) { return B.geom == GEOM_CART ? B.ndim : 3; }
static inline int64_t box_n(const Box& B, int d) { return d < B.ndim ? B.ax[d].n : 1; }

template <typename TS>
void launch_fill(const Box* hb, int nbox, const Box* boxes_d, const Forces& f, const double* tdev, double toff,
                 const FView<TS>& fl, double* xg, hipStream_t st) {
  if (nbox <= 0) return;
  const int nc = box_nc(hb[0]);
  const Arr4<TS> arrs{{fl.rho, fl.vel[0], fl.vel[1], fl.vel[2]}};
  const Arr4<TS> vel{{fl.vel[0], fl.vel[1], fl.vel[2], nullptr}};
  const unsigned na = (unsigned)(nc + 1);
  const double qOmega = f.q * f.Omega;
  // the v_y ghosts across a shear face carry the boost -/+ q Omega L_x,
  // except for the residual velocities of orbital advection
  const int boost = f.kind == FORCE_SHEARBOX;
  if (xg)
    for_box_grids(hb, nbox, [](const Box& B) { return B.xg_base >= 0; },
                  [](const Box& B) { return blocks_for((box_n(B, 1) + 2) * (box_n(B, 2) + 2)); },
                  [&](const BoxGrid& g, uint32_t nb) {
                    hipLaunchKernelGGL((k_fill_xghost<TS>), dim3(nb, (unsigned)nc), dim3(256), 0, st, boxes_d, g,
                                       vel, xg, qOmega, tdev, toff, boost);
                  });
  for_box_grids(hb, nbox, [](const Box& B) { return B.ax[0].bc_lo != BC_OPEN; },
                [](const Box& B) { return blocks_for(box_n(B, 1) * box_n(B, 2)); },
                [&](const BoxGrid& g, uint32_t nb) {
                  hipLaunchKernelGGL((k_fill_x<TS>), dim3(nb, na), dim3(256), 0, st, boxes_d, g, arrs, boost,
                                     qOmega, tdev, toff);
                });
  for_box_grids(hb, nbox, [](const Box& B) { return B.ax[1].bc_lo == BC_PERIODIC; },
                [](const Box& B) { return blocks_for((box_n(B, 0) + 2) * box_n(B, 2)); },
                [&](const BoxGrid& g, uint32_t nb) {
                  hipLaunchKernelGGL((k_fill_y<TS>), dim3(nb, na), dim3(256), 0, st, boxes_d, g, arrs);
                });
  for_box_grids(hb, nbox, [](const Box& B) { return B.ndim > 2 && B.ax[2].bc_lo == BC_PERIODIC; },
                [](const Box& B) { return blocks_for((box_n(B, 0) + 2) * (box_n(B, 1) + 2)); },
                [&](const BoxGrid& g, uint32_t nb) {
                  hipLaunchKernelGGL((k_fill_z<TS>), dim3(nb, na), dim3(256), 0, st, boxes_d, g, arrs);
                });
}

template <typename TS>
void launch_fold(const Box* hb, int nbox, const Box* boxes_d, const Forces& f, const double* tdev, double toff,
                 const FView<TS>& fl, hipStream_t st) {
  if (nbox <= 0) return;
  const int nc = box_nc(hb[0]);
  const double qOmega = f.q * f.Omega;
  const Arr4<TS> deps{{fl.dep[0], fl.dep[1], fl.dep[2], fl.dep[3]}};
  const unsigned na = (unsigned)(nc + 1);
  for_box_grids(hb, nbox, [](const Box& B) { return B.ndim > 2 && B.ax[2].bc_lo == BC_PERIODIC; },
                [](const Box& B) { return blocks_for((box_n(B, 0) + 2) * (box_n(B, 1) + 2)); },
                [&](const BoxGrid& g, uint32_t nb) {
                  hipLaunchKernelGGL((k_fold_z<TS>), dim3(nb, na), dim3(256), 0, st, boxes_d, g, deps);
                });
  for_box_grids(hb, nbox, [](const Box& B) { return B.ax[1].bc_lo == BC_PERIODIC; },
                [](const Box& B) { return blocks_for((box_n(B, 0) + 2) * box_n(B, 2)); },
                [&](const BoxGrid& g, uint32_t nb) {
                  hipLaunchKernelGGL((k_fold_y<TS>), dim3(nb, na), dim3(256), 0, st, boxes_d, g, deps);
                });
  // the energy channel reads the D_y ghosts, which no thread of this launch
  // writes (they are cleared by the next one); the energy term of the boost:
  // standard shearing box only
  const TS* dy = fl.dep[hb[0].ndim > 1 ? 1 : 0];
  const int boost_energy = f.kind == FORCE_SHEARBOX;
  auto xfold = [](const Box& B) { return B.ax[0].bc_lo != BC_OPEN; };
  auto xblocks = [](const Box& B) { return blocks_for(box_n(B, 1) * box_n(B, 2)); };
  for_box_grids(hb, nbox, xfold, xblocks, [&](const BoxGrid& g, uint32_t nb) {
    hipLaunchKernelGGL((k_fold_x<TS>), dim3(nb, na), dim3(256), 0, st, boxes_d, g, deps, dy, boost_energy,
                       qOmega, tdev, toff);
  });
  for_box_grids(hb, nbox, xfold, xblocks, [&](const BoxGrid& g, uint32_t nb) {
    hipLaunchKernelGGL((k_clear_x_ghosts<TS>), dim3(nb, na), dim3(256), 0, st, boxes_d, g, deps);
  });
}

template <typename TS>
void launch_feedback(const Box* hb, int nbox, const Box* boxes_d, const FView<TS>& fl, hipStream_t st) {
  for_box_grids(hb, nbox, [](const Box&) { return true; }, [](const Box& B) { return blocks_for(B.ncell); },
                [&](const BoxGrid& g, uint32_t nb) {
                  hipLaunchKernelGGL((k_feedback<TS>), dim3(nb), dim3(256), 0, st, boxes_d, g, fl);
                });
}

template <typename TS>
void launch_grid_sums(const Box* hb, int nbox, const Box* boxes_d, const FView<TS>& fl, DiagDev* dg, double* part,
                      hipStream_t st) {
  if (nbox <= 0) return;
  const int nc = box_nc(hb[0]);
  // blocks shared out in proportion to the stored cells of each launch's
  // boxes (at most GRID_SUM_BLOCKS + MB_BOXES in all)
  for (int b0 = 0; b0 < nbox; b0 += MB_BOXES) {
    const int b1 = std::min(nbox, b0 + MB_BOXES);
    int64_t tot = 0;
    for (int b = b0; b < b1; ++b) tot += hb[b].nstore;
    if (tot == 0) continue;
    for_box_grids(hb + b0, b1 - b0, [](const Box& B) { return B.nstore > 0; },
                  [&](const Box& B) {
                    const int64_t share = (int64_t)GRID_SUM_BLOCKS * B.nstore / tot;
                    return (uint32_t)std::max<int64_t>(1, std::min<int64_t>(blocks_for(B.nstore), share));
                  },
                  [&](BoxGrid g, uint32_t nb) {
                    for (int e = 0; e < g.n; ++e) g.box[e] += b0;
                    hipLaunchKernelGGL((k_grid_sums<TS>), dim3(nb), dim3(256), 0, st, boxes_d, g, fl, part);
                    hipLaunchKernelGGL(k_reduce_grid_partials, dim3(1), dim3(256), 0, st, (const double*)part,
                                       (int)nb, nc, dg);
                  });
  }
}

template <typename TS> void launch_clear_deposits(const FView<TS>& fl, int nch, int64_t n, hipStream_t st) {
  if (n <= 0 || nch <= 0) return;
  const Arr4<TS> deps{{fl.dep[0], fl.dep[1], fl.dep[2], fl.dep[3]}};
  hipLaunchKernelGGL((k_fill_values<TS>), dim3(blocks_for(n), (unsigned)nch), dim3(256), 0, st, deps, n,
                     TS(0));
}

template <typename TS> void launch_fill_value(TS* a, int64_t n, TS v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_fill_value<TS>), dim3(blocks_for(n)), dim3(256), 0, st, a, n, v);
}

#define DUST_INST(TS, A, TW)                                                                      \
  template void launch_gather<TS, A, TW>(const PView<TS>&, const Box*, int, int, int, int,             \
                                         const FView<TS>&, const double*, TW*, TW* const[3],       \
                                         DiagDev*,                                                \
                                         hipStream_t);                                            \
  template void launch_kick<TS, A, TW>(const PView<TS>&, const Box*, int, int, int, int, const Forces&, \
                                       const Species*, int, double, const TW*, const TW* const[3], \
                                       TW* const[4], DiagDev*, double*, hipStream_t);             \
  template void launch_deposit<TS, A, TW>(const PView<TS>&, const Box*, int, int, int, int,            \
                                          const FView<TS>&, const TW* const[4], DiagDev*,         \
                                          hipStream_t);                                           \
  template void launch_deposit_pull<TS, A, TW>(const PView<TS>&, const Box&, int, int, int, const FView<TS>&, \
                                               int, double, const TW* const[4], const uint32_t*,       \
                                               const int64_t*, hipStream_t);

#define DUST_INST_DRIFT(TS, A)                                                                    \
  template void launch_drift<TS, A>(const PView<TS>&, const Box*, int, int, int, int, const Forces&,   \
                                    double, const double*, double, int, DiagDev*, hipStream_t);         \
  template void launch_drag_source<TS, A>(const PView<TS>&, const Box*, int, int, int, int,        \
                                          const FView<TS>&, const Forces&, const Species*, int,     \
                                          double, DiagDev*, hipStream_t);                          \
  template void launch_mass_density<TS, A>(const PView<TS>&, const Box*, int, int, int, int, TS*,  \
                                           const Species*, DiagDev*, hipStream_t);                \
  template void launch_source_coeffs<TS, A>(const PView<TS>&, const Box*, int, int, int, int,      \
                                            const FView<TS>&, const Forces&, const Species*, int,  \
                                            double, bool, A* const[3], DiagDev*, hipStream_t);

DUST_INST_DRIFT(float, double)
DUST_INST_DRIFT(float, float)
DUST_INST_DRIFT(double, double)
DUST_INST(float, double, float)
DUST_INST(float, double, double)
DUST_INST(float, float, float)
DUST_INST(double, double, double)

#define DUST_INST_GRID(TS)                                                                        \
  template void launch_fill<TS>(const Box*, int, const Box*, const Forces&, const double*, double,   \
                                const FView<TS>&, double*, hipStream_t);                          \
  template void launch_fold<TS>(const Box*, int, const Box*, const Forces&, const double*, double,   \
                                const FView<TS>&, hipStream_t);                                   \
  template void launch_feedback<TS>(const Box*, int, const Box*, const FView<TS>&, hipStream_t);     \
  template void launch_grid_sums<TS>(const Box*, int, const Box*, const FView<TS>&, DiagDev*, double*, \
                                     hipStream_t);                                                \
  template void launch_fill_value<TS>(TS*, int64_t, TS, hipStream_t);                              \
  template void launch_clear_deposits<TS>(const FView<TS>&, int, int64_t, hipStream_t);

DUST_INST_GRID(float)
DUST_INST_GRID(double)

}  // namespace dust
