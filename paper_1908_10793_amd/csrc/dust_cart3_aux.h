// Predictor drag source and dust density on the binned layout of the
// uniform-Cartesian FP32 path (gfx950): the tile kernel and its launcher;
// dust_cart3_aux.hip instantiates it for every tile shape.
#pragma once

#include "dust_cart3_kern.h"

namespace dust {

// ------------------------------------------------------------------ predictor source, dust density

// Source of the gas predictor (drag force density with tau' = max(tau, dt))
// or dust density, on the binned layout that the last fused step left: the
// threads, cells and slots of that step's last rebinning (c3_layout over
// tmap and bin_start), whose particles have since moved by at most a few
// steps.  A particle in its thread's cell adds its stencil to the thread's
// register sums over the 27 cells around it; one elsewhere in the window
// adds it to the FP64 LDS window; one whose stencil leaves the window (or
// any particle of the slots after the binned ones, the extra workgroups)
// is done against global memory, in its own cell's frame.  At current
// positions, no drift.  MASS: the density (one channel, mass m_p, no gas);
// else the source -W m_p / tau'_p (v_g - v_p) / dV into the three momentum
// channels, with the slip in the residual form of the tile kernel (SB: v_y
// relative to the background shear).
template <bool SB>
__device__ __forceinline__ float aux_gas_residual(const Box& B, const FView<float>& fl, int m, int i, int j,
                                                  int k, double qO) {
  const double v = double(fl.vel[m][stored_index(B, i, j, k)]);
  if (SB && m == 1) return float(v + qO * (B.ax[0].lo + (double(i) + 0.5) * B.ax[0].d));
  return float(v);
}

template <int TX, int TY, int TZ, bool SB, bool MASS>
__global__ void __launch_bounds__(FUSED_THREADS)
    k_c3_aux(const TileDesc* __restrict__ tiles, int ntiles, const uint8_t* __restrict__ tmap,
             PView<float> p, const Box* __restrict__ boxes, int nbox, FView<float> fl,
             float* __restrict__ out0, float* __restrict__ out1, float* __restrict__ out2, Forces f,
             const Species* __restrict__ sp, float inv_dt, const int64_t* __restrict__ bin_start,
             int64_t nbins, DiagDev* dg) {
  constexpr int H = FUSED_HALO;
  constexpr int RX = TX + 2 * H, RY = TY + 2 * H, RZ = TZ + 2 * H;
  constexpr int RC = RX * RY * RZ;
  constexpr int NC = MASS ? 1 : 3;
  extern __shared__ double smem[];
  double* dep = smem;                                          // NC * RC (FP64)
  float4* gas = reinterpret_cast<float4*>(smem + NC * RC);     // RC (source only)
  __shared__ float sp_k[DUST_MAX_SPECIES];
  __shared__ float2 xres[RX];
  float* const outs[3] = {out0, out1, out2};
  if (threadIdx.x < sp->n) {
    const double it = sp->inv_tau[threadIdx.x];
    sp_k[threadIdx.x] = MASS ? float(sp->mass[threadIdx.x])
                             : float(sp->mass[threadIdx.x] * (it < double(inv_dt) ? it : double(inv_dt)));
  }
  const double qO = SB ? f.q * f.Omega : 0.0;

  // global-memory step of one particle (own cell's frame: stencil cells are
  // stored cells, ghosts included)
  auto far = [&](const Box& B, const C3Box& cb, const int idx[3], const float off[3], const float mom[3],
                 int spc) {
    float w[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) c3_weights(cb.tsc[d], off[d], w[d]);
    float q[3] = {0.0f, 0.0f, 0.0f};
    if constexpr (MASS) {
      q[0] = sp_k[spc];
    } else {
      float u[3] = {mom[0], mom[1], mom[2]};
      if (SB) u[1] = float(double(mom[1]) + qO * (B.ax[0].lo + (double(idx[0]) + 0.5 + double(off[0])) * B.ax[0].d));
      float v[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const float wt = w[0][a] * w[1][bb] * w[2][c];
#pragma unroll
            for (int m = 0; m < 3; ++m)
              v[m] += wt * (aux_gas_residual<SB>(B, fl, m, idx[0] + a - 1, idx[1] + bb - 1, idx[2] + c - 1, qO) - u[m]);
          }
#pragma unroll
      for (int m = 0; m < 3; ++m) q[m] = -sp_k[spc] * v[m];
    }
    const float iv = float(inv_volume(B, 0, 0, 0));
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int bb = 0; bb < 3; ++bb)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float wt = w[0][a] * w[1][bb] * w[2][c] * iv;
          const int64_t id = stored_index(B, idx[0] + a - 1, idx[1] + bb - 1, idx[2] + c - 1);
#pragma unroll
          for (int m = 0; m < NC; ++m) unsafeAtomicAdd(&outs[m][id], wt * q[m]);
        }
  };
  auto load_far = [&](int64_t i) {
    const int32_t cid = p.cell[i];
    if (cid < 0) return;
    const int b = find_box(boxes, nbox, cid);
    const Box& B = boxes[b];
    if (cid >= B.cell_base + B.ncell) {
      flag(dg, DUST_FLAG_BAD_CELL);
      return;
    }
    const C3Box cb = c3_box(B, 0.0f);
    int idx[3];
    c3_unravel(cid - cb.cell_base, cb.n[0], cb.n[1], B.ax[0].inv_n, B.ax[1].inv_n, idx);
    float off[3], mom[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      off[d] = p.off[d][i];
      mom[d] = MASS ? 0.0f : p.mom[d][i];
    }
    int spc = p.species ? p.species[i] : 0;
    if (spc >= sp->n) spc = 0;
    far(B, cb, idx, off, mom, spc);
  };

  if ((int)blockIdx.x >= ntiles) {
    // slots after the binned ones (normally particles without a cell)
    const int64_t first = bin_start[nbins];
    for (int64_t i = first + (int64_t)(blockIdx.x - ntiles) * FUSED_THREADS + threadIdx.x; i < p.n;
         i += (int64_t)(gridDim.x - ntiles) * FUSED_THREADS)
      load_far(i);
    return;
  }

  const TileDesc td = tiles[blockIdx.x];
  const Box& B = boxes[td.box];
  const C3Box cb = c3_box(B, 0.0f);
  const int ox = td.i0 - H, oy = td.j0 - H, oz = td.k0 - H;
  const double x_lo = B.ax[0].lo, dx0 = B.ax[0].d;
  if (SB && threadIdx.x < RX) {
    const double v = qO * (x_lo + (double(ox + (int)threadIdx.x) + 0.5) * dx0);
    const float hi = float(v);
    xres[threadIdx.x] = make_float2(hi, float(v - double(hi)));
  }
  const int n0 = cb.n[0], n1 = cb.n[1], n2 = cb.n[2];
  // the window: stored cells (ghosts) within one cell of the box, periodic
  // images beyond; gas staged as read (residual form), deposits cleared
  for (int r = threadIdx.x; r < RC; r += FUSED_THREADS) {
    const int a = r % RX, bq = (r / RX) % RY, cq = r / (RX * RY);
    int i = ox + a, j = oy + bq, k = oz + cq;
    if (cb.per[0] && (i < -1 || i > n0)) i = wrap_index(i, n0);
    if (cb.per[1] && (j < -1 || j > n1)) j = wrap_index(j, n1);
    if (cb.per[2] && (k < -1 || k > n2)) k = wrap_index(k, n2);
    const bool in = i >= -1 && i <= n0 && j >= -1 && j <= n1 && k >= -1 && k <= n2;
    if constexpr (!MASS) {
      float gv[3] = {0.0f, 0.0f, 0.0f};
      if (in) {
#pragma unroll
        for (int m = 0; m < 3; ++m) gv[m] = aux_gas_residual<SB>(B, fl, m, i, j, k, qO);
      }
      gas[r] = make_float4(gv[0], gv[1], gv[2], 0.0f);
    }
#pragma unroll
    for (int m = 0; m < NC; ++m) dep[m * RC + r] = 0.0;
  }
  __syncthreads();

  const int lc = (int)threadIdx.x < td.ex * td.ey * td.ez ? (int)tmap[(size_t)blockIdx.x * 256 + threadIdx.x]
                                                         : -1;
  int64_t ps;
  const WaveLevels wl = c3_layout(td, lc, bin_start, ps);
  const bool own = lc >= 0;
  const int lx = own ? lc % td.ex : 0, ly = own ? (lc / td.ex) % td.ey : 0,
            lz = own ? lc / (td.ex * td.ey) : 0;
  const int mycell[3] = {td.i0 + lx, td.j0 + ly, td.k0 + lz};
  const int mybase = (lx + H) + RX * ((ly + H) + RY * (lz + H));
  const int32_t mycid = cb.cell_base + mycell[0] + n0 * (mycell[1] + n1 * mycell[2]);
  const float qOdx = float(qO * dx0);

  float acc[27][NC];
#pragma unroll
  for (int o = 0; o < 27; ++o)
#pragma unroll
    for (int m = 0; m < NC; ++m) acc[o][m] = 0.0f;

  uint32_t lvl = wl.base;
  const int nlev = __builtin_amdgcn_readfirstlane(wl.nlev);
  for (int j = 0; j < nlev; ++j) {
    const uint32_t i = level_slot(wl, j, lvl);
    const bool has = wl.cnt > j;
    const uint32_t li = has ? i : wl.base;
    const int32_t cid = at32(p.cell, li);
    float off[3], mom[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      off[d] = at32(p.off[d], li);
      mom[d] = MASS ? 0.0f : at32(p.mom[d], li);
    }
    int spc = p.species ? (int)at32(p.species, li) : 0;
    if (spc >= sp->n) spc = 0;
    bool live = has && cid >= cb.cell_base && cid < cb.cell_base + cb.ncell;
    if (has && cid >= 0 && !live) {
      // another box, or bad: the global path decides
      load_far(i);
    }
    int idx[3] = {mycell[0], mycell[1], mycell[2]};
    if (live && cid != mycid) c3_unravel(cid - cb.cell_base, n0, n1, B.ax[0].inv_n, B.ax[1].inv_n, idx);
    int la = lx + H, lb = ly + H, lcz = lz + H;
    bool inwin = true;
    if (live) {
      la = win_coord(idx[0], ox, n0, RX, cb.per[0]);
      lb = win_coord(idx[1], oy, n1, RY, cb.per[1]);
      lcz = win_coord(idx[2], oz, n2, RZ, cb.per[2]);
      inwin = la >= 1 && la <= RX - 2 && lb >= 1 && lb <= RY - 2 && lcz >= 1 && lcz <= RZ - 2;
      if (!inwin) far(B, cb, idx, off, mom, spc);
    }
    const bool use = live && inwin;
    if (!use) {
#pragma unroll
      for (int d = 0; d < 3; ++d) off[d] = 0.0f;
      la = lx + H;
      lb = ly + H;
      lcz = lz + H;
    }
    float w[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) c3_weights(cb.tsc[d], off[d], w[d]);
    float q[NC];
    if constexpr (MASS) {
      q[0] = use ? sp_k[spc] : 0.0f;
    } else {
      float v[3] = {0.0f, 0.0f, 0.0f};
      int r0 = la + RX * (lb - 1 + RY * (lcz - 1));
#pragma unroll 1
      for (int c = 0; c < 3; ++c, r0 += RX * RY) {
        const float wz = c == 0 ? w[2][0] : c == 1 ? w[2][1] : w[2][2];
        float4 g[9];
#pragma unroll
        for (int q9 = 0; q9 < 9; ++q9) g[q9] = gas[r0 + RX * (q9 / 3) + (q9 % 3) - 1];
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
          const float4 g0 = g[3 * bb], g1 = g[3 * bb + 1], g2 = g[3 * bb + 2];
          const float ux = w[0][0] * g0.x + w[0][1] * g1.x + w[0][2] * g2.x;
          const float uy = w[0][0] * g0.y + w[0][1] * g1.y + w[0][2] * g2.y;
          const float uz = w[0][0] * g0.z + w[0][1] * g1.z + w[0][2] * g2.z;
          const float wbc = w[1][bb] * wz;
          v[0] += wbc * ux;
          v[1] += wbc * uy;
          v[2] += wbc * uz;
        }
      }
      float u1 = mom[1];
      if constexpr (SB) {
        const float2 xr = xres[la];
        u1 = (mom[1] + xr.x) + fmaf(qOdx, off[0], xr.y);
      }
      const float k = use ? -sp_k[spc] : 0.0f;
      q[0] = k * (v[0] - mom[0]);
      q[1] = k * (v[1] - u1);
      q[2] = k * (v[2] - mom[2]);
    }
    const bool mine = use && la == lx + H && lb == ly + H && lcz == lz + H;
    if (use && !mine) {
      const int base = la + RX * (lb + RY * lcz);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const double wt = double(w[0][a] * w[1][bb] * w[2][c]);
            const int r = base + (a - 1) + RX * ((bb - 1) + RY * (c - 1));
#pragma unroll
            for (int m = 0; m < NC; ++m) atomicAdd(&dep[m * RC + r], wt * double(q[m]));
          }
    }
    float qf[NC], wq[3][NC];
#pragma unroll
    for (int m = 0; m < NC; ++m) qf[m] = mine ? q[m] : 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int m = 0; m < NC; ++m) wq[a][m] = w[0][a] * qf[m];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) {
        const float wbc = w[1][bb] * w[2][c];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int m = 0; m < NC; ++m) acc[a + 3 * (bb + 3 * c)][m] = fmaf(wbc, wq[a][m], acc[a + 3 * (bb + 3 * c)][m]);
      }
  }
  if (own) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int bb = 0; bb < 3; ++bb)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int r = mybase + (a - 1) + RX * ((bb - 1) + RY * (c - 1));
#pragma unroll
          for (int m = 0; m < NC; ++m)
            if (acc[a + 3 * (bb + 3 * c)][m] != 0.0f) atomicAdd(&dep[m * RC + r], double(acc[a + 3 * (bb + 3 * c)][m]));
        }
  }
  __syncthreads();
  const double iv = inv_volume(B, 0, 0, 0);
  for (int r = threadIdx.x; r < RC; r += FUSED_THREADS) {
    const int a = r % RX, bq = (r / RX) % RY, cq = r / (RX * RY);
    int i = ox + a, j = oy + bq, k = oz + cq;
    if (cb.per[0] && (i < -1 || i > n0)) i = wrap_index(i, n0);
    if (cb.per[1] && (j < -1 || j > n1)) j = wrap_index(j, n1);
    if (cb.per[2] && (k < -1 || k > n2)) k = wrap_index(k, n2);
    const bool in = i >= -1 && i <= n0 && j >= -1 && j <= n1 && k >= -1 && k <= n2;
    if (!in) continue;
    const int64_t id = stored_index(B, i, j, k);
#pragma unroll
    for (int m = 0; m < NC; ++m) {
      const double x = dep[m * RC + r];
      if (x != 0.0) unsafeAtomicAdd(&outs[m][id], float(x * iv));
    }
  }
}

// extra workgroups of k_c3_aux for the slots after the binned ones
static constexpr int AUX_TAIL_BLOCKS = 64;

template <int TX, int TY, int TZ>
void launch_c3_aux_shape(const FusedPlan& plan, const PView<float>& p, const Box* boxes_d, int nbox,
                         const FView<float>& fl, float* const out[3], bool mass, const Forces& f,
                         const Species* sp, double dt, const int64_t* bin_start, int64_t nbins, DiagDev* dg,
                         hipStream_t st) {
  constexpr int RC = (TX + 2 * FUSED_HALO) * (TY + 2 * FUSED_HALO) * (TZ + 2 * FUSED_HALO);
  const dim3 grid(plan.ntiles + AUX_TAIL_BLOCKS);
  const float inv_dt = float(1.0 / dt);
  if (mass) {
    hipLaunchKernelGGL((k_c3_aux<TX, TY, TZ, false, true>), grid, dim3(FUSED_THREADS), RC * sizeof(double), st,
                       plan.tiles_d, plan.ntiles, plan.tile_map, p, boxes_d, nbox, fl, out[0], out[1], out[2], f,
                       sp, inv_dt, bin_start, nbins, dg);
    return;
  }
  const size_t lds = RC * (3 * sizeof(double) + sizeof(float4));
  if (f.kind == FORCE_SHEARBOX)
    hipLaunchKernelGGL((k_c3_aux<TX, TY, TZ, true, false>), grid, dim3(FUSED_THREADS), lds, st, plan.tiles_d,
                       plan.ntiles, plan.tile_map, p, boxes_d, nbox, fl, out[0], out[1], out[2], f, sp, inv_dt,
                       bin_start, nbins, dg);
  else
    hipLaunchKernelGGL((k_c3_aux<TX, TY, TZ, false, false>), grid, dim3(FUSED_THREADS), lds, st, plan.tiles_d,
                       plan.ntiles, plan.tile_map, p, boxes_d, nbox, fl, out[0], out[1], out[2], f, sp, inv_dt,
                       bin_start, nbins, dg);
}

#define DUST_C3_AUX_SHAPE_DECL(PREFIX, TX, TY, TZ)                                                          \
  PREFIX template void launch_c3_aux_shape<TX, TY, TZ>(                                                     \
      const FusedPlan&, const PView<float>&, const Box*, int, const FView<float>&, float* const[3], bool,   \
      const Forces&, const Species*, double, const int64_t*, int64_t, DiagDev*, hipStream_t);
#define DUST_C3_AUX_SHAPES(PREFIX)                                                                          \
  DUST_C3_AUX_SHAPE_DECL(PREFIX, 8, 8, 4)                                                                   \
  DUST_C3_AUX_SHAPE_DECL(PREFIX, 16, 4, 4)                                                                  \
  DUST_C3_AUX_SHAPE_DECL(PREFIX, 4, 16, 4)                                                                  \
  DUST_C3_AUX_SHAPE_DECL(PREFIX, 4, 4, 16)                                                                  \
  DUST_C3_AUX_SHAPE_DECL(PREFIX, 8, 4, 8)                                                                   \
  DUST_C3_AUX_SHAPE_DECL(PREFIX, 4, 8, 8)

}  // namespace dust
