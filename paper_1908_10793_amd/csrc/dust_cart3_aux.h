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

// One particle against global memory, in its own cell's frame (stencil
// cells are stored cells, ghosts included): the path of particles whose
// stencil leaves their tile's window, of particles of another box, and of
// the slots after the binned ones.
template <bool SB, bool MASS>
__device__ void aux_far_particle(const PView<float>& p, int64_t i, const Box* __restrict__ boxes, int nbox,
                                 const FView<float>& fl, float* const outs[3], const Forces& f,
                                 const Species* __restrict__ sp, float inv_dt, DiagDev* dg) {
  constexpr int NC = MASS ? 1 : 3;
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
  const double it = sp->inv_tau[spc];
  const float k = MASS ? float(sp->mass[spc])
                       : float(sp->mass[spc] * (it < double(inv_dt) ? it : double(inv_dt)));
  const double qO = SB ? f.q * f.Omega : 0.0;
  float w[3][3];
#pragma unroll
  for (int d = 0; d < 3; ++d) c3_weights(cb.tsc[d], off[d], w[d]);
  float q[3] = {0.0f, 0.0f, 0.0f};
  if constexpr (MASS) {
    q[0] = k;
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
    for (int m = 0; m < 3; ++m) q[m] = -k * v[m];
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
}

// The listed particles of k_c3_aux, then the slots after the binned ones;
// the last workgroup to finish clears the list's count for the next launch.
template <bool SB, bool MASS>
__global__ void __launch_bounds__(256)
    k_c3_aux_far(PView<float> p, const Box* __restrict__ boxes, int nbox, FView<float> fl,
                 float* __restrict__ out0, float* __restrict__ out1, float* __restrict__ out2, Forces f,
                 const Species* __restrict__ sp, float inv_dt, const uint32_t* __restrict__ list,
                 uint32_t* __restrict__ count, const int64_t* __restrict__ bin_start, int64_t nbins,
                 uint32_t* __restrict__ done, DiagDev* dg) {
  float* const outs[3] = {out0, out1, out2};
  const uint32_t nl = *count;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t e = t; e < nl; e += stride)
    aux_far_particle<SB, MASS>(p, list[e], boxes, nbox, fl, outs, f, sp, inv_dt, dg);
  for (int64_t i = bin_start[nbins] + t; i < p.n; i += stride)
    aux_far_particle<SB, MASS>(p, i, boxes, nbox, fl, outs, f, sp, inv_dt, dg);
  // every workgroup has read the count once it reaches here
  __syncthreads();
  if (threadIdx.x == 0) {
    if (atomicAdd(done, 1u) == gridDim.x - 1) {
      *count = 0u;
      *done = 0u;
    }
  }
}

template <int TX, int TY, int TZ, bool SB, bool MASS>
__global__ void __launch_bounds__(FUSED_THREADS) __attribute__((amdgpu_waves_per_eu(MASS ? 4 : 3)))
    k_c3_aux(const TileDesc* __restrict__ tiles, const uint8_t* __restrict__ tmap, PView<float> p,
             const Box* __restrict__ boxes, FView<float> fl, float* __restrict__ out0,
             float* __restrict__ out1, float* __restrict__ out2, Forces f, const Species* __restrict__ sp,
             float inv_dt, const int64_t* __restrict__ bin_start, uint32_t* __restrict__ far_list,
             uint32_t* __restrict__ far_count, DiagDev* dg) {
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

  // particles loaded one level ahead of their use (a lane without a
  // particle at a level loads the wave's first one, whose value it ignores)
  uint32_t lvl = wl.base;
  const int nlev = __builtin_amdgcn_readfirstlane(wl.nlev);
  uint32_t slot = level_slot(wl, 0, lvl);
  C3Raw nxt;
  if (nlev > 0) c3_load<false>(p, wl.cnt > 0 ? slot : wl.base, nxt);
  for (int j = 0; j < nlev; ++j) {
    const uint32_t i = slot;
    const bool has = wl.cnt > j;
    const C3Raw cur = nxt;
    slot = level_slot(wl, j + 1, lvl);
    if (j + 1 < nlev) c3_load<false>(p, wl.cnt > j + 1 ? slot : wl.base, nxt);
    const int32_t cid = cur.cell;
    float off[3], mom[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      off[d] = cur.off[d];
      mom[d] = MASS ? 0.0f : cur.mom[d];
    }
    int spc = p.species ? cur.species : 0;
    if (spc >= sp->n) spc = 0;
    bool live = has && cid >= cb.cell_base && cid < cb.cell_base + cb.ncell;
    int idx[3] = {mycell[0], mycell[1], mycell[2]};
    if (live && cid != mycid) c3_unravel(cid - cb.cell_base, n0, n1, B.ax[0].inv_n, B.ax[1].inv_n, idx);
    int la = lx + H, lb = ly + H, lcz = lz + H;
    bool inwin = true;
    if (live) {
      la = win_coord(idx[0], ox, n0, RX, cb.per[0]);
      lb = win_coord(idx[1], oy, n1, RY, cb.per[1]);
      lcz = win_coord(idx[2], oz, n2, RZ, cb.per[2]);
      inwin = la >= 1 && la <= RX - 2 && lb >= 1 && lb <= RY - 2 && lcz >= 1 && lcz <= RZ - 2;
    }
    {
      // a particle of another box, or whose stencil leaves the window: to
      // the list of k_c3_aux_far (one atomic per wave)
      const bool away = (has && cid >= 0 && !live) || (live && !inwin);
      const uint64_t am = __ballot(away);
      if (am) {
        const int lane = threadIdx.x & 63;
        const int leader = __ffsll((unsigned long long)am) - 1;
        uint32_t fb = 0;
        if (lane == leader) fb = atomicAdd(far_count, (uint32_t)__popcll(am));
        fb = __shfl(fb, leader, 64);
        if (away) far_list[fb + lanes_below(am)] = i;
      }
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
    bool dep_reg;   // the particle's register-sum share (with weights shifted to this thread's cell)
    if constexpr (MASS) {
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
      dep_reg = mine;
    } else {
      // the particle's cell relative to this thread's cell: in it or (drag
      // source) a neighbour, the part of its stencil inside the thread's 27
      // cells goes to the register sums (weights shifted by the offset), the
      // planes outside to the window; further away, the whole stencil to the
      // window.  The one-channel density keeps the whole stencil for every
      // particle outside the thread's cell (the shifted weights took it from 6
      // to 5 waves per SIMD and cost more than the atomics they save).
      const int sx = la - (lx + H), sy = lb - (ly + H), sz = lcz - (lz + H);
      const bool near = (sx >= -1) & (sx <= 1) & (sy >= -1) & (sy <= 1) & (sz >= -1) & (sz <= 1);
      const int base = la + RX * (lb + RY * lcz);
      auto lds_add = [&](int a, int bb, int cc, float wt) {
        const int r = base + a + RX * (bb + RY * cc);
#pragma unroll
        for (int m = 0; m < NC; ++m) atomicAdd(&dep[m * RC + r], double(wt) * double(q[m]));
      };
      if (use && !near) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int bb = 0; bb < 3; ++bb)
#pragma unroll
            for (int a = 0; a < 3; ++a) lds_add(a - 1, bb - 1, c - 1, w[0][a] * w[1][bb] * w[2][c]);
      }
      if (use && near && (sx | sy | sz)) {
        // row sy, column sx (rows other than sy), layer sz (the cells in neither)
        if (sy != 0) {
          const float wy = sy > 0 ? w[1][2] : w[1][0];
#pragma unroll
          for (int cc = -1; cc <= 1; ++cc)
#pragma unroll
            for (int a = -1; a <= 1; ++a) lds_add(a, sy, cc, w[0][a + 1] * wy * w[2][cc + 1]);
        }
        if (sx != 0) {
          const float wx = sx > 0 ? w[0][2] : w[0][0];
#pragma unroll
          for (int cc = -1; cc <= 1; ++cc)
#pragma unroll
            for (int bb = -1; bb <= 1; ++bb)
              if (sy == 0 || bb != sy) lds_add(sx, bb, cc, wx * w[1][bb + 1] * w[2][cc + 1]);
        }
        if (sz != 0) {
          const float wz = sz > 0 ? w[2][2] : w[2][0];
#pragma unroll
          for (int bb = -1; bb <= 1; ++bb)
#pragma unroll
            for (int a = -1; a <= 1; ++a)
              if ((sy == 0 || bb != sy) && (sx == 0 || a != sx)) lds_add(a, bb, sz, w[0][a + 1] * w[1][bb + 1] * wz);
        }
      }
      {
        const int sd[3] = {sx, sy, sz};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const float w0 = w[d][0], w1 = w[d][1], w2 = w[d][2];
          w[d][0] = sd[d] == 0 ? w0 : sd[d] < 0 ? w1 : 0.0f;
          w[d][1] = sd[d] == 0 ? w1 : sd[d] < 0 ? w2 : w0;
          w[d][2] = sd[d] == 0 ? w2 : sd[d] < 0 ? 0.0f : w1;
        }
      }
      dep_reg = use && near;
    }
    float qf[NC], wq[3][NC];
#pragma unroll
    for (int m = 0; m < NC; ++m) qf[m] = dep_reg ? q[m] : 0.0f;
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

// Workgroups of k_c3_aux_far.
static constexpr int AUX_FAR_BLOCKS = 256;

template <int TX, int TY, int TZ>
void launch_c3_aux_shape(const FusedPlan& plan, const PView<float>& p, const Box* boxes_d, int nbox,
                         const FView<float>& fl, float* const out[3], bool mass, const Forces& f,
                         const Species* sp, double dt, const int64_t* bin_start, int64_t nbins, DiagDev* dg,
                         hipStream_t st) {
  constexpr int RC = (TX + 2 * FUSED_HALO) * (TY + 2 * FUSED_HALO) * (TZ + 2 * FUSED_HALO);
  const float inv_dt = float(1.0 / dt);
  uint32_t* list = plan.defer_list;
  uint32_t* count = plan.defer_count;
  uint32_t* done = plan.defer_count + 1;   // second word of the count block
  const size_t lds = mass ? RC * sizeof(double) : RC * (3 * sizeof(double) + sizeof(float4));
#define DUST_AUX(SBV, MV)                                                                                  \
  do {                                                                                                    \
    if (plan.ntiles > 0)                                                                                  \
      hipLaunchKernelGGL((k_c3_aux<TX, TY, TZ, SBV, MV>), dim3(plan.ntiles), dim3(FUSED_THREADS), lds, st, \
                         plan.tiles_d, plan.tile_map, p, boxes_d, fl, out[0], out[1], out[2], f, sp, inv_dt, \
                         bin_start, list, count, dg);                                                     \
    hipLaunchKernelGGL((k_c3_aux_far<SBV, MV>), dim3(AUX_FAR_BLOCKS), dim3(256), 0, st, p, boxes_d, nbox,  \
                       fl, out[0], out[1], out[2], f, sp, inv_dt, (const uint32_t*)list, count, bin_start,  \
                       nbins, done, dg);                                                                  \
  } while (0)
  if (mass) DUST_AUX(false, true);
  else if (f.kind == FORCE_SHEARBOX) DUST_AUX(true, false);
  else DUST_AUX(false, false);
#undef DUST_AUX
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
