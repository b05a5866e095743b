// Fused tile step for uniform 3-D Cartesian boxes in FP32 storage and
// arithmetic (gfx950): the path of the batched boxes and of the shearing box.
// The kernel and its launchers; dust_cart3.hip holds the rebinning kernels
// and the dispatcher, dust_cart3_i_*.hip one tile shape each.
//
// Same plan, binning and deferred-particle kernel as the general tile kernel
// (dust_fused_kern.h); what differs is written for the short instruction path
// this case allows:
//  * the cells of a tile are assigned to threads in descending order of their
//    particle count (ranked once per rebinning, k_c3_level_perm), so that a
//    wave, which runs as many levels as its fullest cell, holds cells of
//    similar counts;
//  * the half drift is one FMA per axis with the half step over the cell
//    width formed once per workgroup;
//  * the gather is the plain weighted sum of the staged gas.  In the standard
//    shearing box the window stages the gas velocity relative to the
//    background shear, v_y + q Omega x_c (formed in FP64 at the cell centre;
//    the x ghosts from the FP64 ghost layer), and the particle's v_y + q
//    Omega x_p is formed from the cell-centre term split in two FP32 words:
//    the weights reproduce linear fields exactly, so the slip keeps its
//    accuracy where |v| is a thousand times the slip;
//  * the particle diagnostic sums are FP32 per thread (a thread's cell),
//    added in FP64 across the workgroup.
// Deposits are summed in registers over the 27 cells around the thread's
// cell (with weights shifted for a particle that moved to a neighbouring cell
// since the rebinning; the stencil planes outside go to an FP64 LDS window
// with atomics), then the window is added to the grid.
#pragma once

#include "dust_fused_kern.h"

namespace dust {


// Move by dxc cells along one axis of a uniform grid (offset renormalised into
// [-1/2, 1/2)); returns the new cell index (not wrapped).  Without branches
// (a wave takes a branch whenever one of its lanes crosses a face): the
// nearest integer k splits the new offset d exactly (d - k is exact in FP32
// for |d| < 2^23), a tie at +1/2 goes to the next cell, and an offset that
// stays in its cell is kept as it is.
__device__ __forceinline__ int c3_move(int i, float& off, float v, float hinv) {
  const float dn = fmaf(v, hinv, off);
  const float k = rintf(dn);
  const float r0 = k == 0.0f ? dn : dn - k;
  const bool up = r0 >= 0.5f;
  off = up ? r0 - 1.0f : r0;
  return i + (int)k + (up ? 1 : 0);
}

// floor(a / n) and a - n floor(a / n) for 0 <= a < 2^24, 1 <= n < 2^24,
// through an FP32 reciprocal: a is exact in FP32 and the product is within
// one of the quotient, so one correction step makes it exact.  Both factors
// of q n are below 2^24: the full-rate 24-bit multiply.
__device__ __forceinline__ int c3_div24(int a, int n, float inv, int& rem) {
  int q = (int)(float(a) * inv);
  const int r = a - __umul24((unsigned)q, (unsigned)n);
  const bool hi = r >= n, lo = r < 0;
  q += hi ? 1 : (lo ? -1 : 0);
  rem = hi ? r - n : (lo ? r + n : r);
  return q;
}

// Cell coordinates of a local cell id: FP32 reciprocals where small (ids and
// box sides below 2^24), else FP64 (one correction each).
__device__ __forceinline__ void c3_unravel(int l, int n0, int n1, double inv0, double inv1, int idx[3],
                                           bool small) {
  if (small) {
    const int r = c3_div24(l, n0, float(inv0), idx[0]);
    idx[2] = c3_div24(r, n1, float(inv1), idx[1]);
  } else {
    const int r = div_small(l, n0, inv0);
    const int k = div_small(r, n1, inv1);
    idx[0] = l - r * n0;
    idx[1] = r - k * n1;
    idx[2] = k;
  }
}
__device__ __forceinline__ void c3_unravel(int l, int n0, int n1, double inv0, double inv1, int idx[3]) {
  c3_unravel(l, n0, n1, inv0, inv1, idx, l < (1 << 24) && n0 < (1 << 24) && n1 < (1 << 24));
}

// Uniform constants of the workgroup's box.
struct C3Box {
  int n[3];
  float hinv[3];        // (dt/2) / cell width
  float dtinv[3];       // dt / cell width (displacement diagnostic)
  bool per[3];          // periodic axis
  bool shear;           // shear-periodic x
  bool tsc[3];
  int cell_base, ncell;
};

__device__ __forceinline__ C3Box c3_box(const Box& B, float dt) {
  C3Box c;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    c.n[d] = B.ax[d].n;
    c.hinv[d] = float(0.5 * double(dt) * B.ax[d].inv_d);
    c.dtinv[d] = float(double(dt) * B.ax[d].inv_d);
    c.per[d] = B.ax[d].bc_lo == BC_PERIODIC && B.ax[d].bc_hi == BC_PERIODIC;
    c.tsc[d] = B.ax[d].shape == SHAPE_TSC;
  }
  c.shear = B.ax[0].bc_lo == BC_SHEAR;
  c.cell_base = (int)B.cell_base;
  c.ncell = (int)B.ncell;
  return c;
}

// Cell id of cell (i, j, k) of the box: 24-bit products (full rate) when
// small (the box has fewer than 2^24 cells, so that every factor and product
// fits).
__device__ __forceinline__ int32_t c3_cell_id(const C3Box& cb, int i, int j, int k, bool small) {
  if (small)
    return cb.cell_base + i +
           (int)__umul24((unsigned)cb.n[0], (unsigned)(j + (int)__umul24((unsigned)cb.n[1], (unsigned)k)));
  return cb.cell_base + i + cb.n[0] * (j + cb.n[1] * k);
}

// Weights of cells i-1, i, i+1 of one axis (b-spline overlaps, Eq. b0 / b1),
// middle weight 1 - w0 - w2.
__device__ __forceinline__ void c3_weights(bool tsc, float d, float w[3]) {
  // both forms, blended by t = 1 (TSC) or 0 (CIC): t a + (1 - t) b is a or b
  // exactly, and no branch on the box's shape
  const float t = tsc ? 1.0f : 0.0f, u = 1.0f - t;
  const float m = 0.5f - d, p = 0.5f + d;
  w[0] = fmaf(t, 0.5f * m * m, u * (d < 0.0f ? -d : 0.0f));
  w[2] = fmaf(t, 0.5f * p * p, u * (d > 0.0f ? d : 0.0f));
  w[1] = 1.0f - w[0] - w[2];
}

// Wrap a cell index along a periodic axis: one box length (the normal case),
// else by the remainder (a particle that moved further, whatever its speed,
// still gets a cell of the box).
__device__ __forceinline__ int c3_wrap(int i, int n) {
  i = i < 0 ? i + n : (i >= n ? i - n : i);
  if (i < 0 || i >= n) {
    i %= n;
    if (i < 0) i += n;
  }
  return i;
}

// The wave layout of a tile's particles: thread t owns the tile-local cell
// lc (the cell of rank t by descending particle count, -1 if none); wave w's
// particles follow those of waves 0..w-1 from the tile's first slot on,
// level-major inside the wave.  Returns this thread's WaveLevels; ps: the
// first sorted slot of its cell.
__device__ __forceinline__ WaveLevels c3_layout(const TileDesc& td, int lc,
                                                const int64_t* __restrict__ bin_start, int64_t& ps) {
  __shared__ uint32_t wtot[FUSED_THREADS / 64];
  const int t = threadIdx.x;
  int cnt = 0;
  ps = 0;
  if (lc >= 0) {
    ps = bin_start[td.key0 + lc];
    cnt = (int)(bin_start[td.key0 + lc + 1] - ps);
  }
  const uint32_t tot = (uint32_t)wave_sum(cnt);
  if ((t & 63) == 0) wtot[t >> 6] = tot;
  __syncthreads();
  uint32_t base = (uint32_t)bin_start[td.key0];
  for (int w = 0; w < (t >> 6); ++w) base += wtot[w];
  WaveLevels wl;
  wl.cnt = cnt;
  wl.nlev = wave_max(cnt);
  wl.base = base;
  return wl;
}

// Element i (a slot number) of a particle array through a 32-bit byte
// offset from the (workgroup-uniform) base: the global instructions' scalar
// base + vector offset form, with no 64-bit address arithmetic per access.
// The path takes fewer than 2^30 particles, so 4 i < 2^32.
template <typename T> __device__ __forceinline__ const T& at32(const T* base, uint32_t i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T));
}
template <typename T> __device__ __forceinline__ T& at32(T* base, uint32_t i) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (uint32_t)sizeof(T));
}

// Stored state of a particle and its species (masses and stopping times
// come from the species table on this path).
struct C3Raw {
  int32_t cell, species, id;
  float off[3], mom[3];
};

// ID: also the id (when the attributes are copied to another buffer).
template <bool ID>
__device__ __forceinline__ void c3_load(const PView<float>& p, uint32_t i, C3Raw& r) {
  r.cell = at32(p.cell, i);
  // the id and species arrays may be absent: the loads then read an element
  // of the cell array, and the value is ignored where it is used (a load on
  // a select rather than on a branch, and no wait right after it)
  if constexpr (ID) r.id = at32(p.id ? p.id : p.cell, p.id ? i : 0u);
  else r.id = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    r.off[d] = at32(p.off[d], i);
    r.mom[d] = at32(p.mom[d], i);
  }
  r.species = (int32_t)at32(p.species ? p.species : reinterpret_cast<const uint8_t*>(p.cell),
                            p.species ? i : 0u);
}

// The stencil planes of a particle one cell off its thread's cell (shift
// sx, sy, sz in -1..1, not all 0) that lie outside the thread's 27 cells, to
// the FP64 deposit window: row sy, column sx (rows other than sy), layer sz
// (the cells in neither).  base: window index of the particle's cell; w:
// its weights; q: its 4 deposit channels.
template <int RX, int RY, int RC>
__device__ __forceinline__ void c3_spill_planes(double* dep, int base, int sx, int sy, int sz, const float w[3][3],
                                                const float q[4]) {
  auto lds_add = [&](int a, int bb, int cc, float wt) {
    const int r0 = base + a + RX * (bb + RY * cc);
#pragma unroll
    for (int k = 0; k < 4; ++k) atomicAdd(&dep[k * RC + r0], double(wt * q[k]));
  };
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

// The fused step.  SB: standard shearing-box forces (else none or a constant
// acceleration).  SMALL: every box of the launch has fewer than 2^24 cells.  REBIN: the step after a rebinning (particles read through
// src_index, attributes copied, input checks); else COPY: stale bins written
// to another buffer slot for slot (attributes copied), or in place.  Masses
// and stopping times come from the species table.
template <int TX, int TY, int TZ, bool SB, bool REBIN, bool COPY, bool SMALL>
__global__ void __launch_bounds__(FUSED_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
    k_c3(const TileDesc* __restrict__ tiles, const uint8_t* __restrict__ tmap, PView<float> p,
         PView<float> dst, int copy_attrs, const Box* __restrict__ boxes, FView<float> fl, Forces f,
         const Species* __restrict__ sp, int drag_mode, float dt, const double* __restrict__ tdev,
         const int64_t* __restrict__ bin_start, const double* __restrict__ xg, DiagDev* dg,
         double* __restrict__ part, int sums, uint32_t* __restrict__ defer_list,
         uint32_t* __restrict__ defer_count, const uint32_t* __restrict__ src_index) {
  constexpr int H = FUSED_HALO;
  constexpr int RX = TX + 2 * H, RY = TY + 2 * H, RZ = TZ + 2 * H;
  constexpr int RC = RX * RY * RZ;
  extern __shared__ double smem[];
  double* dep = smem;                                                  // 4 * RC (FP64)
  float4* gas = reinterpret_cast<float4*>(smem + 4 * RC);              // RC
  // per species: mass, c, and the step factors h1 = dt (1 + psi) and dt psi of
  // Eq. exp_midpoint; in the shearing box also W = Omega h1 and 1 / (1 + W^2)
  __shared__ float4 sp_k[DUST_MAX_SPECIES];
  __shared__ float2 sp_w[DUST_MAX_SPECIES];
  __shared__ float2 xres[RX];   // SB: q Omega x_c of the window's x columns, as hi + lo
  // Each wave's queue of particles one cell off their thread's cell (their
  // outer stencil planes go to the window): window index of the particle's
  // cell, shift code, offsets at x^{n+1/2}, deposits.  Queued rather than
  // deposited at once, because a handful of such lanes would otherwise hold
  // the whole wave in the planes' LDS atomics on most iterations; the wave
  // drains its queue with every lane busy.
  constexpr int NW = FUSED_THREADS / 64;
  __shared__ int spq_r[NW][64], spq_s[NW][64];
  __shared__ float spq_o[NW][3][64], spq_q[NW][4][64];
  // where the particles are written: stale bins in place write the arrays
  // they read (the same pointers, held once)
  const PView<float>& out = COPY ? dst : p;
  const TileDesc td = tiles[blockIdx.x];
  const Box& B = boxes[td.box];
  const C3Box cb = c3_box(B, dt);
  const int ox = td.i0 - H, oy = td.j0 - H, oz = td.k0 - H;
  // window index of window coordinates a, b >= 0, c >= 0 (24-bit products:
  // full rate, where a 32-bit product by RX or RX RY would take four passes)
  auto win = [](int a, int b, int c) {
    return a + (int)__umul24((unsigned)RX, (unsigned)(b + (int)__umul24((unsigned)RY, (unsigned)c)));
  };
  if (threadIdx.x < sp->n) {
    float c, psi;
    propagator<float>(dt * float(sp->inv_tau[threadIdx.x]), c, psi);
    const float h1 = dt + dt * psi;
    sp_k[threadIdx.x] = make_float4(float(sp->mass[threadIdx.x]), c, h1, dt * psi);
    if (SB) {
      const float W = float(f.Omega) * h1;
      sp_w[threadIdx.x] = make_float2(W, 1.0f / (1.0f + W * W));
    }
  }
  const double qO = SB ? f.q * f.Omega : 0.0;
  const double x_lo = B.ax[0].lo, dx0 = B.ax[0].d;
  if (SB && threadIdx.x < RX) {
    const double v = qO * (x_lo + (double(ox + (int)threadIdx.x) + 0.5) * dx0);
    const float hi = float(v);
    xres[threadIdx.x] = make_float2(hi, float(v - double(hi)));
  }
  const double t0 = *tdev;
  const int n0 = cb.n[0], n1 = cb.n[1], n2 = cb.n[2];
  // stage the gas window (periodic images beyond the box), clear the deposit window
  for (int r = threadIdx.x; r < RC; r += FUSED_THREADS) {
    const int a = r % RX, bq = (r / RX) % RY, cq = r / (RX * RY);
    int i = ox + a, j = oy + bq, k = oz + cq;
    if (cb.per[0]) i = wrap_index(i, n0);
    if (cb.per[1]) j = wrap_index(j, n1);
    if (cb.per[2]) k = wrap_index(k, n2);
    const bool in = i >= -1 && i <= n0 && j >= -1 && j <= n1 && k >= -1 && k <= n2;
    float gv[3] = {0.0f, 0.0f, 0.0f};
    if (in) {
      if (SB) {
        // velocity relative to the background shear, formed in FP64
        const double xc = x_lo + (double(i) + 0.5) * dx0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const double v = gas_comp(B, fl, xg, m, i, j, k);
          gv[m] = float(m == 1 ? v + qO * xc : v);
        }
      } else {
        const int64_t id = stored_index(B, i, j, k);
#pragma unroll
        for (int m = 0; m < 3; ++m) gv[m] = fl.vel[m][id];
      }
    }
    gas[r] = make_float4(gv[0], gv[1], gv[2], 0.0f);
#pragma unroll
    for (int m = 0; m < 4; ++m) dep[m * RC + r] = 0.0;
  }
  __syncthreads();

  // this thread's cell (ranked by particle count) and the wave's slot layout
  const int lc = (int)threadIdx.x < td.ex * td.ey * td.ez ? (int)tmap[(size_t)blockIdx.x * 256 + threadIdx.x]
                                                         : -1;
  int64_t ps;
  const WaveLevels wl = c3_layout(td, lc, bin_start, ps);
  const bool own = lc >= 0;
  const int lx = own ? lc % td.ex : 0, ly = own ? (lc / td.ex) % td.ey : 0,
            lz = own ? lc / (td.ex * td.ey) : 0;
  const int mycell[3] = {td.i0 + lx, td.j0 + ly, td.k0 + lz};
  const int mybase = (lx + H) + RX * ((ly + H) + RY * (lz + H));
  // boxes of fewer than 2^24 cells: FP32 division and 24-bit products (known
  // at compile time when every box of the launch is that small)
  const bool small = SMALL || cb.ncell < (1 << 24);
  const int32_t mycid = c3_cell_id(cb, mycell[0], mycell[1], mycell[2], small);

  float acc[27][4];
#pragma unroll
  for (int o = 0; o < 27; ++o)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[o][k] = 0.0f;
  // FP32 diagnostic sums of this thread's particles (impulse, energy, |impulse|,
  // largest displacement), added in FP64 across the workgroup at the end
  float s_j0 = 0.0f, s_j1 = 0.0f, s_j2 = 0.0f, s_e = 0.0f, s_abs = 0.0f, s_cells = 0.0f;
  const float Om = float(f.Omega);
  const float qOdx = float(qO * dx0);
  const float g0c = float(f.g[0]), g1c = float(f.g[1]), g2c = float(f.g[2]);
  const bool cg = !SB && f.kind == FORCE_CONST;
  const float gz_c = SB && f.vertical_gravity ? -Om * Om : 0.0f;
  const float z_lo = float(B.ax[2].lo), dz = float(B.ax[2].d);

  // The results of a particle are stored at the top of the next iteration,
  // before the next prefetch: on this target one counter tracks both loads
  // and stores, so waiting for prefetched data also waits for every store
  // issued before that wait; stores issued at the end of an iteration would
  // put a full write round trip on every iteration, while stores issued at
  // its top have had the whole iteration to complete by the next wait.
  bool pend = false, pend_attr = false;
  uint32_t pend_i = 0;
  int32_t pend_cell = 0, pend_sp = 0, pend_id = 0;
  float pend_off[3] = {0.0f, 0.0f, 0.0f}, pend_mom[3] = {0.0f, 0.0f, 0.0f};
  auto store_pending = [&]() {
    if (pend) {
      at32(out.cell, pend_i) = pend_cell;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        at32(out.off[d], pend_i) = pend_off[d];
        at32(out.mom[d], pend_i) = pend_mom[d];
      }
    }
    if constexpr (COPY) {
      if (pend_attr) {
        if (p.species) at32(out.species, pend_i) = (uint8_t)pend_sp;
        if (p.id) at32(out.id, pend_i) = pend_id;
      }
    }
    pend = false;
    pend_attr = false;
  };

  uint32_t lvl = wl.base;
  uint32_t slot = level_slot(wl, 0, lvl);
  uint32_t slot_b = level_slot(wl, 1, lvl);
  // a lane without a particle at a level loads the wave's first particle (a
  // slot of the wave whenever the wave has particles): the loads of a level
  // are then issued in every lane, with no old value to keep across them
  auto valid = [&](int j, uint32_t sl) { return wl.cnt > j ? sl : wl.base; };
  C3Raw nxt;
  uint32_t nxt_si = valid(0, slot), si_b = valid(1, slot_b);
  if (wl.nlev > 0) {
    if constexpr (REBIN) {
      nxt_si = at32(src_index, nxt_si);
      si_b = at32(src_index, si_b);
    }
    c3_load<COPY>(p, nxt_si, nxt);
    // wait for the first particle here (once per thread): otherwise the wait
    // analysis at the loop head, which merges this entry with the back edge,
    // keeps these loads pending there and waits, behind every store of the
    // previous iteration, before the registers are reused
    asm volatile("" ::"v"(nxt.cell), "v"(nxt.species), "v"(nxt.id), "v"(nxt.off[0]), "v"(nxt.off[1]),
                 "v"(nxt.off[2]), "v"(nxt.mom[0]), "v"(nxt.mom[1]), "v"(nxt.mom[2]), "v"(si_b));
  }
  const int nlev = __builtin_amdgcn_readfirstlane(wl.nlev);   // the same in every lane
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int spq_n = 0;   // entries in this wave's queue (wave-uniform)
  // this thread's removals and flags, added to the diagnostics once at the
  // end (no atomics, and no branch around them, in the loop)
  uint32_t n_rem = 0, flags_acc = 0;
  auto spill_drain = [&]() {
    // the entries written by other lanes of this wave are visible: a wave's
    // LDS operations complete in order
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < spq_n) {
      const int code = spq_s[wv][lane];
      float w2[3][3], q2[4];
#pragma unroll
      for (int d = 0; d < 3; ++d) c3_weights(cb.tsc[d], spq_o[wv][d][lane], w2[d]);
#pragma unroll
      for (int k = 0; k < 4; ++k) q2[k] = spq_q[wv][k][lane];
      c3_spill_planes<RX, RY, RC>(dep, spq_r[wv][lane], code % 3 - 1, (code / 3) % 3 - 1, code / 9 - 1, w2, q2);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    spq_n = 0;
  };
  for (int j = 0; j < nlev; ++j) {
    const bool has = wl.cnt > j;
    const uint32_t i = slot;
    const uint32_t si = nxt_si;
    const C3Raw cur = nxt;
    store_pending();
    slot = slot_b;
    nxt_si = si_b;
    slot_b = level_slot(wl, j + 2, lvl);
    // issued at the last level too (the wave's first slot then, in range;
    // the values go unused): with no skipped load, the prefetch registers
    // need no copy of their old values on every iteration
    c3_load<COPY>(p, nxt_si, nxt);
    si_b = valid(j + 2, slot_b);
    if constexpr (REBIN) {
      if (j + 2 < nlev) si_b = at32(src_index, si_b);
    }

    int idx[3] = {mycell[0], mycell[1], mycell[2]};
    const int32_t cid = has ? cur.cell : -1;
    bool live = cid >= cb.cell_base && cid < cb.cell_base + cb.ncell;
    bool deferred = false;
    if constexpr (REBIN) {
      // inputs from the caller (every call starts with a rebinning): cell ids
      // and offsets are checked here; later steps write them in range
      if (cid >= 0 && !live) flags_acc |= DUST_FLAG_BAD_CELL;
      bool bad = false;
#pragma unroll
      for (int d = 0; d < 3; ++d) bad |= live && !(cur.off[d] >= -0.5f && cur.off[d] < 0.5f);
      if (bad) flags_acc |= DUST_FLAG_OFFSET_RANGE;
    }
    if constexpr (COPY) {
      if (has && !live) {
        // a particle without a cell is carried unchanged
        at32(out.cell, i) = cid;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          at32(out.off[d], i) = cur.off[d];
          at32(out.mom[d], i) = cur.mom[d];
        }
      }
    }
    // a lane without a live particle drifts a particle at rest in the centre
    // of its thread's cell (no branch around the drift)
    float off[3], mom[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      off[d] = live ? cur.off[d] : 0.0f;
      mom[d] = live ? cur.mom[d] : 0.0f;
    }
    {
      // after a rebinning every particle is in its thread's cell; on stale
      // bins some lane of a wave nearly always is not: no branch then (a box
      // of fewer than 2^24 cells takes the FP32 division, a uniform choice)
      if constexpr (REBIN) {
        if (live && cid != mycid)
          c3_unravel(cid - cb.cell_base, n0, n1, B.ax[0].inv_n, B.ax[1].inv_n, idx, small);
      } else {
        c3_unravel((live ? cid : mycid) - cb.cell_base, n0, n1, B.ax[0].inv_n, B.ax[1].inv_n, idx, small);
      }
      // half drift to x^{n+1/2} (periodic images, open faces remove, a
      // shear-periodic x face defers); one test for the three axes
      bool removed = false;
#pragma unroll
      for (int d = 0; d < 3; ++d) idx[d] = c3_move(idx[d], off[d], mom[d], cb.hinv[d]);
      if ((unsigned)idx[0] >= (unsigned)n0 || (unsigned)idx[1] >= (unsigned)n1 || (unsigned)idx[2] >= (unsigned)n2) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
          if (idx[d] < 0 || idx[d] >= cb.n[d]) {
            if (cb.per[d]) idx[d] = c3_wrap(idx[d], cb.n[d]);
            else if (d == 0 && cb.shear) deferred = true;
            else removed = true;
          }
        if (removed) {
          // left through an open face: no cell from now on (it keeps the
          // offsets and momenta it had when it left)
          at32(out.cell, i) = -1;
          if (COPY) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              at32(out.off[d], i) = off[d];
              at32(out.mom[d], i) = mom[d];
            }
          }
          ++n_rem;
          live = false;
        }
      }
    }
    // window coordinates (every lane: those without a live particle take
    // their thread's cell below); a stencil that leaves the window defers
    int la = win_coord(idx[0], ox, n0, RX, cb.per[0]);
    int lb = win_coord(idx[1], oy, n1, RY, cb.per[1]);
    int lcz = win_coord(idx[2], oz, n2, RZ, cb.per[2]);
    deferred = live & (deferred | !((la >= 1) & (la <= RX - 2) & (lb >= 1) & (lb <= RY - 2) & (lcz >= 1) &
                                     (lcz <= RZ - 2)));
    {
      const uint64_t dm = __ballot(deferred);
      if (dm) {
        const int lane = threadIdx.x & 63;
        const int leader = __ffsll((unsigned long long)dm) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(defer_count, (uint32_t)__popcll(dm));
        base = __shfl(base, leader, 64);
        if (deferred) {
          defer_list[2 * (base + lanes_below(dm))] = i;
          defer_list[2 * (base + lanes_below(dm)) + 1] = si;
        }
      }
    }
    if (deferred) live = false;
    // a lane without a live particle: a dummy at the centre of this thread's
    // cell, with zero deposits (selects: a divergent skip would keep two
    // copies of the register sums, and a branch costs more than the selects)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      off[d] = live ? off[d] : 0.0f;
      idx[d] = live ? idx[d] : mycell[d];
    }
    la = live ? la : lx + H;
    lb = live ? lb : ly + H;
    lcz = live ? lcz : lz + H;
    // weights at x^{n+1/2}
    float w[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) c3_weights(cb.tsc[d], off[d], w[d]);
    const int sx = la - (lx + H), sy = lb - (ly + H), sz = lcz - (lz + H);
    const bool near = sx >= -1 && sx <= 1 && sy >= -1 && sy <= 1 && sz >= -1 && sz <= 1;
    // gather (Eq. Delta_vp), one z-plane of the stencil at a time: the nine
    // reads of a plane are issued together, and an empty asm with a memory
    // clobber keeps the next plane's reads after this plane's sums
    // (straight-line code would otherwise issue all 27 reads first, 81
    // registers)
    float v[3] = {0.0f, 0.0f, 0.0f};
    {
      const int r00 = win(la, lb - 1, lcz - 1);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int r0 = r00 + c * RX * RY;
        float4 g[9];
#pragma unroll
        for (int q9 = 0; q9 < 9; ++q9) g[q9] = gas[r0 + RX * (q9 / 3) + (q9 % 3) - 1];
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
          const float4 g0 = g[3 * bb], g1 = g[3 * bb + 1], g2 = g[3 * bb + 2];
          const float ux = w[0][0] * g0.x + w[0][1] * g1.x + w[0][2] * g2.x;
          const float uy = w[0][0] * g0.y + w[0][1] * g1.y + w[0][2] * g2.y;
          const float uz = w[0][0] * g0.z + w[0][1] * g1.z + w[0][2] * g2.z;
          const float wbc = w[1][bb] * w[2][c];
          v[0] += wbc * ux;
          v[1] += wbc * uy;
          v[2] += wbc * uz;
        }
        if (c < 2) asm volatile("" ::: "memory");
      }
    }
    // kick (Eq. exp_midpoint; App. B.1 Eq. standard_SB_exp_midpoint)
    int spc = live && p.species ? cur.species : 0;
    flags_acc |= spc >= sp->n ? (uint32_t)DUST_FLAG_BAD_CELL : 0u;
    spc = spc >= sp->n ? 0 : spc;
    const float4 kc = sp_k[spc];
    const float m = kc.x, c = kc.y, h1 = kc.z, dtp = kc.w;
    float dp[3], jj[3];
    if constexpr (SB) {
      // y relative to the background shear: v_y + q Omega x at x^{n+1/2}
      const float2 xr = xres[la];
      const float uy = (mom[1] + xr.x) + fmaf(qOdx, off[0], xr.y);
      const float s0 = v[0] - mom[0], s1 = v[1] - uy, s2 = v[2] - mom[2];
      const float gz = gz_c * (z_lo + (float(idx[2]) + 0.5f + off[2]) * dz);
      const float an0 = 2.0f * Om * uy, an1 = -2.0f * Om * mom[0];
      const float r0 = c * s0 + h1 * an0, r1 = c * s1 + h1 * an1;
      const float2 wk = sp_w[spc];
      const float W = wk.x, den = wk.y;
      dp[0] = (r0 + W * r1) * den;
      dp[1] = (r1 - W * r0) * den;
      dp[2] = c * s2 + h1 * gz;
      const float a0 = an0 + Om * dp[1], a1 = an1 - Om * dp[0];
      jj[0] = c * s0 + dtp * a0;
      jj[1] = c * s1 + dtp * a1;
      jj[2] = c * s2 + dtp * gz;
    } else {
      const float gk[3] = {cg ? g0c : 0.0f, cg ? g1c : 0.0f, cg ? g2c : 0.0f};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float sk = v[k] - mom[k];
        dp[k] = c * sk + h1 * gk[k];
        jj[k] = c * sk + dtp * gk[k];
      }
    }
    float qd[4];
    float e = 0.0f, cells = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float vbar = mom[k] + 0.5f * dp[k];
      e += vbar * jj[k];
      qd[k] = live ? -m * jj[k] : 0.0f;   // deposits carry the minus sign of Eq. dust_feedback_final
      cells = fmaxf(cells, fabsf(vbar) * cb.dtinv[k]);
      mom[k] += dp[k];
    }
    qd[3] = live ? -m * e : 0.0f;
    s_cells = live ? fmaxf(s_cells, cells) : s_cells;
    s_j0 -= qd[0];
    s_j1 -= qd[1];
    s_j2 -= qd[2];
    s_e -= qd[3];
    s_abs += fabsf(qd[0]) + fabsf(qd[1]) + fabsf(qd[2]);
    // deposit (same weights and cells as the gather): register sums over the
    // 27 cells around the thread's cell, the rest through the FP64 window
    {
      const int base = win(la, lb, lcz);
      auto lds_add = [&](int a, int bb, int cc, float wt) {
        const int r0 = base + a + RX * (bb + RY * cc);
#pragma unroll
        for (int k = 0; k < 4; ++k) atomicAdd(&dep[k * RC + r0], double(wt * qd[k]));
      };
      if (live && !near) {
#pragma unroll
        for (int cc = -1; cc <= 1; ++cc)
#pragma unroll
          for (int bb = -1; bb <= 1; ++bb)
#pragma unroll
            for (int a = -1; a <= 1; ++a) lds_add(a, bb, cc, w[0][a + 1] * w[1][bb + 1] * w[2][cc + 1]);
      }
    }
    {
      // weights shifted to this thread's cell (zero where the stencil leaves
      // its 27 cells)
      const int sd[3] = {sx, sy, sz};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float w0 = w[d][0], w1 = w[d][1], w2 = w[d][2];
        w[d][0] = sd[d] == 0 ? w0 : sd[d] < 0 ? w1 : 0.0f;
        w[d][1] = sd[d] == 0 ? w1 : sd[d] < 0 ? w2 : w0;
        w[d][2] = sd[d] == 0 ? w2 : sd[d] < 0 ? 0.0f : w1;
      }
      // the x weight times the deposit (12 products), then one FMA per cell
      // and channel with the y-z weight
      float qf[4], wq[3][4];
#pragma unroll
      for (int k = 0; k < 4; ++k) qf[k] = live && near ? qd[k] : 0.0f;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = 0; k < 4; ++k) wq[a][k] = w[0][a] * qf[k];
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
          const float wbc = w[1][bb] * w[2][cc];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const int oo = a + 3 * (bb + 3 * cc);
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[oo][k] = fmaf(wbc, wq[a][k], acc[oo][k]);
          }
        }
    }
    // a particle one cell off its thread's cell: its outer stencil planes via
    // the wave's queue
    {
      const bool spill = live && near && (sx | sy | sz);
      const uint64_t sm = __ballot(spill);
      const int nnew = __popcll(sm);
      if (nnew) {
        if (spq_n + nnew > 64) spill_drain();
        if (spill) {
          const int e = spq_n + (int)lanes_below(sm);
          spq_r[wv][e] = win(la, lb, lcz);
          spq_s[wv][e] = (sx + 1) + 3 * ((sy + 1) + 3 * (sz + 1));
#pragma unroll
          for (int d = 0; d < 3; ++d) spq_o[wv][d][e] = off[d];
#pragma unroll
          for (int k = 0; k < 4; ++k) spq_q[wv][k][e] = qd[k];
        }
        spq_n += nnew;
      }
    }
    // second half drift to x^{n+1} (a lane without a live particle: its
    // dummy at rest, no branch around the drift)
    {
      bool alive = true;
#pragma unroll
      for (int d = 0; d < 3; ++d) idx[d] = c3_move(idx[d], off[d], live ? mom[d] : 0.0f, cb.hinv[d]);
      if ((unsigned)idx[0] >= (unsigned)n0 || (unsigned)idx[1] >= (unsigned)n1 || (unsigned)idx[2] >= (unsigned)n2) {
        if (cb.shear && (idx[0] < 0 || idx[0] >= n0)) shear_image<float, false>(B, f, t0 + double(dt), idx, off, mom);
#pragma unroll
        for (int d = 0; d < 3; ++d)
          if (idx[d] < 0 || idx[d] >= cb.n[d]) {
            if (cb.per[d] || (d == 0 && cb.shear)) idx[d] = c3_wrap(idx[d], cb.n[d]);
            else alive = false;
          }
      }
      pend = live;
      const int32_t ncid = c3_cell_id(cb, idx[0], idx[1], idx[2], small);
      pend_cell = alive ? ncid : -1;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        pend_off[d] = off[d];
        pend_mom[d] = mom[d];
      }
      n_rem += live && !alive ? 1u : 0u;
    }
    pend_i = i;
    if constexpr (COPY) {
      if (has && !deferred) {
        pend_attr = true;
        pend_sp = cur.species;
        pend_id = cur.id;
      }
    }
  }
  store_pending();
  if (spq_n) spill_drain();
  if (dg) {
    if (n_rem) {
      atomicAdd(&dg->n_removed, (unsigned long long)n_rem);
      flags_acc |= DUST_FLAG_LEFT_OPEN;
    }
    if (flags_acc) atomicOr(&dg->flags, (unsigned)flags_acc);
  }

  // register sums of my cell's stencil -> deposit window
  if (own) {
#pragma unroll
    for (int cc = -1; cc <= 1; ++cc)
#pragma unroll
      for (int bb = -1; bb <= 1; ++bb)
#pragma unroll
        for (int a = -1; a <= 1; ++a) {
          const int oo = (a + 1) + 3 * ((bb + 1) + 3 * (cc + 1));
          const int r0 = mybase + a + RX * (bb + RY * cc);
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (acc[oo][k] != 0.0f) atomicAdd(&dep[k * RC + r0], double(acc[oo][k]));
        }
  }
  __syncthreads();
  // the deposit window to the grid (periodic images to their cells; uniform
  // cell volume)
  const double iv = inv_volume(B, 0, 0, 0);
  for (int r = threadIdx.x; r < RC; r += FUSED_THREADS) {
    const int a = r % RX, bq = (r / RX) % RY, cq = r / (RX * RY);
    int i = ox + a, j = oy + bq, k = oz + cq;
    if (cb.per[0]) i = wrap_index(i, n0);
    if (cb.per[1]) j = wrap_index(j, n1);
    if (cb.per[2]) k = wrap_index(k, n2);
    const bool in = i >= -1 && i <= n0 && j >= -1 && j <= n1 && k >= -1 && k <= n2;
    if (!in) continue;
    const int64_t id = stored_index(B, i, j, k);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const double x = dep[m * RC + r];
      if (x != 0.0) unsafeAtomicAdd(&fl.dep[m][id], float(x * iv));
    }
  }
  // diagnostics: the workgroup's FP64 sums to its own slot of `part`
  if (dg) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double s[6] = {double(s_j0), double(s_j1), double(s_j2), double(s_e), double(s_abs), double(s_cells)};
    if (sums) {
#pragma unroll
      for (int k = 0; k < 5; ++k) s[k] = wave_sum(s[k]);
      s[5] = wave_max(s[5]);
    }
    __shared__ double red[FUSED_THREADS / 64][PART_WORDS];
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < 6; ++k) red[wave][k] = s[k];
      red[wave][6] = 0.0;
      red[wave][7] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x < PART_WORDS) {
      const int k = threadIdx.x;
      double vv = red[0][k];
      for (int w2 = 1; w2 < FUSED_THREADS / 64; ++w2) vv = k == 5 ? fmax(vv, red[w2][k]) : vv + red[w2][k];
      part[(size_t)blockIdx.x * PART_WORDS + k] = sums || k >= 6 ? vv : 0.0;
    }
  }
}

template <int TX, int TY, int TZ, bool SB, bool REBIN, bool COPY, bool SMALL>
void launch_c3_t(const FusedPlan& plan, const PView<float>& p, const PView<float>& q, const Box* boxes_d,
                 const FView<float>& fl, const Forces& f, const Species* sp, int drag_mode, double dt,
                 const double* tdev, const int64_t* bin_start, const double* xg, DiagDev* dg, bool sums,
                 const uint32_t* src_index, hipStream_t st) {
  const size_t lds = c3_lds_bytes(plan);
  auto kern = k_c3<TX, TY, TZ, SB, REBIN, COPY, SMALL>;
  if (lds > 64 * 1024) {
    static bool raised = false;
    if (!raised) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      raised = true;
    }
  }
  hipLaunchKernelGGL(kern, dim3(plan.ntiles), dim3(FUSED_THREADS), lds, st, plan.tiles_d, plan.tile_map, p, q,
                     COPY ? 1 : 0, boxes_d, fl, f, sp, drag_mode, float(dt), tdev, bin_start, xg, dg,
                     plan.part_d, (int)sums, plan.defer_list, plan.defer_count, src_index);
}

// The tile kernel of one tile shape: forces (standard shearing box or not)
// and the kind of step (after a rebinning through src_index; stale bins
// written across with copy_attrs; stale bins in place).
template <int TX, int TY, int TZ>
void launch_c3_shape(const FusedPlan& plan, const PView<float>& p, const PView<float>& q, bool copy_attrs,
                     const Box* boxes_d, const FView<float>& fl, const Forces& f, const Species* sp,
                     int drag_mode, double dt, const double* tdev, const int64_t* bin_start, const double* xg,
                     DiagDev* dg, bool sums, const uint32_t* src_index, hipStream_t st) {
#define DUST_C3M(SBV, RB, CP)                                                                               \
  do {                                                                                                      \
    if (plan.small)                                                                                         \
      launch_c3_t<TX, TY, TZ, SBV, RB, CP, true>(plan, p, q, boxes_d, fl, f, sp, drag_mode, dt, tdev,       \
                                                 bin_start, xg, dg, sums, src_index, st);                   \
    else                                                                                                    \
      launch_c3_t<TX, TY, TZ, SBV, RB, CP, false>(plan, p, q, boxes_d, fl, f, sp, drag_mode, dt, tdev,      \
                                                  bin_start, xg, dg, sums, src_index, st);                  \
  } while (0)
  const bool sb = f.kind == FORCE_SHEARBOX;
  if (src_index) {
    if (sb) DUST_C3M(true, true, true);
    else DUST_C3M(false, true, true);
  } else if (copy_attrs) {
    if (sb) DUST_C3M(true, false, true);
    else DUST_C3M(false, false, true);
  } else {
    if (sb) DUST_C3M(true, false, false);
    else DUST_C3M(false, false, false);
  }
#undef DUST_C3M
}

#define DUST_C3_SHAPE_DECL(PREFIX, TX, TY, TZ)                                                              \
  PREFIX template void launch_c3_shape<TX, TY, TZ>(                                                         \
      const FusedPlan&, const PView<float>&, const PView<float>&, bool, const Box*, const FView<float>&,     \
      const Forces&, const Species*, int, double, const double*, const int64_t*, const double*, DiagDev*,   \
      bool, const uint32_t*, hipStream_t);
#define DUST_C3_SHAPES(PREFIX)                                                                              \
  DUST_C3_SHAPE_DECL(PREFIX, 8, 8, 4)                                                                       \
  DUST_C3_SHAPE_DECL(PREFIX, 16, 4, 4)                                                                      \
  DUST_C3_SHAPE_DECL(PREFIX, 4, 16, 4)                                                                      \
  DUST_C3_SHAPE_DECL(PREFIX, 4, 4, 16)                                                                      \
  DUST_C3_SHAPE_DECL(PREFIX, 8, 4, 8)                                                                       \
  DUST_C3_SHAPE_DECL(PREFIX, 4, 8, 8)


}  // namespace dust
