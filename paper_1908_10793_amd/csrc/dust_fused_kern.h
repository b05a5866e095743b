// Fused gather - exponential-midpoint push - deposit kernel (gfx950).
//
// One workgroup per grid tile of 256 cells and one thread per cell.  The
// particles are binned tile by tile (tile-major keys of the cell each reaches
// in the first half drift); the particles of a wave's cells occupy one range
// of slots, level-major (iteration j of the wave touches consecutive slots).
// The workgroup stages the gas velocity of the tile plus a two-cell halo in
// LDS (one 4-vector of the storage type per cell; periodic images beyond the
// box along periodic axes).  For every particle the thread does the half
// drift, the weights at x^{n+1/2}, the gather from LDS, the kick, the drag
// impulse and energy, the second half drift and the store.  Deposits are
// summed in registers over the 27 cells around the thread's cell: fully for
// a particle in that cell, through weights shifted to it for a particle in a
// neighbouring cell (the stencil planes outside go to an FP64 LDS window with
// atomics, which gfx950 executes about twenty times faster than FP32 ones);
// the sums go to the window once per thread.  The window is then added to the
// global deposit arrays with one atomic per touched cell and channel, scaled
// by the inverse cell volume.  A particle whose stencil at x^{n+1/2} leaves
// the window (it moved more than one cell beyond its tile since the binning,
// or crossed a shear-periodic face) is stepped by a second kernel against
// global memory.
// Kernels of the fused tile step (gfx950): the tile kernel, the
// deferred-particle kernel and their launchers, templated on storage and
// arithmetic types, geometry, dimension, uniformity and tile shape.  The
// launchers are instantiated in several translation units (dust_fused_i_*.hip)
// so that the library builds in parallel; dust_fused.hip holds the plan, the
// dispatcher and the rebinning kernels.
#pragma once

#include <algorithm>

#include "dust_device.h"
#include "dust_fused.h"
#include "dust_launch.h"
#include "dust_particle.h"

namespace dust {

static constexpr int FUSED_THREADS = 256;
static constexpr int PART_WORDS = 8;   // per-workgroup diagnostic partials
static constexpr int DEFER_BLOCKS = 256;  // workgroups of the deferred-particle kernel
static constexpr int FUSED_HALO = 2;

template <typename T> struct Vec4;
template <> struct Vec4<float> {
  using type = float4;
  static __device__ __forceinline__ float4 make(float a, float b, float c, float d) {
    return make_float4(a, b, c, d);
  }
};
template <> struct Vec4<double> {
  using type = double4;
  static __device__ __forceinline__ double4 make(double a, double b, double c, double d) {
    return make_double4(a, b, c, d);
  }
};

// Level-major layout of the particles of one wave's cells.  The cells of a
// wave are consecutive tile-major keys (a wave covers whole rows or layers of
// its tile), so their particles occupy one range [base, base + total) of
// slots.  Level j of the range holds the j-th particle of every cell that has
// more than j, in lane order; the slot of lane l in level j is the level's
// start plus the number of lower lanes whose cells have more than j.
// Periodic axes in the tile window: the window holds the periodic images of
// the cells beyond the box (not the ghost layer), and a particle that
// crossed a periodic face since the binning is placed at its image next to
// the window, so it stays with its tile.  win_coord: window coordinate of
// cell i along an axis whose window starts at o (R cells), the periodic
// image inside the window's interior [1, R-2] when one lies within a box
// length (a particle further away is deferred).
__device__ __forceinline__ int win_coord(int i, int o, int n, int R, bool periodic) {
  int l = i - o;
  if (periodic) l += l < 1 ? n : l > R - 2 ? -n : 0;
  return l;
}
__device__ __forceinline__ int wrap_index(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}
__device__ __forceinline__ bool axis_periodic(const Axis& ax) {
  return ax.bc_lo == BC_PERIODIC && ax.bc_hi == BC_PERIODIC;
}

// Set bits of a wave mask in the lanes below this one.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

struct WaveLevels {
  int cnt;          // particles of this lane's cell
  int nlev;         // largest count in the wave
  uint32_t base;    // first slot of the wave's range (counts are below 2^31)
};

__device__ __forceinline__ WaveLevels wave_levels(int cnt, int64_t start) {
  WaveLevels w;
  w.cnt = cnt;
  w.nlev = wave_max(cnt);
  const uint64_t any = __ballot(cnt > 0);
  // the first lane with particles has the smallest start of the range
  w.base = any ? (uint32_t)__shfl(start, __ffsll((unsigned long long)any) - 1, 64) : 0u;
  return w;
}

// Slot of this lane's particle of level j; lvl: start of level j on entry,
// of level j+1 on return (call once per level, in order, in every lane).
__device__ __forceinline__ uint32_t level_slot(const WaveLevels& w, int j, uint32_t& lvl) {
  const uint64_t m = __ballot(w.cnt > j);
  const uint32_t s = lvl + lanes_below(m);
  lvl += (uint32_t)__popcll(m);
  return s;
}

// Raw stored state of one particle (prefetched one particle ahead), with the
// attributes the kick reads (species, mass, drag: each only if present) and,
// when the attributes are copied to another buffer, the id: no load of the
// loop's body waits on memory.
template <typename TS> struct Raw {
  int32_t cell;
  TS off[3], mom[3];
  int32_t species, id;
  TS mass, drag;
};

template <typename TS, int NDIM, int NC>
__device__ __forceinline__ void load_raw(const PView<TS>& p, int64_t i, Raw<TS>& r, bool with_id) {
  r.id = with_id && p.id ? p.id[i] : 0;
  r.cell = p.cell[i];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    r.off[d] = d < NDIM ? p.off[d][i] : TS(0);
    r.mom[d] = d < NC ? p.mom[d][i] : TS(0);
  }
  r.species = p.species ? (int32_t)p.species[i] : 0;
  r.mass = p.mass ? p.mass[i] : TS(0);
  r.drag = p.drag ? p.drag[i] : TS(1);
}

// Register budget: the FP32 kernel needs about 250 VGPRs (108 of them the
// register sums); the compiler keeps the standard-form shapes but one under
// 256 (2 waves/SIMD) by itself, and 4x4x16, the orbital-advection and the
// curvilinear kernels (whose slip form carries two-word scale factors) with
// an explicit target (an explicit target where it is not needed costs time:
// about 25 us of 900).
template <typename A, typename TS, int GEOM, int TX, int TY, bool FG>
constexpr int fused_waves_target() {
  return sizeof(A) == 4 && sizeof(TS) == 4 && (FG || TX * TY <= 16 || GEOM != GEOM_CART) ? 2 : 1;
}

template <typename TS, typename A, int GEOM, int NDIM, bool U, int TX, int TY, int TZ, bool FG>
__global__ void __launch_bounds__(FUSED_THREADS)
    __attribute__((amdgpu_waves_per_eu(fused_waves_target<A, TS, GEOM, TX, TY, FG>())))
    k_fused(const TileDesc* __restrict__ tiles, PView<TS> p, PView<TS> dst, int copy_attrs,
            const Box* __restrict__ boxes, FView<TS> fl, Forces f, const Species* __restrict__ sp,
            int drag_mode, A dt, const double* __restrict__ tdev,
            const int64_t* __restrict__ bin_start, const double* __restrict__ xg, DiagDev* dg,
            double* __restrict__ part, int sums, uint32_t* __restrict__ defer_list,
            uint32_t* __restrict__ defer_count, const uint32_t* __restrict__ src_index) {
  // The descriptors (tiles, boxes, species, time, bin starts) are read-only
  // and never aliased by the particle and field arrays: __restrict__ lets
  // their fields stay in scalar registers / the scalar cache, so the loop's
  // waits on particle loads do not also wait on descriptor reloads.
  // p: particles read; dst: where the updated particles are written, in the
  // binned (level-major) slot order.  Slot i reads particle src_index[i] of
  // p (right after a rebinning, dst != p), or particle i (src_index null, in
  // place).  copy_attrs copies the attributes the step does not change.
  // FG: the forces are the orbital-advection shearing box (kernels of their
  // own, so that neither form's code costs the other registers)
  constexpr int nc = GEOM == GEOM_CART ? NDIM : 3;
  constexpr int c2 = NDIM > 2 ? 1 : 0;
  constexpr int H = FUSED_HALO;
  constexpr int HZ = NDIM > 2 ? H : 0;
  constexpr int RX = TX + 2 * H, RY = TY + 2 * H, RZ = TZ + 2 * HZ;
  constexpr int RC = RX * RY * RZ;
  using G4 = typename Vec4<TS>::type;
  extern __shared__ double smem[];
  double* dep = smem;                                                    // (nc+1) * RC
  G4* gas = reinterpret_cast<G4*>(smem + ((RC * (nc + 1) + 3) & ~3));   // RC cells
  // per-species drag propagator and mass (species mode: tau depends only on
  // the species, so c and psi of Eq. phi1 are computed once per workgroup)
  __shared__ A sp_c[DUST_MAX_SPECIES], sp_psi[DUST_MAX_SPECIES], sp_m[DUST_MAX_SPECIES];
  const TileDesc td = tiles[blockIdx.x];
  const Box& B = boxes[td.box];
  const int ox = td.i0 - H, oy = td.j0 - H, oz = td.k0 - HZ;  // window origin
  if (threadIdx.x < sp->n) {
    A c, psi;
    propagator<A>(dt * A(sp->inv_tau[threadIdx.x]), c, psi);
    sp_c[threadIdx.x] = c;
    sp_psi[threadIdx.x] = psi;
    sp_m[threadIdx.x] = A(sp->mass[threadIdx.x]);
  }
  const double t0 = *tdev;
  const A h = A(0.5) * dt;
  const int n0 = B.ax[0].n, n1 = B.ax[1].n, n2 = NDIM > 2 ? B.ax[2].n : 1;

  const bool per0 = axis_periodic(B.ax[0]), per1 = axis_periodic(B.ax[1]);
  const bool per2 = NDIM > 2 && axis_periodic(B.ax[2]);
  // stage the gas window (periodic images beyond the box), clear the deposit window
  for (int r = threadIdx.x; r < RC; r += FUSED_THREADS) {
    int a = r % RX, bq = (r / RX) % RY, cq = r / (RX * RY);
    int i = ox + a, j = oy + bq, k = oz + cq;
    if (per0) i = wrap_index(i, n0);
    if (per1) j = wrap_index(j, n1);
    if (per2) k = wrap_index(k, n2);
    bool in = i >= -1 && i <= n0 && j >= -1 && j <= n1 && (NDIM < 3 || (k >= -1 && k <= n2));
    int64_t id = in ? stored_index(B, i, j, k) : 0;
    TS gv[3] = {TS(0), TS(0), TS(0)};
    TS lo = TS(0);
    if (in && xg && B.xg_base >= 0 && (i < 0 || i >= n0)) {
      // x ghost of a shear-periodic box: the FP64 ghost value, its y
      // component (which carries the shear boost) as a sum of two words
#pragma unroll
      for (int m = 0; m < nc; ++m) {
        const double v = gas_comp(B, fl, xg, m, i, j, k);
        gv[m] = TS(v);
        if (m == 1) lo = TS(v - double(gv[m]));
      }
    } else if (in) {
#pragma unroll
      for (int m = 0; m < nc; ++m) gv[m] = fl.vel[m][id];
    }
    gas[r] = Vec4<TS>::make(gv[0], gv[1], gv[2], lo);
#pragma unroll
    for (int m = 0; m <= nc; ++m) dep[m * RC + r] = 0.0;
  }
  __syncthreads();

  // this thread's cell
  const int lx = threadIdx.x % TX, ly = (threadIdx.x / TX) % TY, lz = threadIdx.x / (TX * TY);
  const bool own = lx < td.ex && ly < td.ey && lz < td.ez;
  const int mycell[3] = {td.i0 + lx, td.j0 + ly, td.k0 + lz};
  const int mybase = (lx + H) + RX * ((ly + H) + RY * (lz + HZ));  // window index of my cell
  const int32_t mycid = (int32_t)(B.cell_base + ravel(B, mycell));
  int64_t ps = 0, pe = 0;
  if (own) {
    int64_t key = td.key0 + lx + (int64_t)td.ex * (ly + (int64_t)td.ey * lz);
    ps = bin_start[key];
    pe = bin_start[key + 1];
  }
  // register sums: FP32 for FP32 storage, FP64 for FP64 storage
  using TAcc = TS;
  constexpr int NS = c2 ? 27 : 9;   // stencil cells
  TAcc acc[NS][nc + 1];
#pragma unroll
  for (int o = 0; o < NS; ++o)
#pragma unroll
    for (int k = 0; k <= nc; ++k) acc[o][k] = TAcc(0);
  // FP64 diagnostic sums of this thread (impulse, energy, |impulse|): kept
  // in LDS, each thread its own words, rather than in registers, which the
  // register sums need
  __shared__ double dsum[5][FUSED_THREADS];
  static_assert(FUSED_THREADS <= 256, "static LDS bound");
#pragma unroll
  for (int k = 0; k < 5; ++k) dsum[k][threadIdx.x] = 0.0;
  A a_cells = A(0);
  unsigned long long n_fb = 0;

  // Particle layout of a wave's cells (level-major, see level_slot): in
  // iteration j every lane whose cell has more than j particles takes its
  // cell's j-th particle, and those particles are consecutive slots, so the
  // loads and stores of an iteration are contiguous.
  const WaveLevels wl = wave_levels(own ? (int)(pe - ps) : 0, ps);
  // The particle state is loaded one level ahead of its use, its source
  // index (after a rebinning) two levels ahead.
  uint32_t lvl = wl.base;
  uint32_t slot = level_slot(wl, 0, lvl);
  uint32_t slot_b = level_slot(wl, 1, lvl);
  Raw<TS> nxt;
  uint32_t nxt_si = 0, si_b = slot_b;
  if (wl.cnt > 0) {
    nxt_si = src_index ? src_index[slot] : slot;
    load_raw<TS, NDIM, nc>(p, nxt_si, nxt, copy_attrs);
  }
  if (src_index && wl.cnt > 1) si_b = src_index[slot_b];
  // this thread's flags, raised once after the loop (no atomics in it)
  uint32_t flags_acc = 0;
  for (int j = 0; j < wl.nlev; ++j) {
    const bool has = wl.cnt > j;
    const uint32_t i = slot;       // slot written
    const uint32_t si = nxt_si;    // particle read
    const Raw<TS> cur = nxt;
    slot = slot_b;
    nxt_si = si_b;
    slot_b = level_slot(wl, j + 2, lvl);
    if (wl.cnt > j + 1) load_raw<TS, NDIM, nc>(p, nxt_si, nxt, copy_attrs);   // next particle
    si_b = slot_b;
    if (src_index && wl.cnt > j + 2) si_b = src_index[slot_b];               // and the index after
    // Lanes of one wave walk different cells, so nothing below branches
    // around the register sums: a particle without a cell, or one that left
    // through an open face, continues as a dummy at the centre of this
    // thread's cell with zero deposits (a divergent skip would keep two
    // copies of every register sum live).
    int idx[3] = {mycell[0], mycell[1], mycell[2]};
    A off[3] = {A(0), A(0), A(0)}, mom[3] = {A(0), A(0), A(0)};
    const int32_t cid = has ? cur.cell : -1;
    bool live = cid >= 0 && cid >= B.cell_base && cid < B.cell_base + B.ncell;
    bool removed = false;
    flags_acc |= cid >= 0 && !live ? (uint32_t)DUST_FLAG_BAD_CELL : 0u;
    if (live) {
      if (cid != mycid) unravel(B, cid - B.cell_base, idx);
      bool bad = false;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        off[d] = A(cur.off[d]);
        mom[d] = A(cur.mom[d]);
        bad |= !(off[d] >= A(-0.5) && off[d] < A(0.5));
      }
      flags_acc |= bad ? (uint32_t)DUST_FLAG_OFFSET_RANGE : 0u;
      // half drift to x^{n+1/2}
      if (!drift<A, GEOM, NDIM, U, FG>(B, f, true, h, t0 + double(h), idx, off, mom)) {
        store_particle<TS, A, GEOM, NDIM, FG>(dst, B, f, t0 + double(h), i, false, idx, off, mom, dg);
        live = false;
        removed = true;
      }
    }
    // A particle whose stencil leaves the window (it moved more than a cell
    // since the binning, or wrapped across a periodic face) is left to the
    // deferred kernel, which does its step against global memory; here it
    // continues as a dummy.
    // window coordinates (every lane; a dummy takes this thread's cell below)
    int la = win_coord(idx[0], ox, n0, RX, per0);
    int lb = win_coord(idx[1], oy, n1, RY, per1);
    int lc = c2 ? win_coord(idx[2], oz, n2, RZ, per2) : 0;
    const bool deferred = live & !((la >= 1) & (la <= RX - 2) & (lb >= 1) & (lb <= RY - 2) &
                                   ((c2 == 0) | ((lc >= 1) & (lc <= RZ - 2))));
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
    // the dummy by selects (a branch around them costs more)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      idx[d] = live ? idx[d] : mycell[d];
      off[d] = live ? off[d] : A(0);
      mom[d] = live ? mom[d] : A(0);
    }
    la = live ? la : lx + H;
    lb = live ? lb : ly + H;
    lc = live ? lc : (c2 ? lz + HZ : 0);
    // weights at x^{n+1/2}
    Stencil<A> s;
    stencil_weights<A, GEOM, NDIM, U>(B, idx, off, s);
    constexpr bool AZ = az_gather<A, GEOM>();
    constexpr int PHI = az_comp<GEOM>();
    double wr[3] = {0.0, 0.0, 0.0};
    if constexpr (AZ) radial_weights64<A, GEOM, U>(B, idx[0], off[0], s, wr);
    // cell of the particle relative to this thread's cell
    const int sx = la - (lx + H), sy = lb - (ly + H), sz = c2 ? lc - (lz + HZ) : 0;
    const bool near = sx >= -1 && sx <= 1 && sy >= -1 && sy <= 1 && sz >= -1 && sz <= 1;
    // Gather (Eq. Delta_vp) in slip form: the weights sum to one, so the
    // slip p_g - p is sc * sum_i W_i (v_i - u) with u = p / sc the particle's
    // physical velocity.  Each v_i - u is exact or nearly so when the gas
    // and particle velocities are close (FP32 keeps the slip's relative
    // accuracy where the velocities themselves are large, as in the
    // shearing box's background shear).
    Where<A> wh;
    where<A, GEOM, NDIM, U>(B, idx, off, wh);
    SlipScale<A> ss;
    slip_scale<A, GEOM, NDIM, U>(B, idx, off, mom, wh, ss);
    const A* up = ss.up;
    A v[3] = {A(0), A(0), A(0)};
    double vaz = 0.0;   // azimuthal component in FP64 (AZ)
    // (always true here; kept as a branch, which bounds how far the compiler
    // hoists the window reads and so the register use)
    if (la >= 1) {
      const int base = la + RX * (lb + RY * lc);
#pragma unroll
      for (int c = -c2; c <= c2; ++c)
#pragma unroll
        for (int bb = -1; bb <= 1; ++bb) {
          const int r0 = base + RX * (bb + RY * c);
          A u[3] = {A(0), A(0), A(0)};
          double uaz = 0.0;
#pragma unroll
          for (int a = -1; a <= 1; ++a) {
            const G4 g = gas[r0 + a];
            const TS gv[3] = {g.x, g.y, g.z};
#pragma unroll
            for (int m = 0; m < nc; ++m) u[m] += s.w[0][a + 1] * (A(gv[m]) - up[m]);
            if (nc > 1) u[1] += s.w[0][a + 1] * A(g.w);   // low word (shear x ghosts only)
            if constexpr (AZ) uaz += wr[a + 1] * (double(gv[PHI]) - double(up[PHI]));
          }
          const A wbc = s.w[1][bb + 1] * s.w[2][c + 1];
#pragma unroll
          for (int m = 0; m < nc; ++m) v[m] += wbc * u[m];
          if constexpr (AZ) vaz += (double(s.w[1][bb + 1]) * double(s.w[2][c + 1])) * uaz;
        }
    }
    if constexpr (AZ) v[PHI] = A(vaz);   // (the FP32 sum of that component is dropped)
    // kick
    A sl[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) sl[m] = m < nc ? slip_canonical<A, GEOM>(ss, m, v[m]) : A(0);
    int spc = live ? cur.species : 0;
    flags_acc |= spc >= sp->n ? (uint32_t)DUST_FLAG_BAD_CELL : 0u;
    spc = spc >= sp->n ? 0 : spc;
    A m = p.mass && live ? A(cur.mass) : sp_m[spc];
    A c, psi;
    if (drag_mode == DRAG_SPECIES) {
      c = sp_c[spc];
      psi = sp_psi[spc];
    } else {
      A it = inverse_tau<A, GEOM>(f, drag_mode, live ? A(cur.drag) : A(1), A(0), wh);
      propagator<A>(dt * it, c, psi);
    }
    KickOut<A> o;
    kick<A, GEOM, NDIM, FG>(B, f, dt, c, psi, wh, mom, sl, o);
    A q[4] = {A(0), A(0), A(0), A(0)};
#pragma unroll
    for (int k = 0; k < nc; ++k) {
      q[k] = live ? -m * o.j[k] : A(0);  // deposits carry the minus sign of Eq. dust_feedback_final
      if (sums && live) {
        A cps;
        if constexpr (GEOM == GEOM_CART && U) {
          cps = fabs((mom[k] + A(0.5) * o.dp[k]) * dt * A(B.ax[k].inv_d));
        } else {
          A vbar = (mom[k] + A(0.5) * o.dp[k]) / wh.sc[k];
          A dl = cell_width<A, U>(B.ax[k], idx[k]) * (GEOM == GEOM_CART || k == 0 ? A(1) : wh.sc[k]);
          cps = fabs(vbar * dt / dl);
        }
        a_cells = cps > a_cells ? cps : a_cells;
      }
      mom[k] += o.dp[k];
    }
    q[nc] = live ? -m * o.e : A(0);
    if (sums && live) {
      double ab = 0.0;
#pragma unroll
      for (int k = 0; k < nc; ++k) {
        atomicAdd(&dsum[k][threadIdx.x], -double(q[k]));
        ab += fabs(double(q[k]));
      }
      atomicAdd(&dsum[3][threadIdx.x], -double(q[nc]));
      atomicAdd(&dsum[4][threadIdx.x], ab);
    }
    // Deposit (same weights and cells as the gather).  The register sums
    // cover the 27 cells around this thread's cell.  A particle in that cell
    // or a neighbour (sx, sy, sz in -1..1) adds the part of its stencil that
    // falls inside them to the register sums, through its weights shifted by
    // (sx, sy, sz); the rest, one 3x3 plane per axis it moved along, goes to
    // the window with FP64 LDS atomics.  A particle further away (stale bins)
    // deposits its whole stencil with LDS atomics.
    {
      const int base = la + RX * (lb + RY * lc);
      auto lds_add = [&](int a, int bb, int c, double w) {
        const int r0 = base + a + RX * (bb + RY * c);
#pragma unroll
        for (int k = 0; k <= nc; ++k) atomicAdd(&dep[k * RC + r0], w * double(q[k]));
      };
      if (live && !near) {
#pragma unroll
        for (int c = -c2; c <= c2; ++c)
#pragma unroll
          for (int bb = -1; bb <= 1; ++bb) {
            const double wbc = double(s.w[1][bb + 1] * s.w[2][c + 1]);
#pragma unroll
            for (int a = -1; a <= 1; ++a) lds_add(a, bb, c, double(s.w[0][a + 1]) * wbc);
          }
      }
      // spill planes: particle-relative row sy (all a, c); column sx (rows
      // other than sy); layer sz (the cells in neither)
      if (live && near && sy != 0) {
        const A wy = sy > 0 ? s.w[1][2] : s.w[1][0];
#pragma unroll
        for (int c = -c2; c <= c2; ++c)
#pragma unroll
          for (int a = -1; a <= 1; ++a) lds_add(a, sy, c, double(s.w[0][a + 1] * wy * s.w[2][c + 1]));
      }
      if (live && near && sx != 0) {
        const A wx = sx > 0 ? s.w[0][2] : s.w[0][0];
#pragma unroll
        for (int c = -c2; c <= c2; ++c)
#pragma unroll
          for (int bb = -1; bb <= 1; ++bb)
            if (sy == 0 || bb != sy) lds_add(sx, bb, c, double(wx * s.w[1][bb + 1] * s.w[2][c + 1]));
      }
      if (c2 && live && near && sz != 0) {
        const A wz = sz > 0 ? s.w[2][2] : s.w[2][0];
#pragma unroll
        for (int bb = -1; bb <= 1; ++bb)
#pragma unroll
          for (int a = -1; a <= 1; ++a)
            if ((sy == 0 || bb != sy) && (sx == 0 || a != sx))
              lds_add(a, bb, sz, double(s.w[0][a + 1] * s.w[1][bb + 1] * wz));
      }
    }
    {
      // weights shifted to this thread's cell (zero where the stencil leaves
      // its 27 cells), in place: w'[m] = w[m - s]
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int sd = d == 0 ? sx : d == 1 ? sy : sz;
        const A w0 = s.w[d][0], w1 = s.w[d][1], w2 = s.w[d][2];
        s.w[d][0] = sd == 0 ? w0 : sd < 0 ? w1 : A(0);
        s.w[d][1] = sd == 0 ? w1 : sd < 0 ? w2 : w0;
        s.w[d][2] = sd == 0 ? w2 : sd < 0 ? A(0) : w1;
      }
      TAcc qf[4], wa[3];
#pragma unroll
      for (int k = 0; k <= nc; ++k) qf[k] = live && near ? TAcc(q[k]) : TAcc(0);
#pragma unroll
      for (int a = 0; a < 3; ++a) wa[a] = TAcc(s.w[0][a]);
#pragma unroll
      for (int c = -c2; c <= c2; ++c)
#pragma unroll
        for (int bb = -1; bb <= 1; ++bb) {
          TAcc wbc = TAcc(s.w[1][bb + 1] * s.w[2][c + 1]);
          TAcc qb[4];
#pragma unroll
          for (int k = 0; k <= nc; ++k) qb[k] = wbc * qf[k];
#pragma unroll
          for (int a = -1; a <= 1; ++a) {
            const int oo = (a + 1) + 3 * ((bb + 1) + 3 * (c + c2));
#pragma unroll
            for (int k = 0; k <= nc; ++k) acc[oo][k] += wa[a + 1] * qb[k];
          }
        }
    }
    // second half drift to x^{n+1}
    if (live) {
      bool alive = drift<A, GEOM, NDIM, U, FG>(B, f, false, h, t0 + double(dt), idx, off, mom);
      store_particle<TS, A, GEOM, NDIM, FG>(dst, B, f, t0 + double(dt), i, alive, idx, off, mom, dg);
    }
    if (copy_attrs && has && !deferred) {
      if (!live) {
        // removed or cell-less particles keep their last offsets and momenta
        if (!removed) dst.cell[i] = cid;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          if (d < NDIM) dst.off[d][i] = cur.off[d];
          if (d < nc) dst.mom[d][i] = cur.mom[d];
        }
      }
      if (p.drag) dst.drag[i] = cur.drag;
      if (p.mass) dst.mass[i] = cur.mass;
      if (p.species) dst.species[i] = (uint8_t)cur.species;
      if (p.id) dst.id[i] = cur.id;
    }
  }

  if (dg && flags_acc) atomicOr(&dg->flags, (unsigned)flags_acc);
  // register sums of my cell's stencil -> deposit window
  if (own) {
#pragma unroll
    for (int c = -c2; c <= c2; ++c)
#pragma unroll
      for (int bb = -1; bb <= 1; ++bb)
#pragma unroll
        for (int a = -1; a <= 1; ++a) {
          const int oo = (a + 1) + 3 * ((bb + 1) + 3 * (c + c2));
          const int r0 = mybase + a + RX * (bb + RY * c);
#pragma unroll
          for (int k = 0; k <= nc; ++k)
            if (acc[oo][k] != TAcc(0)) atomicAdd(&dep[k * RC + r0], double(acc[oo][k]));
        }
  }
  __syncthreads();

  // add the deposit window to the grid (periodic images to their cells)
  for (int r = threadIdx.x; r < RC; r += FUSED_THREADS) {
    int a = r % RX, bq = (r / RX) % RY, cq = r / (RX * RY);
    int i = ox + a, j = oy + bq, k = oz + cq;
    if (per0) i = wrap_index(i, n0);
    if (per1) j = wrap_index(j, n1);
    if (per2) k = wrap_index(k, n2);
    bool in = i >= -1 && i <= n0 && j >= -1 && j <= n1 && (NDIM < 3 || (k >= -1 && k <= n2));
    if (!in) continue;
    int64_t id = stored_index(B, i, j, k);
    double iv = inv_volume(B, i, j, k);
#pragma unroll
    for (int m = 0; m <= nc; ++m) {
      double x = dep[m * RC + r];
      if (x != 0.0) unsafeAtomicAdd(&fl.dep[m][id], TS(x * iv));
    }
  }

  // Diagnostics: the workgroup's FP64 sums go to its own slot of `part`
  // (plain stores; a second kernel adds the slots in a fixed order), so no
  // atomics contend on the few diagnostic words.
  if (dg) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double s_cells = double(a_cells);
    double s_j[3] = {dsum[0][threadIdx.x], dsum[1][threadIdx.x], dsum[2][threadIdx.x]};
    double s_e = dsum[3][threadIdx.x], s_abs = dsum[4][threadIdx.x];
    if (sums) {
      for (int k = 0; k < 3; ++k) s_j[k] = wave_sum(s_j[k]);
      s_e = wave_sum(s_e);
      s_abs = wave_sum(s_abs);
      s_cells = wave_max(s_cells);
    }
    unsigned long long fb = wave_sum(n_fb);
    __shared__ double red[FUSED_THREADS / 64][PART_WORDS];
    if (lane == 0) {
      red[wave][0] = s_j[0];
      red[wave][1] = s_j[1];
      red[wave][2] = s_j[2];
      red[wave][3] = s_e;
      red[wave][4] = s_abs;
      red[wave][5] = s_cells;
      red[wave][6] = double(fb);
      red[wave][7] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x < PART_WORDS) {
      const int k = threadIdx.x;
      double v = red[0][k];
      for (int w = 1; w < FUSED_THREADS / 64; ++w) v = k == 5 ? fmax(v, red[w][k]) : v + red[w][k];
      part[(size_t)blockIdx.x * PART_WORDS + k] = sums || k >= 6 ? v : 0.0;
    }
  }
}

// The deferred particles of a fused launch (their stencil at x^{n+1/2} left
// their tile's window): the same step, one thread per particle, gathering
// from and depositing to global memory (FP64 x-ghost layer for the shear
// ghosts).  Their diagnostic sums go to partial slots part0 .. part0 +
// DEFER_BLOCKS - 1; slot word 6 counts them.  Removals through open faces
// and the sticky flags go to dg directly, as in the tile kernel.
template <typename TS, typename A, int GEOM, int NDIM, bool U>
__global__ void __launch_bounds__(256)
    k_fused_deferred(PView<TS> p, PView<TS> dst, int copy_attrs, const Box* __restrict__ boxes,
                     int nbox, FView<TS> fl, Forces f, const Species* __restrict__ sp, int drag_mode,
                     A dt, const double* __restrict__ tdev, const double* __restrict__ xg,
                     const uint32_t* __restrict__ list, const uint32_t* __restrict__ count,
                     double* __restrict__ part, int part0, int sums, DiagDev* dg) {
  constexpr int nc = GEOM == GEOM_CART ? NDIM : 3;
  constexpr int c2 = NDIM > 2 ? 1 : 0;
  const uint32_t n = *count;
  const double t0 = *tdev;
  const A h = A(0.5) * dt;
  double s_j[3] = {0, 0, 0}, s_e = 0, s_abs = 0, s_cells = 0, s_n = 0;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int64_t i = list[2 * e], si = list[2 * e + 1];   // slot written, particle read
    const int32_t cid = p.cell[si];
    const int b = find_box(boxes, nbox, cid);
    const Box& B = boxes[b];
    int idx[3];
    A off[3], mom[3];
    unravel(B, cid - B.cell_base, idx);
    bool bad = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      off[d] = d < NDIM ? A(p.off[d][si]) : A(0);
      mom[d] = d < nc ? A(p.mom[d][si]) : A(0);
      bad |= !(off[d] >= A(-0.5) && off[d] < A(0.5));
    }
    if (bad) flag(dg, DUST_FLAG_OFFSET_RANGE);
    s_n += 1.0;
    bool alive = drift_any<A, GEOM, NDIM, U>(B, f, true, h, t0 + double(h), idx, off, mom);
    if (alive) {
      Stencil<A> s;
      stencil_weights<A, GEOM, NDIM, U>(B, idx, off, s);
      constexpr bool AZ = az_gather<A, GEOM>();
      constexpr int PHI = az_comp<GEOM>();
      double wr[3] = {0.0, 0.0, 0.0};
      if constexpr (AZ) radial_weights64<A, GEOM, U>(B, idx[0], off[0], s, wr);
      Where<A> wh;
      where<A, GEOM, NDIM, U>(B, idx, off, wh);
      SlipScale<A> ss;
      slip_scale<A, GEOM, NDIM, U>(B, idx, off, mom, wh, ss);
      const A* up = ss.up;
      A v[3] = {A(0), A(0), A(0)};
      double vaz = 0.0;   // azimuthal component in FP64 (AZ)
      // The stencil's field values are loaded unconditionally, so that the
      // loads issue together; x ghosts of a shear-periodic box then take the
      // FP64 ghost layer's value (a rare branch).
      const bool xghost = xg && B.xg_base >= 0 && (idx[0] <= 0 || idx[0] >= B.ax[0].n - 1);
#pragma unroll
      for (int c = -c2; c <= c2; ++c)
#pragma unroll
        for (int bb = -1; bb <= 1; ++bb) {
          double g[3][3];
#pragma unroll
          for (int a = -1; a <= 1; ++a) {
            const int64_t id = stored_index(B, idx[0] + a, idx[1] + bb, idx[2] + c);
#pragma unroll
            for (int m = 0; m < nc; ++m) g[a + 1][m] = double(fl.vel[m][id]);
          }
          if (xghost) {
#pragma unroll
            for (int a = -1; a <= 1; ++a)
#pragma unroll
              for (int m = 0; m < nc; ++m)
                g[a + 1][m] = gas_comp(B, fl, xg, m, idx[0] + a, idx[1] + bb, idx[2] + c);
          }
#pragma unroll
          for (int a = -1; a <= 1; ++a) {
            const A w = s.w[0][a + 1] * s.w[1][bb + 1] * s.w[2][c + 1];
#pragma unroll
            for (int m = 0; m < nc; ++m) {
              if (AZ && m == PHI) continue;
              v[m] += w * A(g[a + 1][m] - double(up[m]));
            }
            if constexpr (AZ)
              vaz += wr[a + 1] * (double(s.w[1][bb + 1]) * double(s.w[2][c + 1])) *
                     (g[a + 1][PHI] - double(up[PHI]));
          }
        }
      if constexpr (AZ) v[PHI] = A(vaz);
      A sl[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) sl[m] = m < nc ? slip_canonical<A, GEOM>(ss, m, v[m]) : A(0);
      int spc = p.species ? p.species[si] : 0;
      if (spc >= sp->n) spc = 0;
      const A m = p.mass ? A(p.mass[si]) : A(sp->mass[spc]);
      A it = drag_mode == DRAG_SPECIES ? A(sp->inv_tau[spc])
                                       : inverse_tau<A, GEOM>(f, drag_mode, A(p.drag[si]), A(0), wh);
      A c, psi;
      propagator<A>(dt * it, c, psi);
      KickOut<A> o;
      kick_any<A, GEOM, NDIM>(B, f, dt, it, c, psi, wh, mom, sl, o);
      A q[4] = {A(0), A(0), A(0), A(0)};
#pragma unroll
      for (int k = 0; k < nc; ++k) {
        q[k] = -m * o.j[k];
        if (sums) {
          A vbar = (mom[k] + A(0.5) * o.dp[k]) / wh.sc[k];
          A dl = cell_width<A, U>(B.ax[k], idx[k]) * (GEOM == GEOM_CART || k == 0 ? A(1) : wh.sc[k]);
          const double cps = fabs(double(vbar * dt / dl));
          s_cells = cps > s_cells ? cps : s_cells;
          s_j[k] -= double(q[k]);
          s_abs += fabs(double(q[k]));
        }
        mom[k] += o.dp[k];
      }
      q[nc] = -m * o.e;
      if (sums) s_e -= double(q[nc]);
#pragma unroll
      for (int cc = -c2; cc <= c2; ++cc)
#pragma unroll
        for (int bb = -1; bb <= 1; ++bb)
#pragma unroll
          for (int a = -1; a <= 1; ++a) {
            const int ii = idx[0] + a, jj = idx[1] + bb, kk = idx[2] + cc;
            const A w = s.w[0][a + 1] * s.w[1][bb + 1] * s.w[2][cc + 1] * A(inv_volume(B, ii, jj, kk));
            const int64_t id = stored_index(B, ii, jj, kk);
#pragma unroll
            for (int k = 0; k <= nc; ++k) unsafeAtomicAdd(&fl.dep[k][id], TS(w * q[k]));
          }
      alive = drift_any<A, GEOM, NDIM, U>(B, f, false, h, t0 + double(dt), idx, off, mom);
      store_particle_any<TS, A, GEOM, NDIM>(dst, B, f, t0 + double(dt), i, alive, idx, off, mom, dg);
    } else {
      store_particle_any<TS, A, GEOM, NDIM>(dst, B, f, t0 + double(h), i, false, idx, off, mom, dg);
    }
    if (copy_attrs) {
      if (!alive) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          if (d < NDIM) dst.off[d][i] = p.off[d][si];
          if (d < nc) dst.mom[d][i] = p.mom[d][si];
        }
      }
      if (p.drag) dst.drag[i] = p.drag[si];
      if (p.mass) dst.mass[i] = p.mass[si];
      if (p.species) dst.species[i] = p.species[si];
      if (p.id) dst.id[i] = p.id[si];
    }
  }
  // block partials (fixed order) into slot part0 + blockIdx.x
  __shared__ double red[4][PART_WORDS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double vals[PART_WORDS] = {s_j[0], s_j[1], s_j[2], s_e, s_abs, s_cells, s_n, 0.0};
  for (int k = 0; k < PART_WORDS; ++k) vals[k] = k == 5 ? wave_max(vals[k]) : wave_sum(vals[k]);
  if (lane == 0)
    for (int k = 0; k < PART_WORDS; ++k) red[wave][k] = vals[k];
  __syncthreads();
  if (threadIdx.x < PART_WORDS) {
    const int k = threadIdx.x;
    double v = red[0][k];
    for (int w = 1; w < 4; ++w) v = k == 5 ? fmax(v, red[w][k]) : v + red[w][k];
    part[(size_t)(part0 + blockIdx.x) * PART_WORDS + k] = v;
  }
}

template <typename TS, typename A, int GEOM, int NDIM, bool U, int TX, int TY, int TZ, bool FG>
void launch_fused_t(const FusedPlan& plan, const PView<TS>& p, const PView<TS>& q,
                           bool copy_attrs, const Box* boxes_d,
                           const FView<TS>& fl, const Forces& f, const Species* sp, int drag_mode,
                           double dt, const double* tdev, const int64_t* bin_start, const double* xg,
                           DiagDev* dg, double* part, bool sums, uint32_t* defer_list,
                           uint32_t* defer_count, const uint32_t* src_index, hipStream_t st) {
  constexpr int nc = GEOM == GEOM_CART ? NDIM : 3;
  size_t lds = fused_lds_bytes(plan, nc, (int)sizeof(TS));
  auto kern = k_fused<TS, A, GEOM, NDIM, U, TX, TY, TZ, FG>;
  if (lds > 64 * 1024) {
    static bool raised = false;
    if (!raised) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      raised = true;
    }
  }
  hipLaunchKernelGGL(kern, dim3(plan.ntiles), dim3(FUSED_THREADS), lds, st, plan.tiles_d, p, q,
                     (int)copy_attrs, boxes_d, fl, f, sp, drag_mode, A(dt), tdev, bin_start, xg, dg, part,
                     (int)sums, defer_list, defer_count, src_index);
}

// One fused launch of every tile for one geometry (the tile kernel, then the
// deferred-particle kernel); ev0 / ev1 bracket the tile kernel.
template <typename TS, typename A, int GEOM, int NDIM, bool U>
void launch_fused_g(const FusedPlan& plan, const PView<TS>& p, const PView<TS>& q,
                           bool copy_attrs, const Box* boxes_d,
                           const FView<TS>& fl, const Forces& f, const Species* sp, int drag_mode,
                           double dt, const double* tdev, const int64_t* bin_start, const double* xg,
                           DiagDev* dg, double* part, bool sums, uint32_t* defer_list,
                           uint32_t* defer_count, const uint32_t* src_index, int nbox,
                           hipEvent_t ev0, hipEvent_t ev1, hipStream_t st) {
  if (ev0) (void)hipEventRecord(ev0, st);   // the tile kernel alone is timed
#define DUST_FK(TX, TY, TZ, FK)                                                                    \
  launch_fused_t<TS, A, GEOM, NDIM, U, TX, TY, TZ, FK>(plan, p, q, copy_attrs, boxes_d, fl, f, sp,    \
                                                       drag_mode, dt, tdev, bin_start, xg, dg, part, \
                                                       sums, defer_list, defer_count, src_index, st)
#define DUST_F(TX, TY, TZ) DUST_FK(TX, TY, TZ, false)
  if constexpr (NDIM == 3 && GEOM == GEOM_CART) {
    // the orbital-advection shearing box has kernels of its own
#define DUST_F3(TX, TY, TZ)                      \
  do {                                           \
    if (f.kind == FORCE_FARGO)                   \
      DUST_FK(TX, TY, TZ, true);                 \
    else                                         \
      DUST_FK(TX, TY, TZ, false);                \
  } while (0)
    switch (plan.shape) {
      case 0: DUST_F3(8, 8, 4); break;
      case 1: DUST_F3(16, 4, 4); break;
      case 2: DUST_F3(4, 16, 4); break;
      case 3: DUST_F3(4, 4, 16); break;
      case 4: DUST_F3(8, 4, 8); break;
      default: DUST_F3(4, 8, 8); break;
    }
#undef DUST_F3
  } else if constexpr (NDIM == 3) {
    switch (plan.shape) {
      case 0: DUST_F(8, 8, 4); break;
      case 1: DUST_F(16, 4, 4); break;
      case 2: DUST_F(4, 16, 4); break;
      case 3: DUST_F(4, 4, 16); break;
      case 4: DUST_F(8, 4, 8); break;
      default: DUST_F(4, 8, 8); break;
    }
  } else {
    switch (plan.shape) {
      case 0: DUST_F(16, 16, 1); break;
      case 1: DUST_F(32, 8, 1); break;
      default: DUST_F(8, 32, 1); break;
    }
  }
#undef DUST_F
#undef DUST_FK
  if (ev1) (void)hipEventRecord(ev1, st);
  hipLaunchKernelGGL((k_fused_deferred<TS, A, GEOM, NDIM, U>), dim3(DEFER_BLOCKS), dim3(256), 0, st, p, q,
                     (int)copy_attrs, boxes_d, nbox, fl, f, sp, drag_mode, A(dt), tdev, xg,
                     (const uint32_t*)defer_list, (const uint32_t*)defer_count, part, plan.ntiles, (int)sums,
                     dg);
}


// Explicit instantiations of launch_fused_g (one per translation unit
// group, declared extern where it is called).
#define DUST_FUSED_G_DECL(PREFIX, TS, A, G, D, UU)                                                      \
  PREFIX template void launch_fused_g<TS, A, G, D, UU>(                                               \
      const FusedPlan&, const PView<TS>&, const PView<TS>&, bool, const Box*, const FView<TS>&,       \
      const Forces&, const Species*, int, double, const double*, const int64_t*, const double*,       \
      DiagDev*, double*, bool, uint32_t*, uint32_t*, const uint32_t*, int, hipEvent_t, hipEvent_t,     \
      hipStream_t);
#define DUST_FUSED_G_ALL(PREFIX, TS, A)                                                                \
  DUST_FUSED_G_DECL(PREFIX, TS, A, GEOM_CART, 2, true)                                                 \
  DUST_FUSED_G_DECL(PREFIX, TS, A, GEOM_CART, 2, false)                                                \
  DUST_FUSED_G_DECL(PREFIX, TS, A, GEOM_CART, 3, true)                                                 \
  DUST_FUSED_G_DECL(PREFIX, TS, A, GEOM_CART, 3, false)                                                \
  DUST_FUSED_G_DECL(PREFIX, TS, A, GEOM_CYL, 3, false)                                                 \
  DUST_FUSED_G_DECL(PREFIX, TS, A, GEOM_SPH, 3, false)

}  // namespace dust
