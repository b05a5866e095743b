// Particle load / store and stencil helpers shared by the unfused and fused
// kernels.
#pragma once

#include "dust_device.h"
#include "dust_launch.h"

namespace dust {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ void flag(DiagDev* dg, unsigned int bits) {
  if (dg) atomicOr(&dg->flags, bits);
}

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T> __device__ __forceinline__ T wave_max(T v) {
  for (int o = 32; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, 64);
    v = u > v ? u : v;
  }
  return v;
}

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* a, double v) {
  atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

// Load the position/momentum of particle i.  Returns the box index or -1 if
// the particle has no cell.
template <typename TS, typename A, int GEOM, int NDIM>
__device__ __forceinline__ int load_particle(const PView<TS>& p, const Box* boxes, int nbox,
                                             int64_t i, int idx[3], A off[3], A mom[3],
                                             DiagDev* dg) {
  int64_t c = p.cell[i];
  if (c < 0) return -1;
  int b = find_box(boxes, nbox, c);
  const Box& B = boxes[b];
  if (c >= B.cell_base + B.ncell) {
    flag(dg, DUST_FLAG_BAD_CELL);
    return -1;
  }
  unravel(B, c - B.cell_base, idx);
  constexpr int nc = GEOM == GEOM_CART ? NDIM : 3;
  bool bad = false, nonfinite = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    off[d] = d < NDIM ? A(p.off[d][i]) : A(0);
    mom[d] = d < nc ? A(p.mom[d][i]) : A(0);
    bad |= !(off[d] >= A(-0.5) && off[d] < A(0.5));
    nonfinite |= !isfinite(double(mom[d]));
  }
  if (bad) flag(dg, DUST_FLAG_OFFSET_RANGE);
  if (nonfinite) flag(dg, DUST_FLAG_NONFINITE);
  return b;
}

// Round the offsets to storage precision; an offset that rounds onto the
// upper face moves to the next cell (same point), with the boundary rules.
template <typename TS, typename A, int GEOM, int NDIM, bool FG = false>
__device__ __forceinline__ bool finalize(const Box& B, const Forces& f, double t, int idx[3],
                                         A off[3], A mom[3], TS out[3]) {
#pragma unroll
  for (int d = 0; d < NDIM; ++d) {
    out[d] = TS(off[d]);
    if (out[d] >= TS(0.5)) {
      out[d] = TS(-0.5);
      off[d] = A(-0.5);
      idx[d] += 1;
      if (GEOM == GEOM_CART && NDIM == 3 && d == 0 && B.ax[0].bc_lo == BC_SHEAR) {
        shear_image<A, FG>(B, f, t, idx, off, mom);
        out[1] = TS(off[1]);
      }
      if (!wrap_plain<A>(B.ax[d], idx[d])) return false;
    }
  }
  return true;
}

template <typename TS, typename A, int GEOM, int NDIM, bool FG = false>
__device__ __forceinline__ void store_particle(const PView<TS>& p, const Box& B, const Forces& f,
                                               double t, int64_t i, bool alive, int idx[3],
                                               A off[3], A mom[3], DiagDev* dg) {
  TS o[3];
  if (alive) alive = finalize<TS, A, GEOM, NDIM, FG>(B, f, t, idx, off, mom, o);
  if (!alive) {
    p.cell[i] = -1;
    if (dg) {
      atomicAdd(&dg->n_removed, 1ull);
      atomicOr(&dg->flags, (unsigned)DUST_FLAG_LEFT_OPEN);
    }
    return;
  }
  p.cell[i] = (int32_t)(B.cell_base + ravel(B, idx));
  constexpr int nc = GEOM == GEOM_CART ? NDIM : 3;
#pragma unroll
  for (int d = 0; d < NDIM; ++d) p.off[d][i] = o[d];
#pragma unroll
  for (int d = 0; d < nc; ++d) p.mom[d][i] = TS(mom[d]);
}

// Weights of the 3^ndim stencil at the particle's current position.
template <typename A> struct Stencil {
  A w[3][3];
};

template <typename A, int GEOM, int NDIM, bool U>
__device__ __forceinline__ void stencil_weights(const Box& B, const int idx[3], const A off[3],
                                                Stencil<A>& s) {
  axis_weights<A, axis_kind(GEOM, 0), U>(B.ax[0], idx[0], off[0], s.w[0]);
  axis_weights<A, axis_kind(GEOM, 1), U>(B.ax[1], idx[1], off[1], s.w[1]);
  if constexpr (NDIM > 2) {
    axis_weights<A, axis_kind(GEOM, 2), U>(B.ax[2], idx[2], off[2], s.w[2]);
  } else {
    s.w[2][0] = A(0); s.w[2][1] = A(1); s.w[2][2] = A(0);
  }
}


// FP32 arithmetic in cylindrical and spherical boxes: the azimuthal gas
// velocity spreads over a particle's stencil by about the radial cell width
// over the radius (it varies mostly with radius), far above the slip of a
// particle close to co-rotation, so FP32 radial weights (a few ulp) and an
// FP32 sum would leave errors of that size in the slip.  That component's
// gather therefore sums in FP64 with FP64 radial weights (the other axes'
// weights, exact FP32 values, enter as doubles); every other component
// keeps the FP32 gather.
template <typename A, int GEOM> __host__ __device__ constexpr bool az_gather() {
  return sizeof(A) == 4 && GEOM != GEOM_CART;
}
template <int GEOM> __host__ __device__ constexpr int az_comp() { return GEOM == GEOM_SPH ? 2 : 1; }

// Radial weights in FP64 for that gather, also rounded into s.w[0].
template <typename A, int GEOM, bool U>
__device__ __forceinline__ void radial_weights64(const Box& B, int i, A off0, Stencil<A>& s, double wr[3]) {
  axis_weights<double, axis_kind(GEOM, 0), U>(B.ax[0], i, double(off0), wr);
#pragma unroll
  for (int q = 0; q < 3; ++q) s.w[0][q] = A(wr[q]);
}

// Tile-major key of active cell `local` of box B: tiles in x-fastest order,
// cells x-fastest inside a tile (tiles clipped at the box edges), plus the
// box's first cell id.
// Tile extents are powers of two (the compiled shapes), so the tile of a
// cell is a shift.
__device__ __forceinline__ uint32_t tile_key_idx(const Box& B, const int idx[3], TileShape ts) {
  int n[3] = {B.ax[0].n, B.ax[1].n, B.ndim > 2 ? B.ax[2].n : 1};
  int t[3] = {ts.t[0], ts.t[1], B.ndim > 2 ? ts.t[2] : 1};
  int tid[3], ext[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    tid[d] = idx[d] >> (__ffs(t[d]) - 1);
    int rem = n[d] - tid[d] * t[d];
    ext[d] = rem < t[d] ? rem : t[d];
  }
  int64_t before = (int64_t)tid[2] * t[2] * n[0] * n[1] +
                   (int64_t)tid[1] * t[1] * n[0] * ext[2] +
                   (int64_t)tid[0] * t[0] * ext[1] * ext[2];
  int64_t li = (idx[0] - tid[0] * t[0]) +
               (int64_t)ext[0] * ((idx[1] - tid[1] * t[1]) + (int64_t)ext[1] * (idx[2] - tid[2] * t[2]));
  return (uint32_t)(B.cell_base + before + li);
}

__device__ __forceinline__ uint32_t tile_key(const Box& B, int64_t local, TileShape ts) {
  int idx[3];
  unravel(B, local, idx);
  return tile_key_idx(B, idx, ts);
}

// Gas velocity component m of stored cell (i, j, k), in FP64: from the FP64
// x-ghost layer when the cell is an x ghost of a shear-periodic box and the
// layer is given (xg), else from the field array.
template <typename TS>
__device__ __forceinline__ double gas_comp(const Box& B, const FView<TS>& fl, const double* xg, int m,
                                           int i, int j, int k) {
  if (xg && B.xg_base >= 0 && (i < 0 || i >= B.ax[0].n)) {
    const int64_t g1 = B.ax[1].n + 2, layer = g1 * (B.ax[2].n + 2);
    const int side = i < 0 ? 0 : 1;
    return xg[B.xg_base + (int64_t)(side * 3 + m) * layer + (int64_t)(k + 1) * g1 + (j + 1)];
  }
  return double(fl.vel[m][stored_index(B, i, j, k)]);
}

// Shear offset (y-cells) split into integer and fractional parts.
struct Shift {
  int si;      // floor(s)
  double sf;   // s - floor(s)
  double u;    // q Omega L_x
};

__device__ __forceinline__ Shift make_shift(const Box& B, double qOmega, double t) {
  Shift sh{0, 0.0, 0.0};
  if (B.ax[0].bc_lo != BC_SHEAR) return sh;
  sh.u = qOmega * B.ax[0].L;
  double s = fmod(sh.u * t / B.ax[1].d, (double)B.ax[1].n);
  if (s < 0) s += B.ax[1].n;
  double fl = floor(s);
  sh.si = (int)fl;
  sh.sf = s - fl;
  if (sh.si >= B.ax[1].n) sh.si -= B.ax[1].n;
  return sh;
}


// The orbital-advection flag picked at run time (kernels off the hot loop).
template <typename A, int GEOM, int NDIM, bool U>
__device__ __forceinline__ bool drift_any(const Box& b, const Forces& f, bool first, A h, double t_after,
                                          int idx[3], A off[3], A mom[3]) {
  if (GEOM == GEOM_CART && NDIM == 3 && f.kind == FORCE_FARGO)
    return drift<A, GEOM, NDIM, U, true>(b, f, first, h, t_after, idx, off, mom);
  return drift<A, GEOM, NDIM, U, false>(b, f, first, h, t_after, idx, off, mom);
}
// Semi-implicit kick (Sec. 3.2, Eq. semi-implicit, a_linear, Lambda),
// Cartesian, in the increment form of kick(): Lambda dp = dt (a(x, p^n) +
// s it) with Lambda = I - (dt/2) d a_tot/dv (diagonal 1 + dt it / 2, the
// rotation block of the shearing box), it = 1/tau; o.j = dp - dt a(p_bar),
// o.e = p_bar . o.j.  A comparison integrator: the unfused kernels only.
template <typename A, int NDIM>
__device__ __forceinline__ void kick_si(const Forces& f, A dt, A it, const Where<A>& w, const A p[3],
                                        const A s[3], KickOut<A>& o) {
  A ae[3] = {A(0), A(0), A(0)};
  A j01 = A(0), j10 = A(0);   // d a_x / d v_y, d a_y / d v_x
  const A Om = A(f.Omega), q = A(f.q);
  if (NDIM == 3 && (f.kind == FORCE_SHEARBOX || f.kind == FORCE_FARGO)) {
    const bool fg = f.kind == FORCE_FARGO;
    j01 = A(2) * Om;
    j10 = fg ? (q - A(2)) * Om : A(-2) * Om;
    ae[0] = A(2) * Om * (p[1] + (fg ? A(0) : q * Om * w.x[0]));
    ae[1] = j10 * p[0];
    if (f.vertical_gravity) ae[2] = -Om * Om * w.x[2];
  } else if (f.kind == FORCE_CONST) {
#pragma unroll
    for (int d = 0; d < 3; ++d) ae[d] = A(f.g[d]);
  }
  const A dg = A(1) + A(0.5) * dt * it;   // diagonal of Lambda
  A r[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) r[d] = d < NDIM ? dt * (ae[d] + s[d] * it) : A(0);
  // [[dg, -dt/2 j01], [-dt/2 j10, dg]] (dp_x, dp_y) = (r_x, r_y)
  const A m01 = A(-0.5) * dt * j01, m10 = A(-0.5) * dt * j10;
  const A den = A(1) / (dg * dg - m01 * m10);
  o.dp[0] = (dg * r[0] - m01 * r[1]) * den;
  o.dp[1] = (dg * r[1] - m10 * r[0]) * den;
  o.dp[2] = NDIM > 2 ? r[2] / dg : A(0);
  if (NDIM < 2) o.dp[1] = A(0);
  const A a[3] = {ae[0] + A(0.5) * j01 * o.dp[1], ae[1] + A(0.5) * j10 * o.dp[0], ae[2]};
  o.e = A(0);
  o.cells = A(0);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    o.j[d] = d < NDIM ? o.dp[d] - dt * a[d] : A(0);
    if (d < NDIM) o.e += (p[d] + A(0.5) * o.dp[d]) * o.j[d];
  }
}

// (it: 1/tau, which the semi-implicit kick takes instead of c and psi)
template <typename A, int GEOM, int NDIM>
__device__ __forceinline__ void kick_any(const Box& b, const Forces& f, A dt, A it, A c, A psi,
                                         const Where<A>& w, const A p[3], const A s[3], KickOut<A>& o) {
  if constexpr (GEOM == GEOM_CART) {
    if (f.integrator == DUST_INTEGRATOR_SEMI_IMPLICIT) {
      kick_si<A, NDIM>(f, dt, it, w, p, s, o);
      return;
    }
  }
  if (GEOM == GEOM_CART && NDIM == 3 && f.kind == FORCE_FARGO)
    kick<A, GEOM, NDIM, true>(b, f, dt, c, psi, w, p, s, o);
  else
    kick<A, GEOM, NDIM, false>(b, f, dt, c, psi, w, p, s, o);
}
template <typename TS, typename A, int GEOM, int NDIM>
__device__ __forceinline__ void store_particle_any(const PView<TS>& p, const Box& B, const Forces& f,
                                                   double t, int64_t i, bool alive, int idx[3], A off[3],
                                                   A mom[3], DiagDev* dg) {
  if (GEOM == GEOM_CART && NDIM == 3 && f.kind == FORCE_FARGO)
    store_particle<TS, A, GEOM, NDIM, true>(p, B, f, t, i, alive, idx, off, mom, dg);
  else
    store_particle<TS, A, GEOM, NDIM, false>(p, B, f, t, i, alive, idx, off, mom, dg);
}

}  // namespace dust
