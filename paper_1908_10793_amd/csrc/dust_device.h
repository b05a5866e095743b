// Per-particle device arithmetic of the dust hot path (gfx950).
//
// Templates: TS = storage type of reals (float or double), A = arithmetic
// type of the per-particle math (double by default also for float storage:
// gfx950 issues FP64 vector FMAs at the rate of unpacked FP32 ones, and the
// slip v_g - v_p that the drag acts on is often far below FP32 resolution of
// the velocities themselves).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dust_types.h"

namespace dust {

// ---------------------------------------------------------------- math helpers

template <typename A> __device__ __forceinline__ A dsin(A x);
template <> __device__ __forceinline__ double dsin<double>(double x) { return sin(x); }
template <> __device__ __forceinline__ float dsin<float>(float x) { return sinf(x); }
template <typename A> __device__ __forceinline__ A dcos(A x);
template <> __device__ __forceinline__ double dcos<double>(double x) { return cos(x); }
template <> __device__ __forceinline__ float dcos<float>(float x) { return cosf(x); }
template <typename A> __device__ __forceinline__ A dsqrt(A x);
template <> __device__ __forceinline__ double dsqrt<double>(double x) { return sqrt(x); }
template <> __device__ __forceinline__ float dsqrt<float>(float x) { return sqrtf(x); }
template <typename A> __device__ __forceinline__ A dexpm1(A x);
template <> __device__ __forceinline__ double dexpm1<double>(double x) { return expm1(x); }
template <> __device__ __forceinline__ float dexpm1<float>(float x) { return expm1f(x); }
template <typename A> __device__ __forceinline__ A dfloor(A x);
template <> __device__ __forceinline__ double dfloor<double>(double x) { return floor(x); }
template <> __device__ __forceinline__ float dfloor<float>(float x) { return floorf(x); }
template <typename A> __device__ __forceinline__ A drint(A x);
template <> __device__ __forceinline__ double drint<double>(double x) { return rint(x); }
template <> __device__ __forceinline__ float drint<float>(float x) { return rintf(x); }

// h - sin h without cancellation (series for small h; reciprocal constants
// instead of divisions).
template <typename A> __device__ __forceinline__ A h_minus_sin(A h) {
  if (h < A(0.5) && h > A(-0.5)) {
    A h2 = h * h;
    A s = A(1) - h2 * A(1.0 / 210);
    s = A(1) - h2 * A(1.0 / 156) * s;
    s = A(1) - h2 * A(1.0 / 110) * s;
    s = A(1) - h2 * A(1.0 / 72) * s;
    s = A(1) - h2 * A(1.0 / 42) * s;
    s = A(1) - h2 * A(1.0 / 20) * s;
    return h * h2 * A(1.0 / 6) * s;
  }
  return h - dsin(h);
}

// Drag propagator terms for h = dt/tau >= 0 (Eq. h1, phi1 of Sec. 3.2.2):
//   c   = 1 - e^{-h}               (= h1/tau), from expm1
//   psi = phi1(-h) - 1 = (h1 - dt)/dt, series for small h
// so that h1 = dt (1 + psi) and the kick is written in increments.
template <typename A> __device__ __forceinline__ void propagator(A h, A& c, A& psi) {
  if (h == A(0)) {
    c = A(0);
    psi = A(0);
    return;
  }
  c = -dexpm1(-h);
  if (h < A(0.25)) {
    // psi = sum_{k>=1} (-h)^k/(k+1)!, nested
    A s = A(1) - h * A(1.0 / 14);
    s = A(1) - h * A(1.0 / 13) * s;
    s = A(1) - h * A(1.0 / 12) * s;
    s = A(1) - h * A(1.0 / 11) * s;
    s = A(1) - h * A(1.0 / 10) * s;
    s = A(1) - h * A(1.0 / 9) * s;
    s = A(1) - h * A(1.0 / 8) * s;
    s = A(1) - h * A(1.0 / 7) * s;
    s = A(1) - h * A(1.0 / 6) * s;
    s = A(1) - h * A(1.0 / 5) * s;
    s = A(1) - h * A(1.0 / 4) * s;
    s = A(1) - h * A(1.0 / 3) * s;
    psi = -h * A(0.5) * s;
  } else {
    psi = c / h - A(1);
  }
}

// ---------------------------------------------------------------- geometry

// Weight formula of axis d of a geometry (known at compile time, so that a
// kernel carries only the formulas of its own geometry).
constexpr int axis_kind(int geom, int d) {
  return geom == GEOM_CYL ? (d == 0 ? AX_CYL_R : AX_PLAIN)
       : geom == GEOM_SPH ? (d == 0 ? AX_SPH_R : (d == 1 ? AX_THETA : AX_PLAIN))
       : AX_PLAIN;
}

// Coordinate of the centre and width of cell i (i in [-1, n]) on an axis.
// U: every axis of the boxes is known to be uniform (no face table needed);
// otherwise uniformity is read from the axis.
template <typename A, bool U> __device__ __forceinline__ A cell_centre(const Axis& ax, int i) {
  if (U || ax.uniform) return A(ax.lo + (double(i) + 0.5) * ax.d);
  return A(0.5 * (ax.faces[i + 1] + ax.faces[i + 2]));
}
template <typename A, bool U> __device__ __forceinline__ A cell_width(const Axis& ax, int i) {
  if (U || ax.uniform) return A(ax.d);
  return A(ax.faces[i + 2] - ax.faces[i + 1]);
}

// Weights of cells i-1, i, i+1 along one axis for a particle at offset delta
// (host-cell widths) from the centre of host cell i.  The shape spans the
// host cell's width; what lies beyond the host cell's faces goes to the
// neighbour on that side, so sum w = 1 up to rounding and the middle weight
// is 1 - w[0] - w[2].
template <typename A, int KIND, bool U>
__device__ __forceinline__ void axis_weights(const Axis& ax, int i, A delta, A w[3]) {
  const A half = A(0.5);
  if constexpr (KIND == AX_PLAIN) {
    if (ax.shape == SHAPE_CIC) {
      w[0] = delta < A(0) ? -delta : A(0);
      w[2] = delta > A(0) ? delta : A(0);
    } else {
      A m = half - delta, p = half + delta;
      w[0] = half * m * m;
      w[2] = half * p * p;
    }
  } else if constexpr (KIND == AX_CYL_R) {
    // Eq. CIC_cylindrical / TSC_cylindrical, nu = R_i / Delta R_i
    A nu = cell_centre<A, U>(ax, i) / cell_width<A, U>(ax, i);
    if (ax.shape == SHAPE_VOL) {
      // Eq. CIC_vol: linear in R^2 between the two cell centres around R_p,
      // in factored form (R_c^2 - R_p^2 = (R_c - R_p)(R_c + R_p))
      const A c = cell_centre<A, U>(ax, i), dr = delta * cell_width<A, U>(ax, i), rp = c + dr;
      if (delta < A(0)) {
        const A cl = cell_centre<A, U>(ax, i - 1);
        w[0] = (-dr) * (c + rp) / ((c - cl) * (c + cl));
        w[2] = A(0);
      } else {
        const A ch = cell_centre<A, U>(ax, i + 1);
        w[2] = dr * (rp + c) / ((ch - c) * (ch + c));
        w[0] = A(0);
      }
    } else if (ax.shape == SHAPE_CIC) {
      A den = A(2) * (delta + nu);
      w[0] = delta < A(0) ? (delta + A(2) * nu - A(1)) / den * (-delta) : A(0);
      w[2] = delta > A(0) ? (delta + A(2) * nu + A(1)) / den * delta : A(0);
    } else {
      A den = A(3) * (delta + nu);
      A m = half - delta, p = half + delta;
      w[0] = (delta + A(3) * nu - A(2)) / den * half * m * m;
      w[2] = (delta + A(3) * nu + A(2)) / den * half * p * p;
    }
  } else if constexpr (KIND == AX_SPH_R) {
    // App. C: Eq. CIC_spherical_r / TSC_spherical_r
    A nu = cell_centre<A, U>(ax, i) / cell_width<A, U>(ax, i);
    A dn = delta + nu;
    if (ax.shape == SHAPE_CIC) {
      A den = A(12) * dn * dn + A(1);
      if (delta < A(0)) {
        A t = A(2) * delta + A(3) * nu - A(1.5), u = nu - half;
        w[0] = (t * t + A(3) * u * u) / den * (-delta);
        w[2] = A(0);
      } else {
        A t = A(2) * delta + A(3) * nu + A(1.5), u = nu + half;
        w[2] = (t * t + A(3) * u * u) / den * delta;
        w[0] = A(0);
      }
    } else {
      A den = A(6) * dn * dn + A(1);
      A m = half - delta, p = half + delta;
      A d2 = delta * delta, n2 = A(6) * nu * nu;
      w[0] = (d2 + (A(4) * nu - A(3)) * delta + n2 - A(8) * nu + A(2.75)) / den * half * m * m;
      w[2] = (d2 + (A(4) * nu + A(3)) * delta + n2 + A(8) * nu + A(2.75)) / den * half * p * p;
    }
  } else {
    // theta axis, metric sin(theta): App. C Eq. CIC_spherical_theta (minus
    // branch sign corrected) in product form, and the TSC analogue from the
    // antiderivative of (1 -+ (t - t_p)/D) sin t.
    A tc = cell_centre<A, U>(ax, i), D = cell_width<A, U>(ax, i);
    A tp = tc + delta * D;
    A sp = dsin(tp), sh = dsin(half * D);
    if (ax.shape == SHAPE_CIC) {
      A den = sp * sh;
      if (delta > A(0)) {
        w[2] = dsin(tc + half * D + half * delta * D) * dsin(half * delta * D) / den;
        w[0] = A(0);
      } else {
        w[0] = dsin(tc - half * D + half * delta * D) * dsin(-half * delta * D) / den;
        w[2] = A(0);
      }
    } else {
      A den = A(4) * sp * sh * sh;
      A hp = (half + delta) * D, hm = (half - delta) * D;
      A Ap = tc + half * D, Bm = tc - half * D;
      A s1 = dsin(half * hp), s2 = dsin(half * hm);
      w[2] = (dcos(Ap) * h_minus_sin(hp) + A(2) * dsin(Ap) * s1 * s1) / den;
      w[0] = (-dcos(Bm) * h_minus_sin(hm) + A(2) * dsin(Bm) * s2 * s2) / den;
    }
  }
  w[1] = A(1) - w[0] - w[2];
}

// Stored (ghosted) linear index of active-grid cell (i, j, k), each in [-1, n].
__device__ __forceinline__ int64_t stored_index(const Box& b, int i, int j, int k) {
  return b.store_base + (int64_t)(i + 1) +
         (int64_t)b.g0 * ((int64_t)(j + 1) + (int64_t)b.g1 * (int64_t)(k + b.k_off));
}

// Inverse cell volume of cell (i, j, k) (separable per-axis factors).
__device__ __forceinline__ double inv_volume(const Box& b, int i, int j, int k) {
  double v = b.ax[0].ivol[i + 1] * b.ax[1].ivol[j + 1];
  if (b.ndim > 2) v *= b.ax[2].ivol[k + 1];
  return v;
}

// Box of a global cell id (boxes sorted by cell_base).
__device__ __forceinline__ int find_box(const Box* boxes, int nbox, int64_t cell) {
  int b = 0;
  while (b + 1 < nbox && cell >= boxes[b + 1].cell_base) ++b;
  return b;
}

// q = floor(a / n) for 0 <= a < 2^31, n >= 1, through FP64 (exact after one
// correction step).
__device__ __forceinline__ int div_small(int a, int n, double inv_n) {
  int q = (int)(double(a) * inv_n);
  int r = a - q * n;
  if (r < 0) --q;
  else if (r >= n) ++q;
  return q;
}

__device__ __forceinline__ void unravel(const Box& b, int64_t local, int idx[3]) {
  int n0 = b.ax[0].n, n1 = b.ax[1].n;
  int l = (int)local;
  int r = div_small(l, n0, b.ax[0].inv_n);
  idx[0] = l - r * n0;
  if (b.ndim > 2) {
    int k = div_small(r, n1, b.ax[1].inv_n);
    idx[1] = r - k * n1;
    idx[2] = k;
  } else {
    idx[1] = r;
    idx[2] = 0;
  }
}

__device__ __forceinline__ int64_t ravel(const Box& b, const int idx[3]) {
  int64_t c = idx[0] + (int64_t)b.ax[0].n * idx[1];
  if (b.ndim > 2) c += (int64_t)b.ax[0].n * b.ax[1].n * idx[2];
  return c;
}

// ---------------------------------------------------------------- motion

// Move along axis d by a coordinate increment dxi.  Returns the new cell
// index, which may fall outside [0, n) (the caller applies the boundary).
template <typename A, bool U>
__device__ __forceinline__ int move_axis(const Axis& ax, int i, A& delta, A dxi) {
  const A half = A(0.5);
  if (U || ax.uniform) {
    // without branches (a wave would take one whenever a lane crosses a
    // face): the nearest integer k splits the new offset exactly (dn - k is
    // exact for |dn| < 2^23 in FP32), a tie at +1/2 goes to the next cell,
    // and an offset that stays in its cell is kept as it is
    const A dn = delta + dxi * A(ax.inv_d);
    const A k = drint(dn);
    const A r = k == A(0) ? dn : dn - k;
    const bool up = r >= half;
    delta = up ? r - A(1) : r;
    return i + (int)k + (up ? 1 : 0);
  }
  A dn = delta + dxi / cell_width<A, U>(ax, i);
  if (dn < half && dn >= -half) {
    delta = dn;
    return i;
  }
  // FP64 crossing test against the face table (non-uniform axis)
  double xi = 0.5 * (ax.faces[i + 1] + ax.faces[i + 2]) +
              double(delta) * (ax.faces[i + 2] - ax.faces[i + 1]) + double(dxi);
  while (i < ax.n && xi >= ax.faces[i + 2]) ++i;
  while (i >= 0 && xi < ax.faces[i + 1]) --i;
  if (i >= 0 && i < ax.n) {
    double c = 0.5 * (ax.faces[i + 1] + ax.faces[i + 2]), w = ax.faces[i + 2] - ax.faces[i + 1];
    A dl = A((xi - c) / w);
    if (dl >= half) { dl -= A(1); ++i; }  // rounding onto the upper face
    if (dl < -half) dl = -half;
    delta = dl;
  }
  return i;
}

// Apply a periodic or open boundary to axis d.  Returns false if removed.
template <typename A>
__device__ __forceinline__ bool wrap_plain(const Axis& ax, int& i) {
  if (i >= 0 && i < ax.n) return true;
  // both boundary kinds are read (uniform loads) before the per-lane choice
  const bool lo_open = ax.bc_lo == BC_OPEN, hi_open = ax.bc_hi == BC_OPEN;
  if (i < 0 ? lo_open : hi_open) return false;
  i %= ax.n;
  if (i < 0) i += ax.n;
  return true;
}

// The boundaries of the first ND axes, with one test for all of them (a
// wave branches only when one of its lanes is outside the box).  Returns
// false if removed.
template <typename A, int ND>
__device__ __forceinline__ bool wrap_all(const Box& b, int idx[3]) {
  bool out = false;
#pragma unroll
  for (int d = 0; d < ND; ++d) out |= (unsigned)idx[d] >= (unsigned)b.ax[d].n;
  if (out) {
#pragma unroll
    for (int d = 0; d < ND; ++d)
      if (!wrap_plain<A>(b.ax[d], idx[d])) return false;
  }
  return true;
}

// Shear-periodic image across the x faces at time t (Sec. 2.1): x -/+ L_x,
// y +/- q Omega L_x t (as a shift in y-cells), v_y +/- q Omega L_x (not for
// the residual velocities of orbital advection, FG).
//
// FG (here and in drift, kick, finalize, store_particle): the forces are
// the orbital-advection shearing box (Eq. FARGO_SB_p).  It is a template
// flag, so that the standard form's code is not touched by it; the *_any
// wrappers pick it at run time.
template <typename A, bool FG = false>
__device__ __forceinline__ void shear_image(const Box& b, const Forces& f, double t, int idx[3],
                                            A off[3], A mom[3]) {
  const Axis& ax = b.ax[0];
  if (idx[0] >= 0 && idx[0] < ax.n) return;
  double u = f.q * f.Omega * ax.L;
  double s = fmod(u * t / b.ax[1].d, (double)b.ax[1].n);
  if (s < 0) s += b.ax[1].n;
  double sfl = floor(s);
  int si = (int)sfl;
  A sf = A(s - sfl);
  int sign = idx[0] >= ax.n ? 1 : -1;
  idx[0] -= sign * ax.n;
  off[1] += A(sign) * sf;
  idx[1] += sign * si;
  if (off[1] >= A(0.5)) { off[1] -= A(1); ++idx[1]; }
  else if (off[1] < A(-0.5)) { off[1] += A(1); --idx[1]; }
  idx[1] %= b.ax[1].n;
  if (idx[1] < 0) idx[1] += b.ax[1].n;
  if constexpr (!FG) mom[1] += A(sign) * A(u);
}

// Drift by a half step h (Eq. exp_midpoint; Eq. drift1_cylindrical,
// drift2_cylindrical; App. B.2).  `first`: the angles use the radius (and
// theta) already moved to n+1/2; otherwise all metric factors are those at
// the start of this half drift.  t_after: time the boundary rules use.
// Returns false if the particle left through an open face.
template <typename A, int GEOM, int NDIM, bool U, bool FG = false>
__device__ __forceinline__ bool drift(const Box& b, const Forces& f, bool first, A h,
                                      double t_after, int idx[3], A off[3], A mom[3]) {
  if constexpr (GEOM == GEOM_CART) {
    if constexpr (FG && NDIM == 3) {
      // orbital advection: y is also carried by the mean shear -q Omega x,
      // taken at x^{n+1/2} (x moves first in the first drift, last in the
      // second)
      const A qO = A(f.q * f.Omega);
      if (first) idx[0] = move_axis<A, U>(b.ax[0], idx[0], off[0], h * mom[0]);
      const A xh = cell_centre<A, U>(b.ax[0], idx[0]) + off[0] * cell_width<A, U>(b.ax[0], idx[0]);
      idx[1] = move_axis<A, U>(b.ax[1], idx[1], off[1], h * (mom[1] - qO * xh));
      if (!first) idx[0] = move_axis<A, U>(b.ax[0], idx[0], off[0], h * mom[0]);
      idx[2] = move_axis<A, U>(b.ax[2], idx[2], off[2], h * mom[2]);
    } else {
      A dx[3] = {h * mom[0], h * mom[1], NDIM > 2 ? h * mom[2] : A(0)};
#pragma unroll
      for (int d = 0; d < NDIM; ++d) idx[d] = move_axis<A, U>(b.ax[d], idx[d], off[d], dx[d]);
    }
    if (NDIM == 3 && b.ax[0].bc_lo == BC_SHEAR) shear_image<A, FG>(b, f, t_after, idx, off, mom);
    return wrap_all<A, NDIM>(b, idx);
  }
  if constexpr (GEOM == GEOM_CYL) {
    if (first) {
      idx[0] = move_axis<A, U>(b.ax[0], idx[0], off[0], h * mom[0]);
      if (!wrap_plain<A>(b.ax[0], idx[0])) return false;
      A R = cell_centre<A, U>(b.ax[0], idx[0]) + off[0] * cell_width<A, U>(b.ax[0], idx[0]);
      idx[1] = move_axis<A, U>(b.ax[1], idx[1], off[1], h * mom[1] / (R * R));
      idx[2] = move_axis<A, U>(b.ax[2], idx[2], off[2], h * mom[2]);
    } else {
      A R = cell_centre<A, U>(b.ax[0], idx[0]) + off[0] * cell_width<A, U>(b.ax[0], idx[0]);
      idx[1] = move_axis<A, U>(b.ax[1], idx[1], off[1], h * mom[1] / (R * R));
      idx[0] = move_axis<A, U>(b.ax[0], idx[0], off[0], h * mom[0]);
      idx[2] = move_axis<A, U>(b.ax[2], idx[2], off[2], h * mom[2]);
    }
  } else {
    if (first) {
      idx[0] = move_axis<A, U>(b.ax[0], idx[0], off[0], h * mom[0]);
      if (!wrap_plain<A>(b.ax[0], idx[0])) return false;
      A r = cell_centre<A, U>(b.ax[0], idx[0]) + off[0] * cell_width<A, U>(b.ax[0], idx[0]);
      idx[1] = move_axis<A, U>(b.ax[1], idx[1], off[1], h * mom[1] / (r * r));
      if (!wrap_plain<A>(b.ax[1], idx[1])) return false;
      A th = cell_centre<A, U>(b.ax[1], idx[1]) + off[1] * cell_width<A, U>(b.ax[1], idx[1]);
      A s = dsin(th);
      idx[2] = move_axis<A, U>(b.ax[2], idx[2], off[2], h * mom[2] / (r * r * s * s));
    } else {
      A r = cell_centre<A, U>(b.ax[0], idx[0]) + off[0] * cell_width<A, U>(b.ax[0], idx[0]);
      A th = cell_centre<A, U>(b.ax[1], idx[1]) + off[1] * cell_width<A, U>(b.ax[1], idx[1]);
      A s = dsin(th);
      idx[2] = move_axis<A, U>(b.ax[2], idx[2], off[2], h * mom[2] / (r * r * s * s));
      idx[1] = move_axis<A, U>(b.ax[1], idx[1], off[1], h * mom[1] / (r * r));
      idx[0] = move_axis<A, U>(b.ax[0], idx[0], off[0], h * mom[0]);
    }
  }
  return wrap_all<A, 3>(b, idx);
}

// ---------------------------------------------------------------- kick

// Position quantities the kick needs, at x^{n+1/2}.
template <typename A> struct Where {
  A x[3];  // coordinates (x,y,z) / (R,phi,z) / (r,theta,phi)
  A sc[3]; // canonical = physical * sc: 1, R, r, r sin(theta)
};

template <typename A, int GEOM, int NDIM, bool U>
__device__ __forceinline__ void where(const Box& b, const int idx[3], const A off[3], Where<A>& w) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    w.x[d] = d < NDIM ? cell_centre<A, U>(b.ax[d], idx[d]) + off[d] * cell_width<A, U>(b.ax[d], idx[d])
                      : A(0);
    w.sc[d] = A(1);
  }
  if constexpr (GEOM == GEOM_CYL) w.sc[1] = w.x[0];
  if constexpr (GEOM == GEOM_SPH) {
    w.sc[1] = w.x[0];
    w.sc[2] = w.x[0] * dsin(w.x[1]);
  }
}

// Slip form of the gather in curvilinear boxes.  The slip of a canonical
// component m >= 1 (an angular momentum, l = sc u with u the physical
// velocity) is sc * sum_i W_i (v_i - u), and its relative accuracy is that
// of u and sc.  In FP32 a particle close to co-rotation has a slip a
// thousand times below u, where one FP32 word for u or sc (6e-8 relative)
// would leave 6e-5 in the slip; so in FP32 both are carried as unevaluated
// pairs hi + lo: sc evaluated in FP64 at the particle and split in two
// words, and u = l / sc with its remainder formed by an FMA.
// up: the hi part of u, which the gather subtracts from every v_i (those
// differences are exact for close values); ulo, shi, slo: what
// slip_canonical needs.  In FP64, and for Cartesian or radial components,
// u = p / sc with ulo = slo = 0.
template <typename A> struct SlipScale {
  A up[3], ulo[3], shi[3], slo[3];
};

template <typename A, int GEOM, int NDIM, bool U>
__device__ __forceinline__ void slip_scale(const Box& b, const int idx[3], const A off[3], const A mom[3],
                                           const Where<A>& wh, SlipScale<A>& q) {
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    q.up[m] = GEOM == GEOM_CART || m == 0 ? mom[m] : mom[m] / wh.sc[m];
    q.ulo[m] = A(0);
    q.shi[m] = wh.sc[m];
    q.slo[m] = A(0);
  }
  if constexpr (GEOM != GEOM_CART && sizeof(A) == 4) {
    // the particle's radius in FP64 (cell centre plus offset), split in two
    // words: an FP32 offset term would be off by up to half an ulp of half a
    // cell width, which the slip of a particle close to co-rotation does not
    // tolerate
    const double R = fma(double(off[0]), cell_width<double, U>(b.ax[0], idx[0]),
                         cell_centre<double, U>(b.ax[0], idx[0]));
    const float rh = float(R);
    q.shi[1] = rh;
    q.slo[1] = float(R - double(rh));
    if constexpr (GEOM == GEOM_SPH) {
      // sin(theta_c + d) = S + (S (cos d - 1) + C sin d), S and C from the
      // FP64 table of cell centres, with series in d, |d| below half a cell
      // (truncated at d^7 / 5040: below 1e-12 for cells up to 0.1 rad), and
      // R sin(theta) in FP64
      const double* tg = b.ax[1].trig + 2 * (idx[1] + 1);
      const double S = tg[0], C = tg[1];
      const double d = double(off[1]) * cell_width<double, U>(b.ax[1], idx[1]);
      const double d2 = d * d;
      const double sd = d * (1.0 - d2 * (1.0 / 6.0) * (1.0 - d2 * (1.0 / 20.0)));
      const double cm1 = -0.5 * d2 * (1.0 - d2 * (1.0 / 12.0) * (1.0 - d2 * (1.0 / 30.0)));
      const double pr = R * (S + (S * cm1 + C * sd));
      const float ph = float(pr);
      q.shi[2] = ph;
      q.slo[2] = float(pr - double(ph));
    }
#pragma unroll
    for (int m = 1; m < 3; ++m) {
      if (GEOM == GEOM_CYL && m == 2) continue;   // v_z: Cartesian
      const float S = q.shi[m] + q.slo[m];
      const float u = mom[m] / S;
      const float e = fmaf(-u, q.shi[m], mom[m]) - u * q.slo[m];   // mom - u (hi + lo)
      q.up[m] = u;
      q.ulo[m] = e / S;
    }
  }
}

// Canonical slip from the gathered sum_i W_i (v_i - up) of component m.
template <typename A, int GEOM>
__device__ __forceinline__ A slip_canonical(const SlipScale<A>& q, int m, A v) {
  if (GEOM == GEOM_CART || m == 0) return v;
  const A s = v - q.ulo[m];
  return fma(s, q.shi[m], s * q.slo[m]);
}

// Result of one kick: momentum increments, drag impulse per unit mass
// J/m = c s + dt psi a (s = p_g - p, the slip; a = the non-drag part of G as
// evaluated in the kick), and the energy e/m = v_bar . (J/m) (physical).
template <typename A> struct KickOut {
  A dp[3];
  A j[3];
  A e;
  A cells;  // max_d |v_bar_d| dt / dl_d
};

// Exponential-midpoint kick (Eq. exp_midpoint with A = -diag(1/tau);
// App. B.1 Eq. standard_SB_exp_midpoint; App. B.2 Eq. kick_cylindrical and
// its spherical analogue) for canonical momenta p, slip s = p_g - p (canonical; the gas
// momentum at the particle minus p) and the drag propagator terms c, psi
// of h = dt/tau (see propagator()).
template <typename A, int GEOM, int NDIM, bool FG = false>
__device__ __forceinline__ void kick(const Box& b, const Forces& f, A dt, A c, A psi,
                                     const Where<A>& w, const A p[3], const A s[3],
                                     KickOut<A>& o) {
  A h1 = dt + dt * psi;
  A a[3] = {A(0), A(0), A(0)};
  constexpr int nc = GEOM == GEOM_CART ? NDIM : 3;
  if constexpr (GEOM == GEOM_CART) {
    if constexpr (FG && NDIM == 3) {
      // orbital advection (App. B.1, Eq. FARGO_SB_exp_midpoint), residual
      // velocities: R dp = c s + h1 a(p^n), R = [[1, -W1], [W2, 1]],
      // W1 = Omega h1, W2 = W1 (1 - q/2)
      A Om = A(f.Omega), q = A(f.q);
      A gz = f.vertical_gravity ? -Om * Om * w.x[2] : A(0);
      A an[3] = {A(2) * Om * p[1], (q - A(2)) * Om * p[0], gz};
      A r[3] = {c * s[0] + h1 * an[0], c * s[1] + h1 * an[1], c * s[2] + h1 * an[2]};
      A W1 = Om * h1, W2 = W1 * (A(1) - A(0.5) * q), den = A(1) / (A(1) + W1 * W2);
      o.dp[0] = (r[0] + W1 * r[1]) * den;
      o.dp[1] = (r[1] - W2 * r[0]) * den;
      o.dp[2] = r[2];
      a[0] = an[0] + Om * o.dp[1];
      a[1] = an[1] + A(0.5) * (q - A(2)) * Om * o.dp[0];
      a[2] = gz;
    } else if (NDIM == 3 && f.kind == FORCE_SHEARBOX) {
      // R dp = c s + h1 a(x, p^n), R = I - W J_rot, W = Omega h1
      A Om = A(f.Omega), q = A(f.q);
      A gz = f.vertical_gravity ? -Om * Om * w.x[2] : A(0);
      A an[3] = {A(2) * Om * (p[1] + q * Om * w.x[0]), A(-2) * Om * p[0], gz};
      A r[3] = {c * s[0] + h1 * an[0], c * s[1] + h1 * an[1], c * s[2] + h1 * an[2]};
      A W = Om * h1, den = A(1) / (A(1) + W * W);
      o.dp[0] = (r[0] + W * r[1]) * den;
      o.dp[1] = (r[1] - W * r[0]) * den;
      o.dp[2] = r[2];
      a[0] = an[0] + Om * o.dp[1];
      a[1] = an[1] - Om * o.dp[0];
      a[2] = gz;
    } else {
#pragma unroll
      for (int k = 0; k < nc; ++k) {
        a[k] = f.kind == FORCE_CONST ? A(f.g[k]) : A(0);
        o.dp[k] = c * s[k] + h1 * a[k];
      }
      if (nc < 3) o.dp[2] = A(0);
    }
  } else if constexpr (GEOM == GEOM_CYL) {
    A R = w.x[0], z = w.x[2];
    A gR = A(0), gz = A(0);
    if (f.kind == FORCE_POINTMASS) {
      A r2 = R * R + z * z;
      A ir3 = A(f.GM) / (r2 * dsqrt(r2));
      gR = -R * ir3;
      gz = -z * ir3;
    }
    // order v_z, l_phi, v_R
    a[2] = gz;
    o.dp[2] = c * s[2] + h1 * a[2];
    a[1] = A(0);  // R g_phi, axisymmetric potential
    o.dp[1] = c * s[1];
    A l0 = p[1], l1 = p[1] + o.dp[1];
    a[0] = A(0.5) * (l0 * l0 + l1 * l1) / (R * R * R) + gR;
    o.dp[0] = c * s[0] + h1 * a[0];
  } else {
    A r = w.x[0], th = w.x[1];
    A st = dsin(th), ct = dcos(th);
    A gr = f.kind == FORCE_POINTMASS ? A(-f.GM) / (r * r) : A(0);
    // order l_phi, l_theta, v_r; the second midpoint average is that of l_theta^2
    a[2] = A(0);  // r sin(theta) g_phi
    o.dp[2] = c * s[2];
    A lp0 = p[2], lp1 = p[2] + o.dp[2];
    A lp2 = A(0.5) * (lp0 * lp0 + lp1 * lp1);
    a[1] = lp2 * ct / (r * r * st * st * st);  // + r g_theta = 0
    o.dp[1] = c * s[1] + h1 * a[1];
    A lt0 = p[1], lt1 = p[1] + o.dp[1];
    A lt2 = A(0.5) * (lt0 * lt0 + lt1 * lt1);
    a[0] = lt2 / (r * r * r) + lp2 / (r * r * r * st * st) + gr;
    o.dp[0] = c * s[0] + h1 * a[0];
  }
  o.e = A(0);
  o.cells = A(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    o.j[k] = k < nc ? c * s[k] + dt * psi * a[k] : A(0);
    A vbar = (p[k] + A(0.5) * o.dp[k]) / w.sc[k];
    o.e += vbar * (o.j[k] / w.sc[k]);
  }
}

// Inverse stopping time of a particle: species table (1/tau precomputed),
// per-particle tau, or per-particle Stokes number St = tau Omega_K(R) with R
// the cylindrical radius at x^{n+1/2}.
template <typename A, int GEOM>
__device__ __forceinline__ A inverse_tau(const Forces& f, int drag_mode, A dval, A sp_inv_tau,
                                         const Where<A>& w) {
  if (drag_mode == DRAG_SPECIES) return sp_inv_tau;
  if (drag_mode == DRAG_STOKES) {
    A R = GEOM == GEOM_SPH ? w.sc[2] : w.x[0];
    return dsqrt(A(f.GM) / (R * R * R)) / dval;
  }
  return A(1) / dval;
}

}  // namespace dust
