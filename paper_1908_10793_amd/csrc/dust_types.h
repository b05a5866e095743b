// Device-side descriptors of the dust hot path (built by the host from the
// public dust_box_t / dust_forces_t; see include/dust.h).
#pragma once

#include <stdint.h>

#include "../../include/dust.h"

namespace dust {

enum { GEOM_CART = DUST_CART, GEOM_CYL = DUST_CYL, GEOM_SPH = DUST_SPH };
enum { SHAPE_CIC = DUST_CIC, SHAPE_TSC = DUST_TSC, SHAPE_VOL = DUST_VOL };
enum { BC_PERIODIC = DUST_BC_PERIODIC, BC_SHEAR = DUST_BC_SHEAR, BC_OPEN = DUST_BC_OPEN };
enum { FORCE_NONE = DUST_FORCE_NONE, FORCE_SHEARBOX = DUST_FORCE_SHEARBOX,
       FORCE_POINTMASS = DUST_FORCE_POINTMASS, FORCE_CONST = DUST_FORCE_CONST,
       FORCE_FARGO = DUST_FORCE_SHEARBOX_FARGO };
enum { DRAG_TAU = DUST_DRAG_TAU, DRAG_STOKES = DUST_DRAG_STOKES, DRAG_SPECIES = DUST_DRAG_SPECIES,
       DRAG_EPSTEIN = DUST_DRAG_EPSTEIN };

// Weight formula of an axis: plain b-spline overlap (Cartesian, phi, z),
// cylindrical radius, spherical radius, spherical polar angle.
enum { AX_PLAIN = 0, AX_CYL_R = 1, AX_SPH_R = 2, AX_THETA = 3 };

struct Axis {
  int32_t n, bc_lo, bc_hi, shape, uniform, kind;
  double lo, hi, L, d, inv_d;   // domain and (uniform axes) cell width
  double inv_n;                 // 1/n (index arithmetic)
  const double *faces;          // device: face k at faces[k+1], k = -1 .. n+1
  const double *ivol;           // device: inverse volume factor of cell k at ivol[k+1]
  const double *trig;           // device, polar axis only: sin, cos of the centre of cell k
                                // at trig[2(k+1)], trig[2(k+1)+1]; else null
};

struct Box {
  int32_t geom, ndim;
  int32_t g0, g1, g2;           // stored extents (active + 2 ghosts; 1 for a missing axis)
  int32_t k_off;                // 1 in 3-D, 0 in 2-D
  int64_t cell_base, ncell;     // first global active cell id, active cells
  int64_t store_base, nstore;   // first stored cell in the field arrays, stored cells
  int64_t xg_base;              // shear-periodic boxes: first word of the box's FP64 x-ghost
                                // gas layer (2 sides x 3 components x (n1+2)(n2+2)); else -1
  Axis ax[3];
};

struct Forces {
  int32_t kind, vertical_gravity;
  double Omega, q, GM;
  double g[3];
  int32_t integrator;   // DUST_INTEGRATOR_*
};

#define DUST_MAX_SPECIES 16
struct Species {
  int32_t n;
  double tau[DUST_MAX_SPECIES];
  double inv_tau[DUST_MAX_SPECIES];  // 1/tau (0 for tau = +inf)
  double mass[DUST_MAX_SPECIES];
};

// Device diagnostics block (FP64 sums, counters, sticky flags).
struct DiagDev {
  double p_part[3], p_grid[3];
  double e_part, e_grid, sum_abs_j;
  unsigned long long max_cells_bits;   // max of a non-negative double, as bits
  unsigned long long n_removed, n_fallback;
  unsigned int flags;
  unsigned int steps;
};

}  // namespace dust
