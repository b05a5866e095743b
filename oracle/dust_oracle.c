/*
 * dust_oracle.c -- plain, serial FP64 reference of one step of the
 * dust-particle hot path of Mignone, Flock & Vaidya, "A Particle Module for
 * the PLUTO Code: III - Dust" (arXiv:1908.10793).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it (through oracle/__init__.py).  It
 * shares no code, header, table or constant with the HIP library.
 *
 * Design rules: FP64 everywhere, global coordinates (not cell + offset),
 * one particle at a time in index order, every weight evaluated from its
 * definition as an overlap integral (Gauss-Legendre quadrature of the shape
 * function, Eq. weight / shape_cart / shape_curv of Sec. 3.4), the paper's
 * closed forms kept separately for cross-checks only.  Readings of the paper
 * where it is silent or garbled are marked "reading:".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

enum { G_CART = 0, G_CYL = 1, G_SPH = 2 };
enum { BC_PERIODIC = 0, BC_SHEAR = 1, BC_OPEN = 2 };
enum { SH_CIC = 0, SH_TSC = 1, SH_VOL = 2 };
enum { F_NONE = 0, F_SHEARBOX = 1, F_POINTMASS = 2, F_CONST = 3, F_SHEARBOX_FARGO = 4 };
enum { DRAG_TAU = 0, DRAG_STOKES = 1, DRAG_EPSTEIN = 2 };

typedef struct {
  int32_t geom, ndim;
  int32_t n[3];
  int32_t bc_lo[3], bc_hi[3];
  int32_t shape[3];
  const double *faces[3];
} orc_box;

typedef struct {
  int32_t kind;
  int32_t vertical_gravity;
  double Omega, q, GM;
  double g[3];
  int32_t integrator;   /* 0 exponential midpoint, 1 semi-implicit (Cartesian) */
} orc_forces;

/* Particle set in global FP64 coordinates.  p[] are canonical momenta:
 * Cartesian (vx,vy,vz); cylindrical (v_R, l_phi = R v_phi, v_z);
 * spherical (v_r, l_theta = r v_theta, l_phi = r sin(theta) v_phi)
 * (Eq. dust_cylindrical, dust_spherical). */
typedef struct {
  int64_t n;
  double *x[3];
  double *p[3];
  const double *drag;  /* tau (DRAG_TAU, +inf allowed), St (DRAG_STOKES) or
                          rho_s a / v_t (DRAG_EPSTEIN) */
  const double *mass;
  int32_t *active;     /* 1 active, 0 removed through an open face */
} orc_particles;

/* Ghosted cell-centred fields, (n0+2)(n1+2)(n2+2) (an absent third axis has
 * extent 1 and no ghosts).  dep[] are the ndim momentum channels then the
 * energy channel. */
typedef struct {
  double *rho;
  double *vel[3];
  double *dep[4];
} orc_fields;

typedef struct {
  double p_part[3], p_grid[3];
  double e_part, e_grid;
  double sum_abs_j;
  double max_cells_per_step;
  int64_t n_inactive;
} orc_diag;

/* ------------------------------------------------------------------ */
/* Gauss-Legendre nodes on [-1,1], found by Newton iteration on P_n.   */

#define GL_N 16
static double gl_x[GL_N], gl_w[GL_N];
static int gl_ready = 0;

static void gl_init(void) {
  if (gl_ready) return;
  for (int i = 0; i < GL_N; ++i) {
    double x = cos(ORC_PI * (i + 0.75) / (GL_N + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= GL_N; ++k) {
        double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = GL_N * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    gl_x[i] = x;
    gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  gl_ready = 1;
}

/* Integral of f over [a,b] with the GL_N-point rule. */
static double gl_integrate(double (*f)(double, const void *), const void *ctx,
                           double a, double b) {
  gl_init();
  if (!(b > a)) return 0.0;
  double c = 0.5 * (a + b), h = 0.5 * (b - a), s = 0.0;
  for (int i = 0; i < GL_N; ++i) s += gl_w[i] * f(c + h * gl_x[i], ctx);
  return s * h;
}

double orc_gl_integrate_poly(const double *coef, int deg, double a, double b);

/* ------------------------------------------------------------------ */
/* Grid geometry.                                                      */

/* Face k of axis d, k in [-1, n+1]: the ghost cell on either side has the
 * width of the active cell next to it (reading: the paper does not define
 * ghost geometry). */
static double face(const orc_box *b, int d, int k) {
  int n = b->n[d];
  const double *f = b->faces[d];
  if (k < 0) return f[0] - (f[1] - f[0]);
  if (k > n) return f[n] + (f[n] - f[n - 1]);
  return f[k];
}

static int extent(const orc_box *b, int d) { return d < b->ndim ? b->n[d] + 2 : 1; }

/* Ghosted linear index of active-grid cell (i,j,k), each in [-1, n]. */
static int64_t gidx(const orc_box *b, int i, int j, int k) {
  int g0 = extent(b, 0), g1 = extent(b, 1);
  int o2 = b->ndim > 2 ? 1 : 0;
  return (int64_t)(i + 1) + (int64_t)g0 * ((j + 1) + (int64_t)g1 * (k + o2));
}

static int64_t n_ghosted(const orc_box *b) {
  return (int64_t)extent(b, 0) * extent(b, 1) * extent(b, 2);
}

/* Volume of cell (i,j,k) from its faces (Sec. 3.1: Delta V of Eq. Lop). */
static double cell_volume(const orc_box *b, int i, int j, int k) {
  double a0 = face(b, 0, i), b0 = face(b, 0, i + 1);
  double a1 = face(b, 1, j), b1 = face(b, 1, j + 1);
  double a2 = 0.0, b2 = 1.0;
  if (b->ndim > 2) { a2 = face(b, 2, k); b2 = face(b, 2, k + 1); }
  switch (b->geom) {
    case G_CYL: return 0.5 * (b0 * b0 - a0 * a0) * (b1 - a1) * (b2 - a2);
    case G_SPH: return (b0 * b0 * b0 - a0 * a0 * a0) / 3.0 * (cos(a1) - cos(b1)) * (b2 - a2);
    default: return (b0 - a0) * (b1 - a1) * (b2 - a2);
  }
}

double orc_cell_volume(const orc_box *b, int i, int j, int k) { return cell_volume(b, i, j, k); }

/* Active cell i with faces f_i <= xi < f_{i+1} (half-open ownership), or -1. */
int orc_locate(const orc_box *b, int d, double xi) {
  const double *f = b->faces[d];
  int n = b->n[d];
  if (!(xi >= f[0]) || !(xi < f[n])) return -1;
  int lo = 0, hi = n; /* invariant f[lo] <= xi < f[hi] */
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (xi >= f[mid]) lo = mid; else hi = mid;
  }
  return lo;
}

/* Metric factor J of the volume element along axis d (d^3x = J1 J2 J3 dx):
 * cylindrical R dR dphi dz, spherical r^2 sin(theta) dr dtheta dphi. */
static double metric(int geom, int d, double xi) {
  if (geom == G_CYL && d == 0) return xi;
  if (geom == G_SPH && d == 0) return xi * xi;
  if (geom == G_SPH && d == 1) return sin(xi);
  return 1.0;
}

/* ------------------------------------------------------------------ */
/* Weights from their definition (Eq. weight with Eq. shape_cart /      */
/* shape_curv, splines Eq. b0 and b1).                                  */

typedef struct { int geom, d, shape; double xp, width; } shape_ctx;

/* b_0: top hat of unit width; b_1: unit triangle (Eq. b0, b1). */
static double spline(int shape, double u) {
  double a = fabs(u);
  if (shape == SH_CIC) return a < 0.5 ? 1.0 : 0.0;
  return a < 1.0 ? 1.0 - a : 0.0;
}

static double shape_integrand(double xi, const void *vctx) {
  const shape_ctx *c = (const shape_ctx *)vctx;
  return spline(c->shape, (xi - c->xp) / c->width) * metric(c->geom, c->d, xi);
}

/* Integral of b_m((xi - xp)/width) J(xi) over [lo, hi], split at the
 * spline's break points so that each piece is smooth. */
static double shape_overlap(const shape_ctx *c, double lo, double hi) {
  double half = c->shape == SH_CIC ? 0.5 * c->width : c->width;
  double a = fmax(lo, c->xp - half), z = fmin(hi, c->xp + half);
  if (!(z > a)) return 0.0;
  double s = 0.0;
  if (c->shape == SH_TSC && c->xp > a && c->xp < z) {
    s += gl_integrate(shape_integrand, c, a, c->xp);
    s += gl_integrate(shape_integrand, c, c->xp, z);
  } else {
    s += gl_integrate(shape_integrand, c, a, z);
  }
  return s;
}

/* Weights of host cell i and its two neighbours along axis d for a particle
 * at xi_p.  The shape's width is the host cell's width.  Reading: the part of
 * the shape beyond the host cell's lower (upper) face is given to the lower
 * (upper) neighbour, so the support is exactly the 3-zone stencil of Sec. 3.1
 * and the weights add up to one (Eq. shape_norm); on uniform grids this is
 * the plain overlap, since the shape never reaches farther.  The normalising
 * integral over the whole shape plays the role of a/Delta V_p (Eq.
 * shape_curv). */
void orc_weights_axis(const orc_box *b, int d, int i, double xi_p, double w[3]) {
  double fl = face(b, d, i), fh = face(b, d, i + 1);
  if (b->shape[d] == SH_VOL) {
    /* Volume weighting of the cylindrical radius (Eq. CIC_vol): linear
     * interpolation in R^2 between the two cell centres around R_p. */
    double c = 0.5 * (fl + fh);
    w[0] = w[1] = w[2] = 0.0;
    if (xi_p < c) {
      double cl = 0.5 * (face(b, d, i - 1) + fl);
      w[0] = (c * c - xi_p * xi_p) / (c * c - cl * cl);
      w[1] = 1.0 - w[0];
    } else {
      double ch = 0.5 * (fh + face(b, d, i + 2));
      w[2] = (xi_p * xi_p - c * c) / (ch * ch - c * c);
      w[1] = 1.0 - w[2];
    }
    return;
  }
  shape_ctx c = {b->geom, d, b->shape[d], xi_p, fh - fl};
  double big = 4.0 * (fh - fl);
  double norm = shape_overlap(&c, xi_p - big, xi_p + big);
  w[0] = shape_overlap(&c, xi_p - big, fl) / norm;
  w[1] = shape_overlap(&c, fl, fh) / norm;
  w[2] = shape_overlap(&c, fh, xi_p + big) / norm;
}

/* Overlap of the shape with an arbitrary cell k (any k, also outside the
 * 3-zone stencil): used by the brute-force tests on uniform grids. */
double orc_weight_any_cell(const orc_box *b, int d, int i_host, double xi_p, int k) {
  double fl = face(b, d, i_host), fh = face(b, d, i_host + 1);
  shape_ctx c = {b->geom, d, b->shape[d], xi_p, fh - fl};
  double big = 4.0 * (fh - fl);
  double norm = shape_overlap(&c, xi_p - big, xi_p + big);
  const double *f = b->faces[d];
  int n = b->n[d];
  if (k < 0 || k >= n) return 0.0;
  return shape_overlap(&c, f[k], f[k + 1]) / norm;
}

/* The paper's closed forms, kept apart from the definition above and used
 * only to cross-check it.  delta = (xi_p - x_i)/Delta with x_i the cell centre
 * (Sec. 3.4.1); for the theta axis delta is the angle xi_p - x_i.
 * kind: 0 Cartesian (Eq. b0/b1 integrated), 1 cylindrical R (Eq.
 * CIC_cylindrical, TSC_cylindrical), 2 spherical r (Eq. CIC_spherical_r,
 * TSC_spherical_r), 3 spherical theta CIC (Eq. CIC_spherical_theta with the
 * sign of its minus branch corrected).  nu = x_i/Delta; for kind 3 xlo/xhi
 * are the host-cell faces. */
void orc_weights_paper(int kind, int shape, double delta, double nu, double xlo,
                       double xhi, double w[3]) {
  double ad = fabs(delta);
  if (kind == 0) {
    if (shape == SH_CIC) {
      w[1] = 1.0 - ad;
      w[0] = 0.5 * (ad - delta);
      w[2] = 0.5 * (ad + delta);
    } else {
      w[1] = 0.75 - delta * delta;
      w[0] = 0.5 * (0.5 - delta) * (0.5 - delta);
      w[2] = 0.5 * (0.5 + delta) * (0.5 + delta);
    }
  } else if (kind == 1) {
    if (shape == SH_CIC) {
      double den = 2.0 * delta + 2.0 * nu;
      w[1] = (delta + 2.0 * nu) / den * (1.0 - ad);
      w[2] = (delta + 2.0 * nu + 1.0) / den * 0.5 * (ad + delta);
      w[0] = (delta + 2.0 * nu - 1.0) / den * 0.5 * (ad - delta);
    } else {
      double den = 3.0 * delta + 3.0 * nu;
      w[1] = (delta + 3.0 * nu) / den * (0.75 - delta * delta);
      w[2] = (delta + 3.0 * nu + 2.0) / den * 0.5 * (0.5 + delta) * (0.5 + delta);
      w[0] = (delta + 3.0 * nu - 2.0) / den * 0.5 * (0.5 - delta) * (0.5 - delta);
    }
  } else if (kind == 2) {
    if (shape == SH_CIC) {
      double den = 12.0 * (delta + nu) * (delta + nu) + 1.0;
      w[1] = (3.0 * (delta + 2.0 * nu) * (delta + 2.0 * nu) + (ad - 1.0) * (ad - 1.0)) / den *
             (1.0 - ad);
      double tp = 2.0 * delta + 3.0 * nu + 1.5, tm = 2.0 * delta + 3.0 * nu - 1.5;
      w[2] = (tp * tp + 3.0 * (nu + 0.5) * (nu + 0.5)) / den * 0.5 * (ad + delta);
      w[0] = (tm * tm + 3.0 * (nu - 0.5) * (nu - 0.5)) / den * 0.5 * (ad - delta);
    } else {
      double den = 6.0 * (delta + nu) * (delta + nu) + 1.0;
      double s = delta + 2.0 * nu;
      w[1] = ((s * s + 2.0 * nu * nu + 0.75) * (0.75 - delta * delta) - 0.25) / den;
      w[2] = (delta * delta + (4.0 * nu + 3.0) * delta + 6.0 * nu * nu + 8.0 * nu + 2.75) / den *
             0.5 * (0.5 + delta) * (0.5 + delta);
      w[0] = (delta * delta + (4.0 * nu - 3.0) * delta + 6.0 * nu * nu - 8.0 * nu + 2.75) / den *
             0.5 * (0.5 - delta) * (0.5 - delta);
    }
  } else {
    /* theta, CIC: here delta is an angle */
    double den = cos(xlo + delta) - cos(xhi + delta);
    if (delta > 0) {
      w[1] = (cos(xlo + delta) - cos(xhi)) / den;
      w[2] = (cos(xhi) - cos(xhi + delta)) / den;
      w[0] = 0.0;
    } else {
      w[1] = (cos(xlo) - cos(xhi + delta)) / den;
      w[0] = -(cos(xlo) - cos(xlo + delta)) / den;
      w[2] = 0.0;
    }
  }
}

/* ------------------------------------------------------------------ */
/* Ghost cells (reading of the shear-periodic rule of Sec. 2.1: the two */
/* radial sides are offset in y by q Omega L_x t).                      */

static int wrapi(int j, int n) { j %= n; return j < 0 ? j + n : j; }

/* Shear offset in y-cells at time t, reduced to [0, n_y). */
static double shear_cells(const orc_box *b, const orc_forces *f, double t) {
  double lx = b->faces[0][b->n[0]] - b->faces[0][0];
  double dy = b->faces[1][1] - b->faces[1][0];
  double s = f->q * f->Omega * lx * t / dy;
  s = fmod(s, (double)b->n[1]);
  if (s < 0) s += b->n[1];
  return s;
}

/* Fill the ghosts of periodic and shear-periodic axes (open-axis ghosts are
 * left as the caller filled them).  Order: x, then y over all x, then z over
 * all x and y, so edges and corners are consistent. */
static void fill_ghosts_one(const orc_box *b, const orc_forces *f, double t, double *a,
                            int comp_vy) {
  int n0 = b->n[0], n1 = b->n[1], n2 = b->ndim > 2 ? b->n[2] : 1;
  int k0 = 0, k1 = n2;
  /* axis 0 */
  if (b->bc_lo[0] == BC_SHEAR) {
    double s = shear_cells(b, f, t);
    double u = f->q * f->Omega * (b->faces[0][n0] - b->faces[0][0]);
    for (int k = k0; k < k1; ++k)
      for (int j = 0; j < n1; ++j) {
        /* right ghost (x_0 + L_x, y_j) is the image of (x_0, y_j + s) */
        double pos = j + s;
        int jl = (int)floor(pos);
        double fr = pos - jl;
        double v = (1.0 - fr) * a[gidx(b, 0, wrapi(jl, n1), k)] +
                   fr * a[gidx(b, 0, wrapi(jl + 1, n1), k)];
        a[gidx(b, n0, j, k)] = v - (comp_vy ? u : 0.0);
        /* left ghost (x_{n-1} - L_x, y_j) is the image of (x_{n-1}, y_j - s) */
        pos = j - s;
        jl = (int)floor(pos);
        fr = pos - jl;
        v = (1.0 - fr) * a[gidx(b, n0 - 1, wrapi(jl, n1), k)] +
            fr * a[gidx(b, n0 - 1, wrapi(jl + 1, n1), k)];
        a[gidx(b, -1, j, k)] = v + (comp_vy ? u : 0.0);
      }
  } else if (b->bc_lo[0] == BC_PERIODIC) {
    for (int k = k0; k < k1; ++k)
      for (int j = 0; j < n1; ++j) {
        a[gidx(b, -1, j, k)] = a[gidx(b, n0 - 1, j, k)];
        a[gidx(b, n0, j, k)] = a[gidx(b, 0, j, k)];
      }
  }
  /* axis 1 */
  if (b->bc_lo[1] == BC_PERIODIC)
    for (int k = k0; k < k1; ++k)
      for (int i = -1; i <= n0; ++i) {
        a[gidx(b, i, -1, k)] = a[gidx(b, i, n1 - 1, k)];
        a[gidx(b, i, n1, k)] = a[gidx(b, i, 0, k)];
      }
  /* axis 2 */
  if (b->ndim > 2 && b->bc_lo[2] == BC_PERIODIC)
    for (int j = -1; j <= n1; ++j)
      for (int i = -1; i <= n0; ++i) {
        a[gidx(b, i, j, -1)] = a[gidx(b, i, j, n2 - 1)];
        a[gidx(b, i, j, n2)] = a[gidx(b, i, j, 0)];
      }
}

void orc_fill_ghosts(const orc_box *b, const orc_forces *f, double t, orc_fields *fl) {
  int nc = b->ndim;
  fill_ghosts_one(b, f, t, fl->rho, 0);
  for (int c = 0; c < nc; ++c)
    fill_ghosts_one(b, f, t, fl->vel[c], b->geom == G_CART && c == 1 && b->bc_lo[0] == BC_SHEAR &&
                                             f->kind == F_SHEARBOX);
}

/* Fold deposits made into periodic / shear-periodic ghosts back onto their
 * partners: the exact transpose of the fill, applied in the reverse axis
 * order, then zero those ghosts.  The energy channel crossing a shear face
 * gains u * D_y, the work of the momentum change in the partner's frame
 * (reading: the gas kinetic energy differs by the boost u = q Omega L_x).
 * With orbital advection (Eq. FARGO_SB_p) velocities are residuals, which
 * carry no boost across the face: no energy term. */
void orc_fold_ghosts(const orc_box *b, const orc_forces *f, double t, orc_fields *fl) {
  int nc = b->ndim;
  int n0 = b->n[0], n1 = b->n[1], n2 = b->ndim > 2 ? b->n[2] : 1;
  for (int c = 0; c <= nc; ++c) {
    double *a = fl->dep[c];
    if (b->ndim > 2 && b->bc_lo[2] == BC_PERIODIC)
      for (int j = -1; j <= n1; ++j)
        for (int i = -1; i <= n0; ++i) {
          a[gidx(b, i, j, n2 - 1)] += a[gidx(b, i, j, -1)];
          a[gidx(b, i, j, 0)] += a[gidx(b, i, j, n2)];
          a[gidx(b, i, j, -1)] = 0.0;
          a[gidx(b, i, j, n2)] = 0.0;
        }
    if (b->bc_lo[1] == BC_PERIODIC)
      for (int k = 0; k < n2; ++k)
        for (int i = -1; i <= n0; ++i) {
          a[gidx(b, i, n1 - 1, k)] += a[gidx(b, i, -1, k)];
          a[gidx(b, i, 0, k)] += a[gidx(b, i, n1, k)];
          a[gidx(b, i, -1, k)] = 0.0;
          a[gidx(b, i, n1, k)] = 0.0;
        }
  }
  if (b->bc_lo[0] == BC_SHEAR) {
    double s = shear_cells(b, f, t);
    double u = f->kind == F_SHEARBOX ? f->q * f->Omega * (b->faces[0][n0] - b->faces[0][0]) : 0.0;
    double *dy = fl->dep[1];
    for (int k = 0; k < n2; ++k)
      for (int j = 0; j < n1; ++j) {
        double gr_y = dy[gidx(b, n0, j, k)], gl_y = dy[gidx(b, -1, j, k)];
        for (int c = 0; c <= nc; ++c) {
          double *a = fl->dep[c];
          double vr = a[gidx(b, n0, j, k)], vl = a[gidx(b, -1, j, k)];
          if (c == nc) { vr += u * gr_y; vl -= u * gl_y; }
          double pos = j + s;
          int jl = (int)floor(pos);
          double fr = pos - jl;
          a[gidx(b, 0, wrapi(jl, n1), k)] += (1.0 - fr) * vr;
          a[gidx(b, 0, wrapi(jl + 1, n1), k)] += fr * vr;
          pos = j - s;
          jl = (int)floor(pos);
          fr = pos - jl;
          a[gidx(b, n0 - 1, wrapi(jl, n1), k)] += (1.0 - fr) * vl;
          a[gidx(b, n0 - 1, wrapi(jl + 1, n1), k)] += fr * vl;
        }
        for (int c = 0; c <= nc; ++c) {
          fl->dep[c][gidx(b, n0, j, k)] = 0.0;
          fl->dep[c][gidx(b, -1, j, k)] = 0.0;
        }
      }
  } else if (b->bc_lo[0] == BC_PERIODIC) {
    for (int c = 0; c <= nc; ++c) {
      double *a = fl->dep[c];
      for (int k = 0; k < n2; ++k)
        for (int j = 0; j < n1; ++j) {
          a[gidx(b, n0 - 1, j, k)] += a[gidx(b, -1, j, k)];
          a[gidx(b, 0, j, k)] += a[gidx(b, n0, j, k)];
          a[gidx(b, -1, j, k)] = 0.0;
          a[gidx(b, n0, j, k)] = 0.0;
        }
    }
  }
}

/* ------------------------------------------------------------------ */
/* Particle boundary handling after a drift.                            */

/* Bring x back into the domain at time t: periodic images, the
 * shear-periodic image (x -/+ L_x, y +/- q Omega L_x t, v_y +/- q Omega L_x;
 * with orbital advection the residual v_y is continuous: no boost) and
 * removal through open faces (reading; the paper removes particles that
 * leave a global disk). Returns 0 if the particle was removed. */
static int wrap_particle(const orc_box *b, const orc_forces *f, double t, double x[3],
                         double p[3]) {
  for (int d = 0; d < b->ndim; ++d) {
    const double *fc = b->faces[d];
    double lo = fc[0], hi = fc[b->n[d]], L = hi - lo;
    if (x[d] >= lo && x[d] < hi) continue;
    int bc = x[d] < lo ? b->bc_lo[d] : b->bc_hi[d];
    if (bc == BC_OPEN) return 0;
    if (bc == BC_SHEAR) {
      double u = f->q * f->Omega * L;
      double sy = u * t, boost = f->kind == F_SHEARBOX ? u : 0.0;
      while (x[0] >= hi) { x[0] -= L; x[1] += sy; p[1] += boost; }
      while (x[0] < lo) { x[0] += L; x[1] -= sy; p[1] -= boost; }
    } else {
      double r = fmod(x[d] - lo, L);
      if (r < 0) r += L;
      x[d] = lo + r;
      if (x[d] >= hi) x[d] = lo;
    }
  }
  return 1;
}

/* ------------------------------------------------------------------ */
/* Drift (Eq. exp_midpoint; Eq. drift1_cylindrical / drift2_cylindrical; */
/* App. B.2 drifts).  h = dt/2.  In the first drift the angles use the    */
/* radius (and theta) already advanced to n+1/2; in the second drift all  */
/* metric factors are those of level n+1/2, frozen before the update.     */

/* Orbital advection (Eq. FARGO_SB_p): p holds the residual velocity v' and
 * y is also carried by the mean shear -q Omega x; reading: the shear term
 * takes x^{n+1/2}, so x moves first in the first drift and last in the
 * second (as the radius does in the curvilinear drifts). */
static void drift_first(int geom, const orc_forces *f, double h, double x[3], const double p[3]) {
  if (geom == G_CART && f->kind == F_SHEARBOX_FARGO) {
    x[0] += h * p[0];
    x[1] += h * (p[1] - f->q * f->Omega * x[0]);
    x[2] += h * p[2];
  } else if (geom == G_CART) {
    for (int d = 0; d < 3; ++d) x[d] += h * p[d];
  } else if (geom == G_CYL) {
    x[0] += h * p[0];
    x[1] += h * p[1] / (x[0] * x[0]);
    x[2] += h * p[2];
  } else {
    x[0] += h * p[0];
    x[1] += h * p[1] / (x[0] * x[0]);
    double s = sin(x[1]);
    x[2] += h * p[2] / (x[0] * x[0] * s * s);
  }
}

static void drift_second(int geom, const orc_forces *f, double h, double x[3], const double p[3]) {
  if (geom == G_CART && f->kind == F_SHEARBOX_FARGO) {
    x[1] += h * (p[1] - f->q * f->Omega * x[0]);
    x[0] += h * p[0];
    x[2] += h * p[2];
  } else if (geom == G_CART) {
    for (int d = 0; d < 3; ++d) x[d] += h * p[d];
  } else if (geom == G_CYL) {
    double R = x[0];
    x[1] += h * p[1] / (R * R);
    x[0] += h * p[0];
    x[2] += h * p[2];
  } else {
    double r = x[0], s = sin(x[1]);
    x[2] += h * p[2] / (r * r * s * s);
    x[1] += h * p[1] / (r * r);
    x[0] += h * p[0];
  }
}

/* ------------------------------------------------------------------ */
/* Exponential-midpoint kick (Eq. exp_midpoint, h1, kick_modified; App.   */
/* B.1 Eq. standard_SB_exp_midpoint; App. B.2 Eq. kick_cylindrical and    */
/* its spherical analogue).                                               */

/* Inputs: position x at n+1/2, canonical momenta p (level n), canonical gas
 * momenta pg at the particle, inverse stopping time, dt.  Outputs: p at
 * n+1 (in place) and a[] = the non-drag part of G evaluated as in the kick
 * (the a_p^{n+1/2} of Eq. dust_feedback_final). */
/* Semi-implicit kick (Sec. 3.2, Eq. semi-implicit, a_linear, Lambda; the
 * comparison integrator of BS10), Cartesian: Lambda dv = dt a_tot(x, v^n,
 * v_g) with Lambda = I - (dt/2) d a_tot / d v, solved by Gaussian
 * elimination; a = the non-drag acceleration at (v^n + v^{n+1})/2 (linear
 * in v, so exactly the non-drag part of the linearised a_tot^{n+1/2}). */
static void kick_semi_implicit(int ndim, const orc_forces *f, double dt, double inv_tau,
                               const double x[3], double p[3], const double pg[3], double a[3]) {
  double Om = f->Omega, q = f->q;
  double ae[3] = {0, 0, 0}, Ja[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  if (ndim == 3 && f->kind == F_SHEARBOX) {
    ae[0] = 2.0 * Om * (p[1] + q * Om * x[0]);
    ae[1] = -2.0 * Om * p[0];
    Ja[0][1] = 2.0 * Om;
    Ja[1][0] = -2.0 * Om;
  } else if (ndim == 3 && f->kind == F_SHEARBOX_FARGO) {
    ae[0] = 2.0 * Om * p[1];
    ae[1] = (q - 2.0) * Om * p[0];
    Ja[0][1] = 2.0 * Om;
    Ja[1][0] = (q - 2.0) * Om;
  } else if (f->kind == F_CONST) {
    for (int d = 0; d < 3; ++d) ae[d] = f->g[d];
  }
  if ((f->kind == F_SHEARBOX || f->kind == F_SHEARBOX_FARGO) && f->vertical_gravity && ndim == 3)
    ae[2] = -Om * Om * x[2];
  double M[3][4];
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) M[r][k] = (r == k ? 1.0 + 0.5 * dt * inv_tau : 0.0) - 0.5 * dt * Ja[r][k];
    M[r][3] = dt * (ae[r] + (pg[r] - p[r]) * inv_tau);
  }
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
    if (piv != col)
      for (int k = 0; k < 4; ++k) { double tmp = M[col][k]; M[col][k] = M[piv][k]; M[piv][k] = tmp; }
    for (int r = col + 1; r < 3; ++r) {
      double fct = M[r][col] / M[col][col];
      for (int k = col; k < 4; ++k) M[r][k] -= fct * M[col][k];
    }
  }
  double dv[3];
  for (int r = 2; r >= 0; --r) {
    double s = M[r][3];
    for (int k = r + 1; k < 3; ++k) s -= M[r][k] * dv[k];
    dv[r] = s / M[r][r];
  }
  for (int d = ndim; d < 3; ++d) dv[d] = 0.0;
  for (int d = 0; d < 3; ++d) {
    /* non-drag acceleration at the mean velocity */
    a[d] = ae[d];
    for (int k = 0; k < 3; ++k) a[d] += 0.5 * Ja[d][k] * dv[k];
    p[d] += dv[d];
  }
}

static void kick(int geom, int ndim, const orc_forces *f, double dt, double inv_tau,
                 const double x[3], double p[3], const double pg[3], double a[3]) {
  if (f->integrator == 1 && geom == G_CART) {
    kick_semi_implicit(ndim, f, dt, inv_tau, x, p, pg, a);
    return;
  }
  double hh = dt * inv_tau;                       /* Delta t / tau_s          */
  double e = exp(-hh);                            /* e^{A Delta t}            */
  double c = -expm1(-hh);                         /* 1 - e = h1 / tau_s       */
  double h1 = inv_tau > 0 ? c / inv_tau : dt;     /* Eq. h1; tau = inf: dt    */
  int nc = geom == G_CART ? ndim : 3;
  double p0[3] = {p[0], p[1], p[2]};

  if (geom == G_CART && f->kind == F_SHEARBOX_FARGO) {
    /* Orbital advection (App. B.1, Eq. FARGO_SB_exp_midpoint): residual
     * velocities, G(x, v', v'_g) = (2 Omega v'_y, (q - 2) Omega v'_x,
     * -Omega^2 z) + v'_g/tau, kick taken with v' = (v'^n + v'^{n+1})/2:
     * the 2x2 block solved by Cramer's rule. */
    double Om = f->Omega, q = f->q;
    double gz = f->vertical_gravity ? -Om * Om * x[2] : 0.0;
    /* row x: v'_x - h1 Om v'_y = e v_x + h1 Om v_y + c vg_x */
    double a00 = 1.0, a01 = -h1 * Om, r0 = e * p0[0] + h1 * Om * p0[1] + c * pg[0];
    /* row y: v'_y - h1 (q-2) Om v'_x / 2 = e v_y + h1 (q-2) Om v_x / 2 + c vg_y */
    double a10 = -0.5 * h1 * (q - 2.0) * Om, a11 = 1.0;
    double r1 = e * p0[1] + 0.5 * h1 * (q - 2.0) * Om * p0[0] + c * pg[1];
    double det = a00 * a11 - a01 * a10;
    p[0] = (r0 * a11 - a01 * r1) / det;
    p[1] = (a00 * r1 - a10 * r0) / det;
    p[2] = e * p0[2] + h1 * gz + c * pg[2];
    double vbx = 0.5 * (p0[0] + p[0]), vby = 0.5 * (p0[1] + p[1]);
    a[0] = 2.0 * Om * vby;
    a[1] = (q - 2.0) * Om * vbx;
    a[2] = gz;
    return;
  }
  if (geom == G_CART && f->kind == F_SHEARBOX) {
    /* G(x, v, v_g) = (2 Omega (v_y + q Omega x), -2 Omega v_x,
     * -Omega^2 z) + v_g/tau, kick taken with v = (v^n + v^{n+1})/2: solve
     * the 3x3 linear system by Gaussian elimination with pivoting. */
    double Om = f->Omega, q = f->q;
    double gz = f->vertical_gravity ? -Om * Om * x[2] : 0.0;
    double M[3][4];
    /* unknown v' : v' - h1 G(x, (v + v')/2, vg) = e v */
    /* row x: v'_x - h1 Om v'_y = e v_x + h1 (Om v_y + 2 q Om^2 x) + c vg_x */
    M[0][0] = 1.0; M[0][1] = -h1 * Om; M[0][2] = 0.0;
    M[0][3] = e * p0[0] + h1 * (Om * p0[1] + 2.0 * q * Om * Om * x[0]) + c * pg[0];
    /* row y: v'_y + h1 Om v'_x = e v_y - h1 Om v_x + c vg_y */
    M[1][0] = h1 * Om; M[1][1] = 1.0; M[1][2] = 0.0;
    M[1][3] = e * p0[1] - h1 * Om * p0[0] + c * pg[1];
    /* row z */
    M[2][0] = 0.0; M[2][1] = 0.0; M[2][2] = 1.0;
    M[2][3] = e * p0[2] + h1 * gz + c * pg[2];
    for (int col = 0; col < 3; ++col) {
      int piv = col;
      for (int r = col + 1; r < 3; ++r)
        if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
      if (piv != col)
        for (int k = 0; k < 4; ++k) { double tmp = M[col][k]; M[col][k] = M[piv][k]; M[piv][k] = tmp; }
      for (int r = col + 1; r < 3; ++r) {
        double fct = M[r][col] / M[col][col];
        for (int k = col; k < 4; ++k) M[r][k] -= fct * M[col][k];
      }
    }
    double v[3];
    for (int r = 2; r >= 0; --r) {
      double s = M[r][3];
      for (int k = r + 1; k < 3; ++k) s -= M[r][k] * v[k];
      v[r] = s / M[r][r];
    }
    p[0] = v[0]; p[1] = v[1]; p[2] = v[2];
    double vbx = 0.5 * (p0[0] + p[0]), vby = 0.5 * (p0[1] + p[1]);
    a[0] = 2.0 * Om * (vby + q * Om * x[0]);
    a[1] = -2.0 * Om * vbx;
    a[2] = gz;
    return;
  }
  if (geom == G_CART) {
    /* drag plus an optional constant acceleration: G = v_g/tau + g */
    for (int d = 0; d < nc; ++d) {
      double g = f->kind == F_CONST ? f->g[d] : 0.0;
      p[d] = e * p0[d] + h1 * g + c * pg[d];
      a[d] = g;
    }
    return;
  }
  /* point-mass gravity g = -GM x/|x|^3 in the local basis */
  double gr = 0.0, gth = 0.0, gz = 0.0;
  if (geom == G_CYL) {
    double R = x[0], z = x[2];
    if (f->kind == F_POINTMASS) {
      double r3 = pow(R * R + z * z, 1.5);
      gr = -f->GM * R / r3;
      gz = -f->GM * z / r3;
    }
    /* order v_z, l_phi, v_R (App. B.2, cylindrical) */
    p[2] = e * p0[2] + h1 * gz + c * pg[2];
    a[2] = gz;
    double gphi = 0.0; /* axisymmetric potential */
    p[1] = e * p0[1] + h1 * (R * gphi) + c * pg[1];
    a[1] = R * gphi;
    double l2 = 0.5 * (p0[1] * p0[1] + p[1] * p[1]);
    double aR = l2 / (R * R * R) + gr;
    p[0] = e * p0[0] + h1 * aR + c * pg[0];
    a[0] = aR;
    return;
  }
  {
    double r = x[0], th = x[1], s = sin(th), ct = cos(th);
    if (f->kind == F_POINTMASS) gr = -f->GM / (r * r);
    /* order l_phi, l_theta, v_r (App. B.2, spherical); the second average in the
     * printed midpoint formula is read as (l_theta^2)^{n+1/2}. */
    double gphi = 0.0; /* axisymmetric potential, g_theta = 0 too */
    p[2] = e * p0[2] + h1 * (r * s * gphi) + c * pg[2];
    a[2] = r * s * gphi;
    double lp2 = 0.5 * (p0[2] * p0[2] + p[2] * p[2]);
    double ath = lp2 * ct / (r * r * s * s * s) + r * gth;
    p[1] = e * p0[1] + h1 * ath + c * pg[1];
    a[1] = ath;
    double lt2 = 0.5 * (p0[1] * p0[1] + p[1] * p[1]);
    double ar = lt2 / (r * r * r) + lp2 / (r * r * r * s * s) + gr;
    p[0] = e * p0[0] + h1 * ar + c * pg[0];
    a[0] = ar;
  }
}

/* Exposed for the unit tests: one kick with a given gathered gas momentum. */
void orc_kick(int geom, int ndim, const orc_forces *f, double dt, double inv_tau,
              const double x[3], double p[3], const double pg[3], double a[3]) {
  kick(geom, ndim, f, dt, inv_tau, x, p, pg, a);
}

/* Physical scale factors of the canonical components at x: v_phys =
 * p / scale (cylindrical l_phi/R; spherical l_theta/r, l_phi/(r sin theta)). */
static void canon_scale(int geom, const double x[3], double sc[3]) {
  sc[0] = sc[1] = sc[2] = 1.0;
  if (geom == G_CYL) sc[1] = x[0];
  if (geom == G_SPH) { sc[1] = x[0]; sc[2] = x[0] * sin(x[1]); }
}

/* rho_p: the gas density weighted to the particle (Epstein regime, Sec. 2:
 * tau_s = rho_s a / (rho_g v_t), the drag value holding rho_s a / v_t). */
static double inverse_tau(int geom, int drag_mode, const orc_forces *f, double dval,
                          const double x[3], double rho_p) {
  if (drag_mode == DRAG_EPSTEIN) return rho_p / dval;
  if (drag_mode == DRAG_STOKES) {
    /* St = tau Omega_K with Omega_K = sqrt(GM/R^3), R the cylindrical radius */
    double R = geom == G_SPH ? x[0] * sin(x[1]) : x[0];
    double omk = sqrt(f->GM / (R * R * R));
    return omk / dval;
  }
  return 1.0 / dval; /* tau = +inf gives 0 */
}

/* ------------------------------------------------------------------ */
/* Gather (Eq. Delta_vp, component by component in the local basis).    */

typedef struct { int cell[3]; double w[3][3]; } stencil;

static int make_stencil(const orc_box *b, const double x[3], stencil *s) {
  for (int d = 0; d < 3; ++d) {
    if (d >= b->ndim) {
      s->cell[d] = 0;
      s->w[d][0] = 0.0; s->w[d][1] = 1.0; s->w[d][2] = 0.0;
      continue;
    }
    int i = orc_locate(b, d, x[d]);
    if (i < 0) return 0;
    s->cell[d] = i;
    orc_weights_axis(b, d, i, x[d], s->w[d]);
  }
  return 1;
}

static void gather(const orc_box *b, const orc_fields *fl, const stencil *s, double *rho_p,
                   double vg[3]) {
  int nc = b->geom == G_CART ? b->ndim : 3;
  double r = 0.0, v[3] = {0, 0, 0};
  int c2 = b->ndim > 2 ? 1 : 0;
  for (int c = -c2; c <= c2; ++c)
    for (int bb = -1; bb <= 1; ++bb)
      for (int a = -1; a <= 1; ++a) {
        double w = s->w[0][a + 1] * s->w[1][bb + 1] * s->w[2][c + 1];
        int64_t id = gidx(b, s->cell[0] + a, s->cell[1] + bb, s->cell[2] + c);
        r += w * fl->rho[id];
        for (int m = 0; m < nc; ++m) v[m] += w * fl->vel[m][id];
      }
  *rho_p = r;
  for (int m = 0; m < 3; ++m) vg[m] = m < nc ? v[m] : 0.0;
}

/* Exposed for tests: weights + gather at global position x. */
int orc_gather(const orc_box *b, const orc_fields *fl, const double x[3], double *rho_p,
               double vg[3]) {
  stencil s;
  if (!make_stencil(b, x, &s)) return 0;
  gather(b, fl, &s, rho_p, vg);
  return 1;
}

/* Deposit q_c (c < nc: momentum channels, c = nc: energy) as densities with
 * the same weights as the gather (Eq. deposition, dust_feedback_final). */
static void deposit(const orc_box *b, orc_fields *fl, const stencil *s, const double *q) {
  int nc = b->geom == G_CART ? b->ndim : 3;
  int c2 = b->ndim > 2 ? 1 : 0;
  for (int c = -c2; c <= c2; ++c)
    for (int bb = -1; bb <= 1; ++bb)
      for (int a = -1; a <= 1; ++a) {
        double w = s->w[0][a + 1] * s->w[1][bb + 1] * s->w[2][c + 1];
        int i = s->cell[0] + a, j = s->cell[1] + bb, k = s->cell[2] + c;
        int64_t id = gidx(b, i, j, k);
        double dv = cell_volume(b, i, j, k);
        for (int m = 0; m <= nc; ++m) fl->dep[m][id] -= w * q[m] / dv;
      }
}

/* ------------------------------------------------------------------ */
/* One full step, serial in particle index order.                       */

enum { STEP_APPLY_FEEDBACK = 1, STEP_FILL_GHOSTS = 2 };

/* The particle part of one step for particles [i0, i1): drift, gather,
 * kick, deposit into fl->dep (which the caller has cleared), drift; the
 * particle sums go to dg. */
static void step_particles(const orc_box *b, const orc_forces *f, int drag_mode, orc_particles *P,
                           orc_fields *fl, double dt, double t, int64_t i0, int64_t i1,
                           orc_diag *dg) {
  int nc = b->geom == G_CART ? b->ndim : 3;
  double h = 0.5 * dt, th = t + h;
  for (int64_t ip = i0; ip < i1; ++ip) {
    if (!P->active[ip]) continue;
    double x[3], p[3], p0[3];
    for (int d = 0; d < 3; ++d) { x[d] = P->x[d][ip]; p[d] = P->p[d][ip]; }
    /* drift by dt/2 to x^{n+1/2} */
    drift_first(b->geom, f, h, x, p);
    if (!wrap_particle(b, f, th, x, p)) {
      P->active[ip] = 0;
      for (int d = 0; d < 3; ++d) { P->x[d][ip] = x[d]; P->p[d][ip] = p[d]; }
      continue;
    }
    for (int d = 0; d < 3; ++d) p0[d] = p[d];
    /* weights and gather at x^{n+1/2} */
    stencil s;
    make_stencil(b, x, &s);
    double rho_p, vg[3], pg[3], sc[3];
    gather(b, fl, &s, &rho_p, vg);
    canon_scale(b->geom, x, sc);
    for (int m = 0; m < 3; ++m) pg[m] = vg[m] * sc[m];
    /* kick */
    double it = inverse_tau(b->geom, drag_mode, f, P->drag[ip], x, rho_p), a[3] = {0, 0, 0};
    kick(b->geom, b->ndim, f, dt, it, x, p, pg, a);
    /* drag impulse J = m (Delta p - dt a) and energy e = m vbar . dv */
    double m = P->mass[ip], q[4], e = 0.0;
    for (int c = 0; c < nc; ++c) {
      double J = m * ((p[c] - p0[c]) - dt * a[c]);
      q[c] = J;
      double vbar = 0.5 * (p0[c] + p[c]) / sc[c];
      e += vbar * (J / sc[c]);
      dg->p_part[c] += J;
      dg->sum_abs_j += fabs(J);
    }
    q[nc] = e;
    dg->e_part += e;
    deposit(b, fl, &s, q);
    /* dust time-step diagnostic (Eq. particles_dt): cells crossed per step */
    for (int d = 0; d < b->ndim; ++d) {
      double dl = face(b, d, s.cell[d] + 1) - face(b, d, s.cell[d]);
      double vb = 0.5 * (p0[d] + p[d]) / sc[d];
      double dlen = dl * (b->geom == G_CART ? 1.0 : (d == 0 ? 1.0 : sc[d]));
      double cps = fabs(vb) * dt / dlen;
      if (cps > dg->max_cells_per_step) dg->max_cells_per_step = cps;
    }
    /* drift by dt/2 to x^{n+1} */
    drift_second(b->geom, f, h, x, p);
    if (!wrap_particle(b, f, t + dt, x, p)) P->active[ip] = 0;
    for (int d = 0; d < 3; ++d) { P->x[d][ip] = x[d]; P->p[d][ip] = p[d]; }
  }
}

/* Grid part of one step after the particles: FP64 conservation sums over
 * every stored cell (before folding), fold, feedback, inactive count. */
static void step_grid(const orc_box *b, const orc_forces *f, orc_particles *P, orc_fields *fl,
                      double dt, double t, int flags, orc_diag *dg);

/* One step; particles in index order on one thread. */
int orc_step(const orc_box *b, const orc_forces *f, int drag_mode, orc_particles *P,
             orc_fields *fl, double dt, double t, int flags, orc_diag *dg) {
  int nc = b->geom == G_CART ? b->ndim : 3;
  int64_t ng = n_ghosted(b);
  memset(dg, 0, sizeof(*dg));
  for (int m = 0; m <= nc; ++m) memset(fl->dep[m], 0, sizeof(double) * ng);
  if (flags & STEP_FILL_GHOSTS) orc_fill_ghosts(b, f, t + 0.5 * dt, fl);
  step_particles(b, f, drag_mode, P, fl, dt, t, 0, P->n, dg);
  step_grid(b, f, P, fl, dt, t, flags, dg);
  return 0;
}

/* The same step on several host threads (OpenMP): thread k of T takes the
 * particles [n k / T, n (k+1) / T) and deposits into a private copy of the
 * deposit arrays; the copies and the particle sums are then added in
 * thread order.  Used to time the reference on every host core; the serial
 * orc_step is the reference of the tests.  Returns the thread count. */
int orc_step_threads(const orc_box *b, const orc_forces *f, int drag_mode, orc_particles *P,
                     orc_fields *fl, double dt, double t, int flags, orc_diag *dg) {
  int nc = b->geom == G_CART ? b->ndim : 3;
  int64_t ng = n_ghosted(b);
  memset(dg, 0, sizeof(*dg));
  for (int m = 0; m <= nc; ++m) memset(fl->dep[m], 0, sizeof(double) * ng);
  if (flags & STEP_FILL_GHOSTS) orc_fill_ghosts(b, f, t + 0.5 * dt, fl);
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
#endif
  double *priv = (double *)calloc((size_t)nt * (nc + 1) * ng, sizeof(double));
  orc_diag *pd = (orc_diag *)calloc((size_t)nt, sizeof(orc_diag));
  if (!priv || !pd) { free(priv); free(pd); return -1; }
#pragma omp parallel num_threads(nt)
  {
    int k = 0;
#ifdef _OPENMP
    k = omp_get_thread_num();
#endif
    orc_fields mine = *fl;
    for (int m = 0; m <= nc; ++m) mine.dep[m] = priv + ((size_t)k * (nc + 1) + m) * ng;
    int64_t i0 = P->n * k / nt, i1 = P->n * (k + 1) / nt;
    step_particles(b, f, drag_mode, P, &mine, dt, t, i0, i1, &pd[k]);
  }
  for (int k = 0; k < nt; ++k) {
    for (int m = 0; m <= nc; ++m) {
      const double *src = priv + ((size_t)k * (nc + 1) + m) * ng;
      for (int64_t i = 0; i < ng; ++i) fl->dep[m][i] += src[i];
    }
    for (int c = 0; c < 3; ++c) dg->p_part[c] += pd[k].p_part[c];
    dg->e_part += pd[k].e_part;
    dg->sum_abs_j += pd[k].sum_abs_j;
    if (pd[k].max_cells_per_step > dg->max_cells_per_step)
      dg->max_cells_per_step = pd[k].max_cells_per_step;
  }
  free(priv);
  free(pd);
  step_grid(b, f, P, fl, dt, t, flags, dg);
  return nt;
}

static void step_grid(const orc_box *b, const orc_forces *f, orc_particles *P, orc_fields *fl,
                      double dt, double t, int flags, orc_diag *dg) {
  int nc = b->geom == G_CART ? b->ndim : 3;
  double th = t + 0.5 * dt;
  /* conservation sums over every stored cell, before folding */
  int n0 = b->n[0], n1 = b->n[1], n2 = b->ndim > 2 ? b->n[2] : 1;
  int g2 = b->ndim > 2 ? 1 : 0;
  for (int k = -g2; k < n2 + g2; ++k)
    for (int j = -1; j <= n1; ++j)
      for (int i = -1; i <= n0; ++i) {
        int64_t id = gidx(b, i, j, k);
        double dv = cell_volume(b, i, j, k);
        for (int c = 0; c < nc; ++c) dg->p_grid[c] += dv * fl->dep[c][id];
        dg->e_grid += dv * fl->dep[nc][id];
      }
  orc_fold_ghosts(b, f, th, fl);

  if (flags & STEP_APPLY_FEEDBACK) {
    /* v_g += D / rho on active cells, canonical channels turned into
     * physical velocity with the cell-centre metric */
    for (int k = 0; k < n2; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n0; ++i) {
          int64_t id = gidx(b, i, j, k);
          double xc[3] = {0.5 * (face(b, 0, i) + face(b, 0, i + 1)),
                          0.5 * (face(b, 1, j) + face(b, 1, j + 1)), 0.0};
          double sc[3];
          canon_scale(b->geom, xc, sc);
          for (int c = 0; c < nc; ++c) fl->vel[c][id] += fl->dep[c][id] / (fl->rho[id] * sc[c]);
        }
  }
  for (int64_t ip = 0; ip < P->n; ++ip) dg->n_inactive += P->active[ip] ? 0 : 1;
}

/* ------------------------------------------------------------------ */
/* Drag source of the gas predictor (Sec. 3.1, Eq. Delta_vp and f_D):    */
/* at the particles' current positions x^n, the slip between the        */
/* weighted gas velocity and the particle velocity, times m_p / tau_s,p, */
/* deposited with the same weights as a force density:                  */
/*   <f_D>_i -= (1/dV_i) sum_p (m_p / tau'_p) W(x_p - x_i) dv_p,          */
/* with the stiffness limiter tau' = max(tau, dt) the paper takes from   */
/* Bai & Stone (2010).  reading: the momentum channels are the canonical */
/* ones of the step's deposit, so the slip is taken between canonical    */
/* momenta at the particle (the phi components become torques, R_p f_phi */
/* or r_p f_theta and r_p sin(theta_p) f_phi).  Accumulates into the     */
/* momentum channels; the energy channel is not touched (the predictor's */
/* source has no energy part).                                           */

void orc_drag_source(const orc_box *b, const orc_forces *f, int drag_mode,
                     const orc_particles *P, orc_fields *fl, double dt) {
  int nc = b->geom == G_CART ? b->ndim : 3;
  int c2 = b->ndim > 2 ? 1 : 0;
  for (int64_t ip = 0; ip < P->n; ++ip) {
    if (!P->active[ip]) continue;
    double x[3] = {P->x[0][ip], P->x[1][ip], P->x[2][ip]};
    stencil s;
    if (!make_stencil(b, x, &s)) continue;
    double rho_p, vg[3], sc[3];
    gather(b, fl, &s, &rho_p, vg);
    canon_scale(b->geom, x, sc);
    double tau = 1.0 / inverse_tau(b->geom, drag_mode, f, P->drag[ip], x, rho_p);
    double tau_lim = tau > dt ? tau : dt;
    double k = P->mass[ip] / tau_lim;
    double q[3];
    for (int m = 0; m < nc; ++m) q[m] = k * (vg[m] * sc[m] - P->p[m][ip]);
    for (int c = -c2; c <= c2; ++c)
      for (int bb = -1; bb <= 1; ++bb)
        for (int a = -1; a <= 1; ++a) {
          double w = s.w[0][a + 1] * s.w[1][bb + 1] * s.w[2][c + 1];
          int i = s.cell[0] + a, j = s.cell[1] + bb, kk = s.cell[2] + c;
          int64_t id = gidx(b, i, j, kk);
          double dv = cell_volume(b, i, j, kk);
          for (int m = 0; m < nc; ++m) fl->dep[m][id] -= w * q[m] / dv;
        }
  }
}

/* ------------------------------------------------------------------ */
/* Dust density on the grid: each particle's mass spread with the same  */
/* weights as the gather and the deposit, as a density (Sec. 3.4: the    */
/* shape function is the particle's density profile; Sec. 4.3.1 compares */
/* the resulting rho_D with eps rho_g).  Accumulates into rho_d (ghosts  */
/* included, to be folded like the deposit).                             */

void orc_deposit_mass(const orc_box *b, const orc_particles *P, double *rho_d) {
  int c2 = b->ndim > 2 ? 1 : 0;
  for (int64_t ip = 0; ip < P->n; ++ip) {
    if (!P->active[ip]) continue;
    double x[3] = {P->x[0][ip], P->x[1][ip], P->x[2][ip]};
    stencil s;
    if (!make_stencil(b, x, &s)) continue;
    for (int c = -c2; c <= c2; ++c)
      for (int bb = -1; bb <= 1; ++bb)
        for (int a = -1; a <= 1; ++a) {
          double w = s.w[0][a + 1] * s.w[1][bb + 1] * s.w[2][c + 1];
          int i = s.cell[0] + a, j = s.cell[1] + bb, k = s.cell[2] + c;
          rho_d[gidx(b, i, j, k)] += w * P->mass[ip] / cell_volume(b, i, j, k);
        }
  }
}

/* ------------------------------------------------------------------ */
/* One particle pushed through gas given as a function of position      */
/* (physical components in the local basis): drift, kick, drift, with no */
/* grid and no boundaries.  For tests against analytic solutions.       */

typedef void (*orc_gas_fn)(const double *x, double *vg);

void orc_push_one(int geom, int ndim, const orc_forces *f, int drag_mode, double dragval,
                  double dt, double *x, double *p, orc_gas_fn gas, double *a_out) {
  double vg[3] = {0, 0, 0}, pg[3], sc[3];
  drift_first(geom, f, 0.5 * dt, x, p);
  if (gas) gas(x, vg);
  canon_scale(geom, x, sc);
  for (int m = 0; m < 3; ++m) pg[m] = vg[m] * sc[m];
  double it = inverse_tau(geom, drag_mode, f, dragval, x, 1.0); /* no grid: unit density */
  kick(geom, ndim, f, dt, it, x, p, pg, a_out);
  drift_second(geom, f, 0.5 * dt, x, p);
}

/* ------------------------------------------------------------------ */
/* Gauss-Legendre check helper: integral of a polynomial (for tests).   */

typedef struct { const double *c; int deg; } poly_ctx;
static double poly_eval(double x, const void *v) {
  const poly_ctx *p = (const poly_ctx *)v;
  double s = 0.0;
  for (int k = p->deg; k >= 0; --k) s = s * x + p->c[k];
  return s;
}
double orc_gl_integrate_poly(const double *coef, int deg, double a, double b) {
  poly_ctx p = {coef, deg};
  return gl_integrate(poly_eval, &p, a, b);
}

int64_t orc_n_ghosted(const orc_box *b) { return n_ghosted(b); }
int64_t orc_gidx(const orc_box *b, int i, int j, int k) { return gidx(b, i, j, k); }
