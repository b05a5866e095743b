/*
 * dust.h -- C ABI of the MI355X (gfx950) dust-particle hot path:
 * field-weighting gather, exponential-midpoint (EM) drag push and
 * momentum/energy feedback deposit of Mignone, Flock & Vaidya (2019),
 * "A Particle Module for the PLUTO Code: III - Dust".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is a DEVICE pointer owned by the caller
 *   (the library never allocates or frees caller memory); descriptor
 *   structs and face arrays are HOST memory and are copied during the call.
 *   Real-valued arrays have the context precision: float for DUST_F32,
 *   double for DUST_F64.  Cell ids are int32.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the legacy
 *   default stream).  Calls are asynchronous on that stream except
 *   dust_ctx_create and dust_ctx_status.  One context per stream; contexts
 *   are not thread safe.
 * Errors.  Every call returns a dust_status_t.  Invalid arguments are found
 *   before anything is launched (DUST_EINVAL / DUST_ESHAPE) and leave all
 *   arrays untouched; the message is in dust_last_error() (per thread).
 *   Anomalies met on the device (non-finite state, an offset outside
 *   [-1/2,1/2), a displacement above 1.8 cells per step, a particle leaving
 *   through an open face, a tile overflow) set sticky bits read by
 *   dust_ctx_status; nothing aborts.
 *
 * Grid.  A context holds one or more boxes.  A box has ndim = 2 (Cartesian
 *   only) or 3 axes; axis 0 varies fastest.  Active cells of a box are
 *   numbered i + n0 (j + n1 k) and offset by the box's first global id (the
 *   sum of the active cells of the boxes before it): that global id is the
 *   particle `cell`; -1 marks a removed particle.  Cell-centred fields are
 *   stored per box with one ghost cell on each side of every axis,
 *   (n0+2)(n1+2)(n2+2) values (2-D: (n0+2)(n1+2)), boxes concatenated in
 *   order; dust_ctx_grid_size gives the sizes.  A ghost cell has the width
 *   of the active cell next to it.  Periodic and shear-periodic axes must be
 *   uniformly spaced.
 *
 * Particles (Sec. 3, a particle carries position, velocity, stopping time
 *   and mass).  Position = host cell + offset delta in [-1/2, 1/2) of the
 *   host-cell width along each axis, the coordinate being
 *   centre_i + delta * width_i.  Momenta are canonical (Eq. dust_cylindrical,
 *   dust_spherical): Cartesian (v_x, v_y, v_z); cylindrical (v_R,
 *   l_phi = R v_phi, v_z); spherical (v_r, l_theta = r v_theta,
 *   l_phi = r sin(theta) v_phi).  Gas velocities are physical components in
 *   the local basis.
 */
#ifndef DUST_H
#define DUST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DUST_OK = 0,
  DUST_EINVAL = -1,       /* invalid argument or descriptor                 */
  DUST_ESHAPE = -2,       /* sizes inconsistent with the context            */
  DUST_ENOMEM = -3,       /* device allocation failed                       */
  DUST_EDEVICE = -4,      /* a HIP call failed                              */
  DUST_EUNSUPPORTED = -5  /* valid but not implemented combination         */
} dust_status_t;

enum { DUST_CART = 0, DUST_CYL = 1, DUST_SPH = 2 };          /* Sec. 2      */
enum { DUST_CIC = 0, DUST_TSC = 1, DUST_VOL = 2 };  /* Eq. b0, b1; Eq. CIC_vol */
enum { DUST_F32 = 0, DUST_F64 = 1 };                          /* storage     */
enum { DUST_ARITH_F64 = 0, DUST_ARITH_F32 = 1 };              /* push math   */
enum { DUST_BC_PERIODIC = 0, DUST_BC_SHEAR = 1, DUST_BC_OPEN = 2 };
enum { DUST_FORCE_NONE = 0, DUST_FORCE_SHEARBOX = 1, DUST_FORCE_POINTMASS = 2,
       DUST_FORCE_CONST = 3, DUST_FORCE_SHEARBOX_FARGO = 4 };
enum { DUST_DRAG_TAU = 0, DUST_DRAG_STOKES = 1, DUST_DRAG_SPECIES = 2, DUST_DRAG_EPSTEIN = 3 };
/* Kick of the drift-kick-drift step: the exponential midpoint (Eq.
 * exp_midpoint, the method of the paper), or the semi-implicit kick of Sec.
 * 3.2 (Eq. semi-implicit with Eq. a_linear and the Lambda matrices), kept for
 * comparison: Cartesian boxes and the unfused step / phase calls only
 * (DUST_EUNSUPPORTED otherwise). */
enum { DUST_INTEGRATOR_EXPMID = 0, DUST_INTEGRATOR_SEMI_IMPLICIT = 1 };
enum { DUST_PHASE_DRIFT1 = 1, DUST_PHASE_KICK = 2, DUST_PHASE_DRIFT2 = 4 };
enum { DUST_BIN_CELL = 0, DUST_BIN_TILE = 1 };

/* dust_step flags */
enum {
  DUST_STEP_APPLY_FEEDBACK = 1,  /* v_g += D / rho after every step          */
  DUST_STEP_FUSED = 2,           /* tiled fused kernel (else the unfused chain) */
  DUST_STEP_DIAG = 4,            /* accumulate FP64 conservation sums        */
  DUST_STEP_GRAPH = 8,           /* capture the nsteps loop in a hipGraph    */
  DUST_STEP_NO_FILL = 16         /* caller already filled the gas ghosts     */
};
/* rebin interval of the fused path, packed in bits 8..15 of the flags */
#define DUST_STEP_REBIN_EVERY(k) (((int32_t)(k) & 0xff) << 8)

/* sticky device flags (dust_diag_t.flags) */
enum {
  DUST_FLAG_NONFINITE = 1,       /* NaN/Inf met in a particle's state        */
  DUST_FLAG_OFFSET_RANGE = 2,    /* an input offset outside [-1/2, 1/2)      */
  DUST_FLAG_CFL = 4,             /* more than 1.8 cells in one step (Eq. particles_dt) */
  DUST_FLAG_LEFT_OPEN = 8,       /* a particle left through an open face     */
  DUST_FLAG_TILE_OVERFLOW = 16,  /* fused path: particle outside its tile halo
                                    (handled by the global fallback)          */
  DUST_FLAG_BAD_CELL = 32        /* a particle cell id out of range          */
};

/* One grid box (Sec. 2 geometries).  faces[d] holds n[d]+1 increasing FP64
 * face coordinates of axis d (HOST memory, copied); theta and phi in
 * radians.  bc: DUST_BC_SHEAR only on axis 0 of a 3-D Cartesian shearing
 * box (both sides), the two sides of an axis must both be periodic or both
 * non-periodic.  shape: DUST_CIC (b_0) or DUST_TSC (b_1) per axis;
 * DUST_VOL, the traditional volume weighting of Eq. CIC_vol (linear in R^2
 * between the two cell centres around the particle), on the radial axis of
 * a cylindrical box only (the comparison scheme of Sec. 3.4). */
typedef struct {
  int32_t geom, ndim;
  int32_t n[3];
  int32_t bc_lo[3], bc_hi[3];
  int32_t shape[3];
  const double *faces[3];
} dust_box_t;

/* External accelerations a_p (Eq. dust_ode).  SHEARBOX: standard
 * shearing box (Eq. standard_SB_p) with Omega, q and, if vertical_gravity,
 * -Omega^2 z.  SHEARBOX_FARGO: the orbital-advection form (Eq. FARGO_SB_p;
 * kick of App. B.1 Eq. FARGO_SB_exp_midpoint): particle momenta and gas
 * velocities are residuals v' = v + q Omega x e_y, y is carried by the mean
 * shear -q Omega x (taken at x^{n+1/2}) in the drifts, and nothing is
 * boosted across the shear-periodic x faces.  POINTMASS: g = -GM x/|x|^3
 * (curvilinear boxes).  CONST: a constant Cartesian g[3].  t: time at the
 * start of the step (shear-periodic offset q Omega L_x t). */
typedef struct {
  int32_t kind, vertical_gravity;
  double Omega, q, GM;
  double g[3];
  double t;
  int32_t integrator;   /* DUST_INTEGRATOR_*: 0 = exponential midpoint */
} dust_forces_t;

/* Particle set, structure of arrays of length n (device memory).
 * drag: tau (DUST_DRAG_TAU; +inf allowed = no drag) or Stokes number
 *   St = tau Omega_K(R) (DUST_DRAG_STOKES); NULL with DUST_DRAG_SPECIES;
 *   with DUST_DRAG_EPSTEIN the constant C = rho_s a / v_t of the Epstein
 *   stopping time tau = C / rho_g (Sec. 2), rho_g the gas density weighted
 *   to the particle (at x^{n+1/2} in the step, at x^n in dust_drag_source;
 *   the unfused step and dust_drag_source only: the fused step, the
 *   autotuner and dust_push_expmid's KICK give DUST_EUNSUPPORTED).
 * mass: per particle, or NULL to take the species table.
 * species: uint8 index into the species table, or NULL (species 0).
 * id: optional int32 label carried along when particles are reordered
 *   (dust_bin with apply_permutation, the fused dust_step), or NULL.
 * In 2-D the third offset and momentum arrays may be NULL.  drag, mass and
 * species are reordered too when they are given. */
typedef struct {
  int32_t *cell;
  void *off[3];
  void *mom[3];
  void *drag;
  void *mass;
  uint8_t *species;
  int32_t *id;
  int64_t n;
} dust_particles_t;

/* Ghosted cell-centred fields (layout above).  vel: gas velocity, physical
 * components (ndim of them in Cartesian, 3 in curvilinear).  dep: drag
 * impulse densities D_c = -(1/dV) sum_p W J_p,c for the ndim (Cartesian) or
 * 3 canonical momentum channels, then the energy density E = -(1/dV)
 * sum_p W e_p (Eq. dust_feedback_final with the energy source of Sec. 2). */
typedef struct {
  void *rho;
  void *vel[3];
  void *dep[4];
} dust_fields_t;

/* FP64 diagnostics accumulated on the device since the last status read. */
typedef struct {
  double p_part[3];      /* sum_p J_p (canonical components)               */
  double p_grid[3];      /* sum_i dV_i D_i over stored cells, before folding */
  double e_part, e_grid; /* the same for the energy channel                */
  double sum_abs_j;      /* sum_p |J_p| (scale of the residual)            */
  double max_cells_per_step; /* max_p,d |v_d^{n+1/2}| dt / dl_d (Eq. particles_dt) */
  int64_t n_removed;     /* particles removed through open faces           */
  int64_t n_fallback;    /* fused path: particles handled outside their tile */
  int32_t flags;         /* sticky DUST_FLAG_* bits                        */
  int32_t steps;         /* steps accumulated                              */
} dust_diag_t;

/* Create a context on `device` for `nbox` boxes.
 * prec: DUST_F32 or DUST_F64 storage of every real array.
 * drag_mode: DUST_DRAG_*; species_tau/species_mass (HOST, nspecies <= 16)
 *   give the species table (tau may be +inf); with DUST_DRAG_SPECIES the
 *   tau table is required; a mass table is required whenever particles are
 *   created without per-particle masses.
 * Allocates the context's device workspace (face tables, diagnostics); the
 * sort and tile workspaces grow on first use.  Synchronous. */
dust_status_t dust_ctx_create(void **ctx, int device, const dust_box_t *boxes, int nbox,
                              int32_t prec, int32_t drag_mode, const double *species_tau,
                              const double *species_mass, int nspecies);

/* Free the context and its workspace (waits for its work to finish). */
dust_status_t dust_ctx_destroy(void *ctx);

/* Per-particle arithmetic of an F32 context in the fused step and in the
 * stage calls (dust_gather, dust_push_expmid, dust_deposit, dust_drag_source,
 * dust_deposit_mass).
 * DUST_ARITH_F32: FP32 registers.  The fused kernel forms the slip p_g - p
 * (Eq. Delta_vp) as a weighted sum of differences, which keeps its relative
 * accuracy where the velocities are much larger than the slip; in
 * cylindrical and spherical boxes the scale factors (R, R sin theta; App. B.2)
 * are FP64 values at the particle carried as two FP32 words, and the
 * azimuthal component's gather sums in FP64 with FP64 radial weights, so
 * that the slip of a particle close to co-rotation keeps its accuracy.
 * DUST_ARITH_F64: FP64 registers, the stored state staying FP32.
 * Defaults: FP32 for the fused step in every geometry; for the stage calls
 * FP32 in Cartesian boxes and FP64 in cylindrical and spherical ones (they
 * form the slip from a gathered velocity passed through memory).  This call
 * sets both.  The unfused chain of dust_step always computes in FP64.
 * Ignored for F64 contexts.  Returns DUST_EINVAL for another value. */
dust_status_t dust_ctx_set_arith(void *ctx, int32_t arith);

/* Deterministic mode (on = 1; 0, the default, turns it off): every result
 * of dust_step, dust_push_expmid, dust_deposit, dust_drag_source and
 * dust_deposit_mass is the same bits on every run with the same inputs.
 * Their deposits (Eq. dust_feedback_final, Sec. 3.1; the predictor's source,
 * Eq. f_D; the dust density) then run without float atomics: a stable sort
 * of the particles by cell, then one thread per stored cell sums, in FP64
 * and in a fixed order, the contributions of the particles of the 3^d cells
 * around it; the kick's diagnostic sums go through per-block partials added
 * in a fixed order.
 * dust_step then runs the unfused chain (DUST_STEP_FUSED and the rebinning
 * interval are ignored), so that the stage calls fill, DRIFT1, gather, KICK,
 * deposit, DRIFT2, fold and feedback give what dust_step gives, bit for bit.
 * Costs a sort per deposit and 3^d weight evaluations per particle; the
 * binned layout of the last fused run is forgotten, and dust_ctx_autotune,
 * which times the fused step, returns DUST_EUNSUPPORTED while the mode is
 * on.  Workspace (sort, partials, per-particle coefficients) grows on first
 * use.
 * Returns DUST_EINVAL for another value of on. */
dust_status_t dust_ctx_set_deterministic(void *ctx, int32_t on);

/* Tile shape of the fused path, in cells per axis (0 keeps the current
 * one).  Compiled shapes (256 cells, one thread per cell): 3-D 8x8x4
 * (default), 16x4x4, 4x16x4, 4x4x16, 8x4x8, 4x8x8; 2-D 16x16 (default), 32x8,
 * 8x32; other shapes give DUST_EUNSUPPORTED.  slack is reserved (0..4). */
dust_status_t dust_ctx_set_tile(void *ctx, int32_t tx, int32_t ty, int32_t tz, int32_t slack);

/* Autotuner of the fused step (batching and tuning row of the hot path):
 * runs `steps` fused steps (after one warm-up step) for every compiled tile
 * shape and rebinning interval 1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48 or 64
 * (timed over whole intervals of at least `steps` steps) on device copies of
 * p and f (the
 * caller's arrays and the context's diagnostics are left unchanged), times
 * them with HIP events on `stream`, and keeps the fastest tile shape and
 * interval in the context (the interval is then used by dust_step when its
 * flags give DUST_STEP_REBIN_EVERY(0)).  flags: any of APPLY_FEEDBACK, DIAG,
 * NO_FILL (else DUST_EINVAL).  result (nullable): tx, ty, tz, interval;
 * ms_per_step (nullable): the best time.  Synchronous; allocates copies of
 * the particles and fields for its duration (DUST_ENOMEM if that fails). */
dust_status_t dust_ctx_autotune(void *ctx, const dust_particles_t *p, const dust_fields_t *f,
                                double dt, const dust_forces_t *frc, int32_t flags, int32_t steps,
                                int32_t *result, float *ms_per_step, void *stream);

/* Kernel timing of the fused path: with max_launches > 0, every dust_step
 * call records a pair of HIP events on its stream around each of its first
 * max_launches fused tile-kernel launches (the tile kernel alone, not the
 * deferred-particle kernel that follows it; also inside a captured graph,
 * as event nodes); dust_ctx_profile then returns, after synchronising, the elapsed
 * milliseconds of the launches of the last dust_step call (count_out of
 * them, at most max_out).  max_launches = 0 turns it off. */
dust_status_t dust_ctx_set_profile(void *ctx, int32_t max_launches);
dust_status_t dust_ctx_profile(void *ctx, float *ms_out, int32_t max_out, int32_t *count_out);

/* Sizes: stored (ghosted) cells over all boxes, active cells over all
 * boxes, and (if box_store_offset != NULL, nbox+1 entries) the first stored
 * cell of every box. */
dust_status_t dust_ctx_grid_size(void *ctx, int64_t *n_stored, int64_t *n_active,
                                 int64_t *box_store_offset);

/* Read and reset the diagnostics.  Synchronises the context's last stream. */
dust_status_t dust_ctx_status(void *ctx, dust_diag_t *diag);

/* Message of the last error of this thread ("" if none). */
const char *dust_last_error(void);

/* Stable counting sort of the particles by key (the replacement of the
 * paper's linked list, Sec. 3).  key_mode DUST_BIN_CELL: key = global cell
 * id; DUST_BIN_TILE: cells renumbered tile by tile with the context's tile
 * shape (tiles and cells in axis-0-fastest order, edge tiles clipped, boxes
 * concatenated).  Removed particles (cell -1) go last; ties keep their
 * input order.  perm_out (n int32, may be NULL): sorted slot -> input index.
 * bin_start_out (nbins+1 int64, may be NULL): first sorted slot of each key,
 * bin_start_out[nbins] = number of particles with a cell.  If
 * apply_permutation, every particle array in `p` is reordered in place. */
dust_status_t dust_bin(void *ctx, dust_particles_t *p, int32_t key_mode, int32_t *perm_out,
                       int64_t *bin_start_out, int apply_permutation, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dust_bin
 * with the same arguments and results (bit for bit), whose sort workspace
 * (keys, values, digit histograms, scan sums, permutation staging) lies in a
 * fixed device array of the library instead of the context's workspace.
 * Calls no hipMalloc, hipFree or other allocating routine.  At most
 * DUST_BIN_NOALLOC_MAX particles (else DUST_ESHAPE, nothing launched).  The
 * array (25 MiB) exists once per GPU until the process ends; its address is
 * taken when the first context on that GPU is created.  All calls on one GPU
 * share it and it keeps the last call's contents: calls that overlap on one
 * GPU (other streams, threads or contexts) race, and the caller must order
 * them. */
#define DUST_BIN_NOALLOC_MAX (1 << 20)
dust_status_t dust_bin_noalloc(void *ctx, dust_particles_t *p, int32_t key_mode, int32_t *perm_out,
                               int64_t *bin_start_out, int apply_permutation, void *stream);

/* Fill the ghosts of periodic and shear-periodic axes of rho and vel at time
 * t (shear offset q Omega L_x t, linear in y between the two nearest cells;
 * v_y of a shear image shifted by -/+ q Omega L_x).  Open-axis ghosts are
 * left as the caller set them. */
dust_status_t dust_fill_ghosts(void *ctx, dust_fields_t *f, const dust_forces_t *frc, double t,
                               void *stream);

/* Field weighting (Eq. Delta_vp): for each particle with a cell, rho_p
 * (n reals, may be NULL) and the gas velocity vg_p[c] (n reals per
 * component) at its current position, component by component in the local
 * basis, with the CIC/TSC weights of Eq. weight (Eq. b0/b1 in Cartesian;
 * Eq. CIC_cylindrical, TSC_cylindrical; Eq. CIC_spherical_r,
 * TSC_spherical_r, CIC_spherical_theta and its TSC analogue) on the 3^ndim
 * stencil of the host cell.  Reads ghosts as stored. */
dust_status_t dust_gather(void *ctx, const dust_particles_t *p, const dust_fields_t *f,
                          void *rho_p, void *vg_p[3], void *stream);

/* Exponential-midpoint push phases (Eq. exp_midpoint; App. B).
 * DRIFT1: half drift to x^{n+1/2}, boundary rules at frc->t + dt/2.
 * KICK: p^{n+1} = e^{-dt/tau} p^n + h1 G, h1 = tau (1 - e^{-dt/tau}) (Eq. h1),
 *   with the gas momentum formed from vg_p (physical, as dust_gather
 *   returns it); writes the drag impulse J = m (p^{n+1} - p^n - dt a^{n+1/2})
 *   (Eq. dust_feedback_final) to impulse[0..nc-1] and the energy
 *   e = m v_bar . (J/m) in physical components to impulse[nc] (entries may
 *   be NULL).  nc = ndim (Cartesian) or 3.
 * DRIFT2: the second half drift, boundary rules at frc->t + dt.
 * Removed particles (cell -1) are skipped. */
dust_status_t dust_push_expmid(void *ctx, dust_particles_t *p, const void *const vg_p[3],
                               double dt, const dust_forces_t *frc, int32_t phases,
                               void *impulse[4], void *stream);

/* Deposit (Eq. deposition, dust_feedback_final): for each particle with a
 * cell, dep[c] -= W J_c / dV (and the energy channel) on the 3^ndim stencil of
 * its current position, with exactly the weights of dust_gather.
 * Accumulates into dep (does not clear it); ghosts receive their share. */
dust_status_t dust_deposit(void *ctx, const dust_particles_t *p, const void *const impulse[4],
                           dust_fields_t *f, void *stream);

/* Drag source of the gas predictor (Sec. 3.1, Eq. Delta_vp and f_D): for
 * each particle with a cell, at its current position x^n, the slip between
 * the gas velocity weighted as in dust_gather and the particle velocity,
 * times m_p / tau'_p with the stiffness limiter tau' = max(tau, dt) of Bai &
 * Stone (2010), is subtracted from the momentum channels with the gather's
 * weights over the cell volume:
 *   dep[c] -= (1/dV) W (m_p / tau'_p) (s_c v_g,c - p_c),
 * c < nc, s_c the canonical factor of the particle (1, R, r, r sin theta),
 * so dep holds force densities in canonical components (torques for the
 * angular channels).  Accumulates (does not clear); the energy channel is
 * neither read nor written, but must be given.  Reads the gas ghosts as
 * stored.  tau = +inf contributes nothing; tau <= dt is limited to dt.
 * The drag mode's arrays (drag, mass or the species tables) are required
 * as for the kick; frc (required) gives GM for Stokes numbers.  dt: finite
 * and > 0, else DUST_EINVAL. */
dust_status_t dust_drag_source(void *ctx, const dust_particles_t *p, dust_fields_t *f, double dt,
                               const dust_forces_t *frc, void *stream);

/* Dust density on the grid (the particle mass spread with the shape
 * function of Sec. 3.4, Eq. weight; compared with eps rho_g in Sec. 4.3.1):
 * for each particle with a cell, rho_d += W m_p / dV on the 3^ndim stencil
 * of its current position, with exactly the weights of dust_gather.
 * rho_d: one ghosted array in the layout of the fields (all boxes, the
 * context's precision); accumulates (does not clear); ghosts receive their
 * share (fold them as a deposit channel with dust_fold_ghosts).  Masses
 * from p->mass or the species mass table (else DUST_EINVAL). */
dust_status_t dust_deposit_mass(void *ctx, const dust_particles_t *p, void *rho_d, void *stream);

/* Fold deposits in periodic / shear-periodic ghosts onto their partners
 * (the transpose of dust_fill_ghosts at time t; the energy channel crossing a
 * shear face gains +/- q Omega L_x D_y) and clear those ghosts. */
dust_status_t dust_fold_ghosts(void *ctx, dust_fields_t *f, const dust_forces_t *frc, double t,
                               void *stream);

/* Feedback on the gas: v_c += D_c / (rho * s_c) on active cells, s_c the
 * canonical-to-physical factor at the cell centre (1, R, r or r sin theta). */
dust_status_t dust_apply_feedback(void *ctx, dust_fields_t *f, void *stream);

/* nsteps full steps at fixed dt from frc->t.  Each step: fill gas ghosts at
 * t + dt/2 (unless DUST_STEP_NO_FILL), clear dep, drift, gather, kick,
 * deposit, drift, (with DUST_STEP_DIAG) FP64 conservation sums, fold,
 * (with DUST_STEP_APPLY_FEEDBACK) feedback.  On return dep holds the last
 * step's deposit.  DUST_STEP_FUSED runs the tiled fused kernel, rebinning
 * the particles every DUST_STEP_REBIN_EVERY(k) steps (k = 0: the context's
 * interval, 1 unless dust_ctx_autotune chose another) by the
 * tile-major key of the cell they reach in the first half drift.  It
 * reorders the particle arrays (give p->id to follow particles): the
 * particles of each group of 64 cells of a tile occupy consecutive slots,
 * level by level (the j-th particle of every cell of the group that has more
 * than j), and particles without a cell come last.  DUST_STEP_GRAPH captures
 * the loop in a hipGraph (replayed while arguments are unchanged). */
dust_status_t dust_step(void *ctx, dust_particles_t *p, dust_fields_t *f, double dt,
                        const dust_forces_t *frc, int32_t nsteps, int32_t flags, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DUST_H */
