// Internal launcher declarations of the dust library (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dust_types.h"

namespace dust {

template <typename TS> struct PView {
  int32_t *cell;
  TS *off[3];
  TS *mom[3];
  TS *drag;
  TS *mass;
  uint8_t *species;
  int32_t *id;
  int64_t n;
};

template <typename TS> struct FView {
  TS *rho;
  TS *vel[3];
  TS *dep[4];
};

template <typename TS, typename A>
void launch_drift(const PView<TS>& p, const Box* boxes, int nbox, int geom, int ndim, int unif,
                  const Forces& f, double h, const double* tdev, double toff, int first,
                  DiagDev* dg, hipStream_t st);
// TW: type of the per-particle gas-velocity / impulse arrays (the caller's
// precision for the stage calls, the arithmetic precision inside dust_step).
template <typename TS, typename A, typename TW>
// xg: the context's FP64 x-ghost gas layers, or null (ghosts from fl).
void launch_gather(const PView<TS>& p, const Box* boxes, int nbox, int geom, int ndim, int unif,
                   const FView<TS>& fl, const double* xg, TW* rho_p, TW* const vg[3], DiagDev* dg,
                   hipStream_t st);
template <typename TS, typename A, typename TW>
// rho_p: the gathered gas density (Epstein drag; else unused, may be null).
// part: null (diagnostic sums by atomics), or kick_partial_words(n) doubles
// of scratch for per-block partials added up in a fixed order
// (deterministic sums).
void launch_kick(const PView<TS>& p, const Box* boxes, int nbox, int geom, int ndim, int unif,
                 const Forces& f, const Species* sp, int drag_mode, double dt, const TW* rho_p,
                 const TW* const vg[3], TW* const imp[4], DiagDev* dg, double* part, hipStream_t st);
int64_t kick_partial_words(int64_t n);
template <typename TS, typename A, typename TW>
void launch_deposit(const PView<TS>& p, const Box* boxes, int nbox, int geom, int ndim, int unif,
                    const FView<TS>& fl, const TW* const imp[4], DiagDev* dg, hipStream_t st);
// A deposit into one box without float atomics (same bits on every run):
// fl.dep[m] += sgn * sum W imp[m] / dV for m < nch; perm and bin_start from
// a stable sort of the particles by global cell id (launch_bin,
// DUST_BIN_CELL).  B: the host copy of the box.
template <typename TS, typename A, typename TW>
void launch_deposit_pull(const PView<TS>& p, const Box& B, int geom, int ndim, int unif, const FView<TS>& fl,
                         int nch, double sgn, const TW* const imp[4], const uint32_t* perm,
                         const int64_t* bin_start, hipStream_t st);
// Per-particle drag source coefficients (Eq. f_D with tau <- max(tau, dt);
// channels of the momentum) or masses (mass) into q[0..2], for
// launch_deposit_pull.
template <typename TS, typename A>
void launch_source_coeffs(const PView<TS>& p, const Box* boxes, int nbox, int geom, int ndim, int unif,
                          const FView<TS>& fl, const Forces& f, const Species* sp, int drag_mode, double dt,
                          bool mass, A* const q[3], DiagDev* dg, hipStream_t st);

// Drag source of the gas predictor (Eq. f_D, tau <- max(tau, dt)) at the
// particles' current positions, accumulated into the momentum channels of fl.
template <typename TS, typename A>
void launch_drag_source(const PView<TS>& p, const Box* boxes, int nbox, int geom, int ndim, int unif,
                        const FView<TS>& fl, const Forces& f, const Species* sp, int drag_mode,
                        double dt, DiagDev* dg, hipStream_t st);

// Dust density rho_d += m W / dV at the particles' current positions.
template <typename TS, typename A>
void launch_mass_density(const PView<TS>& p, const Box* boxes, int nbox, int geom, int ndim, int unif,
                         TS* rho_d, const Species* sp, DiagDev* dg, hipStream_t st);

// The per-box grid operations below take the host copies of the boxes (hb,
// nbox; geometry and ndim shared) and their device table, and launch each
// kernel once for up to 16 boxes.
// Ghost fill of the gas at *tdev + toff; with xg (the context's FP64 x-ghost
// buffer), also the FP64 x-ghost layers of shear-periodic boxes.
template <typename TS>
void launch_fill(const Box* hb, int nbox, const Box* boxes_d, const Forces& f, const double* tdev, double toff,
                 const FView<TS>& fl, double* xg, hipStream_t st);
template <typename TS>
void launch_fold(const Box* hb, int nbox, const Box* boxes_d, const Forces& f, const double* tdev, double toff,
                 const FView<TS>& fl, hipStream_t st);
void launch_set_time(double* tdev, double v, hipStream_t st);
// advance the step time by dt; count: the diagnostics whose step count goes up (or null)
void launch_advance_time(double* tdev, double dt, DiagDev* count, hipStream_t st);
template <typename TS>
void launch_feedback(const Box* hb, int nbox, const Box* boxes_d, const FView<TS>& fl, hipStream_t st);
// FP64 grid sums of the boxes, added to dg; part: GRID_SUM_PARTS * 4
// doubles of scratch.
static constexpr int GRID_SUM_BLOCKS = 2048;
static constexpr int GRID_SUM_PARTS = GRID_SUM_BLOCKS + 16;
template <typename TS>
void launch_grid_sums(const Box* hb, int nbox, const Box* boxes_d, const FView<TS>& fl, DiagDev* dg, double* part,
                      hipStream_t st);
template <typename TS> void launch_fill_value(TS* a, int64_t n, TS v, hipStream_t st);
// Zero the first nch deposit channels over n stored cells (one launch).
template <typename TS> void launch_clear_deposits(const FView<TS>& fl, int nch, int64_t n, hipStream_t st);

// Binning (dust_bin.hip).  Workspace sizes in bytes for n particles.
struct BinWork {
  uint32_t *key[2];
  uint32_t *val[2];
  uint32_t *hist;       // 256 * nblocks, scanned in place
  uint32_t *scan_tmp;   // block sums of the scans
  void *gather_tmp;     // 8 bytes per particle (permutation application)
  size_t cap_n;
};
size_t bin_scan_tmp_words(int64_t n);
int64_t bin_blocks(int64_t n);   // radix-pass blocks for n keys (digit histogram columns)
struct TileShape { int32_t t[3]; };
// Stable sort of particles by key; writes perm (sorted slot -> input index)
// and bin_start (nbins+1) if given.  key_mode: DUST_BIN_CELL or DUST_BIN_TILE;
// keys_ready: w.key[0] already holds the keys (values are the indices).
// Returns the buffer index c with the sorted keys in w.key[c] and the
// permutation in w.val[c].
int launch_bin(const int32_t* cell, int64_t n, const Box* boxes_dev, int nbox, int64_t nbins,
               int key_mode, TileShape tile, BinWork& w, int32_t* perm_out,
               int64_t* bin_start_out, bool keys_ready, hipStream_t st);
// out[i] = in[perm[i]] for an array of `bytes`-sized elements.
void launch_permute(const void* in, void* out, const uint32_t* perm, int64_t n, int bytes,
                    hipStream_t st);

}  // namespace dust
