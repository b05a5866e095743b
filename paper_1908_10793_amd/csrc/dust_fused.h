// Fused tile kernel of the dust hot path: plan (tile table) and launcher.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dust_launch.h"
#include "dust_types.h"

namespace dust {

struct TileDesc {
  int32_t box;
  int32_t i0, j0, k0;    // first active cell of the tile
  int32_t ex, ey, ez;    // tile extents (clipped at the box edge)
  int32_t pad;
  int64_t key0;          // first tile-major key of the tile
};

struct FusedPlan {
  bool ok = false;
  TileShape tile{{8, 8, 4}};
  int shape = 0;          // index of the compiled tile shape
  bool small = false;     // every box has fewer than 2^24 cells
  int halo = 2;           // LDS window beyond the tile: stencil + half drift
  int ntiles = 0;
  int rmax[3] = {0, 0, 0};  // largest region extents
  size_t lds_cells = 0;
  TileDesc* tiles_d = nullptr;
  double* part_d = nullptr;   // per-tile diagnostic partials (+ the deferred kernel's)
  uint32_t* defer_count = nullptr;   // deferred particles of the current launch
  uint32_t* defer_list = nullptr;    // their (slot, source) pairs (capacity defer_cap pairs)
  size_t defer_cap = 0;
  uint8_t* tile_map = nullptr;       // per tile, 256 tile-local cells in thread order (FP32
                                     // Cartesian path: ranked by particle count at each rebinning)
};

// Capacity of the deferred-particle list for n particles.
dust_status_t fused_plan_reserve(FusedPlan& plan, int64_t n);

dust_status_t fused_plan_init(FusedPlan& plan, const Box* boxes, int nbox, TileShape tile, int slack);
void fused_plan_free(FusedPlan& plan);
// LDS of one fused workgroup: the dynamic part (windows), and the static
// part (per-thread diagnostic sums, species tables) as an upper bound.
size_t fused_lds_bytes(const FusedPlan& plan, int nc, int ts_bytes);
static constexpr size_t FUSED_STATIC_LDS = 5 * 256 * sizeof(double) + 3 * DUST_MAX_SPECIES * sizeof(double) + 256;

// One fused step over every tile (binned by tile-major key, bin_start):
// slot s of q receives the update of particle src_index[s] of p, or of
// particle s when src_index is null (then q may be p: in place); copy_attrs
// copies drag / mass / species / id along.  xg: the context's FP64 x-ghost
// gas layers (filled this step), or null.  ev0 / ev1 (nullable) are recorded
// around the tile kernel alone (not the deferred-particle kernel).
template <typename TS, typename A>
void launch_fused(const FusedPlan& plan, const PView<TS>& p, const PView<TS>& q, bool copy_attrs,
                  const Box* boxes_d, int nbox, int geom, int ndim, int unif, const FView<TS>& fl,
                  const Forces& f, const Species* sp, int drag_mode, double dt, const double* tdev,
                  const int64_t* bin_start, const double* xg, DiagDev* dg, bool sums,
                  const uint32_t* src_index, hipEvent_t ev0, hipEvent_t ev1, hipStream_t st);

// Keys (tile-major) of the cells the particles reach in the first half drift
// of a step of length dt starting at *tdev.
template <typename TS, typename A>
void launch_halfstep_keys(const PView<TS>& p, const Box* boxes_d, int nbox, int geom, int ndim,
                          int unif, const Forces& f, double dt, const double* tdev, int64_t nbins,
                          TileShape ts, uint32_t* key, hipStream_t st);

// After a sort of src (perm, bin_start): lm = the source index of every
// binned slot in the fused kernel's level-major layout within each wave's
// range of slots; the particles without a cell (sorted slots from
// bin_start[nbins] on, which no tile visits) are copied to the same slots of
// dst (distinct from src).
template <typename TS>
void launch_level_perm(const FusedPlan& plan, const PView<TS>& src, const PView<TS>& dst,
                       const uint32_t* perm, const int64_t* bin_start, int64_t nbins, uint32_t* lm,
                       hipStream_t st);

// The particles without a cell (slots from bin_start[nbins] on): dst[s] =
// src[perm[s]], or src[s] when perm is null (distinct arrays).
template <typename TS>
void launch_copy_tail(const PView<TS>& src, const PView<TS>& dst, const int64_t* bin_start, int64_t nbins,
                      hipStream_t st, const uint32_t* perm = nullptr);

// Adds the per-workgroup diagnostic partials of the last fused launch (tile
// kernel and deferred kernel) to the diagnostics block, and resets the
// deferred-particle count.
void launch_reduce_fused(const FusedPlan& plan, DiagDev* dg, bool sums, hipStream_t st);

// The fused step of uniform 3-D Cartesian boxes in FP32 storage and
// arithmetic (dust_cart3.hip), with forces none, constant or standard
// shearing box: the tile kernel (ev0 / ev1 around it), the deferred-particle
// kernel and the reduction of their diagnostic partials.
void launch_c3(const FusedPlan& plan, const PView<float>& p, const PView<float>& q, bool copy_attrs,
               const Box* boxes_d, int nbox, const FView<float>& fl, const Forces& f, const Species* sp,
               int drag_mode, double dt, const double* tdev, const int64_t* bin_start, const double* xg,
               DiagDev* dg, bool sums, const uint32_t* src_index, hipEvent_t ev0, hipEvent_t ev1,
               hipStream_t st);
// Its rebinning: half-step tile keys with its own drift, and after the sort
// the per-tile ranking of cells by count (plan.tile_map) with the source
// index of every slot (lm).
void launch_c3_keys(const PView<float>& p, const Box* boxes_d, int nbox, double dt, int64_t nbins,
                    TileShape ts, uint32_t* key, hipStream_t st);
void launch_c3_level_perm(const FusedPlan& plan, const uint32_t* perm, const int64_t* bin_start, uint32_t* lm,
                          hipStream_t st);
// Predictor drag source (mass: dust density) on the binned layout of the
// last fused step (see k_c3_aux): out[0..2] the momentum deposit channels
// (mass: out[0] the density array).
void launch_c3_aux(const FusedPlan& plan, const PView<float>& p, const Box* boxes_d, int nbox,
                   const FView<float>& fl, float* const out[3], bool mass, const Forces& f, const Species* sp,
                   double dt, const int64_t* bin_start, int64_t nbins, DiagDev* dg, hipStream_t st);
size_t c3_lds_bytes(const FusedPlan& plan);

// dst = src, every particle array.
template <typename TS>
void launch_copy_particles(const PView<TS>& src, const PView<TS>& dst, hipStream_t st);


}  // namespace dust
