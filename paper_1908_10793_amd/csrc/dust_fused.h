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
  int halo = 2;           // LDS window beyond the tile: stencil + half drift
  int ntiles = 0;
  int rmax[3] = {0, 0, 0};  // largest region extents
  size_t lds_cells = 0;
  TileDesc* tiles_d = nullptr;
};

dust_status_t fused_plan_init(FusedPlan& plan, const Box* boxes, int nbox, TileShape tile, int slack);
void fused_plan_free(FusedPlan& plan);
size_t fused_lds_bytes(const FusedPlan& plan, int nc);

template <typename TS, typename A>
void launch_fused(const FusedPlan& plan, const PView<TS>& p, const Box* boxes_d, int nbox, int geom,
                  int ndim, int unif, const FView<TS>& fl, const Forces& f, const Species* sp, int drag_mode,
                  double dt, const double* tdev, const int64_t* bin_start, DiagDev* dg, bool sums,
                  hipStream_t st);

void launch_count_step(DiagDev* dg, hipStream_t st);

}  // namespace dust
