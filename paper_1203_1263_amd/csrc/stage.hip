// Stage-kernel dispatch by grid dimension and the list of compiled tile
// shapes (see stage1d.hip, stage2d.hip, stage3d.hip for the kernels).
#include "nlse_internal.h"

hipError_t nlse_launch_stage_1d(const nlse::StageLaunch& L, hipStream_t st);
hipError_t nlse_launch_stage_2d(const nlse::StageLaunch& L, hipStream_t st);
hipError_t nlse_launch_stage_3d(const nlse::StageLaunch& L, hipStream_t st);

hipError_t nlse_launch_stage(const nlse::StageLaunch& L, hipStream_t st) {
  if (L.stage < 1 || L.stage > 4) return hipErrorInvalidValue;
  switch (L.ndim) {
    case 1: return nlse_launch_stage_1d(L, st);
    case 2: return nlse_launch_stage_2d(L, st);
    case 3: return nlse_launch_stage_3d(L, st);
    default: return hipErrorInvalidValue;
  }
}

// Tile shapes compiled into the stage kernels: (x-width, y-height, z-chunk).
extern "C" int nlse_internal_tile_supported(int ndim, int dtype, const int tile[3]) {
  (void)dtype;
  const int tx = tile[0], ty = tile[1], cz = tile[2];
  // 1D: 256 = per-stage kernels, 1024 = whole-grid kernel (small grids)
  if (ndim == 1) return (tx == 256 || tx == 1024) && ty == 1 && cz == 1;
  const bool xy = (tx == 32 && ty == 8) || (tx == 64 && ty == 4) || (tx == 64 && ty == 8);
  // 2D also: 128x4, 64x16, 32x16 and 32x32 (the batched integrator's other tiles)
  if (ndim == 2)
    return (xy || (tx == 128 && ty == 4) || (tx == 64 && ty == 16) || (tx == 32 && ty == 16) ||
            (tx == 32 && ty == 32)) &&
           cz == 1;
  return xy && cz >= 1 && cz <= 4096;
}
