// kernels_tile_12.hip -- instances of the tile stage kernel for
// N=12 K+1=1
// (FP64 and FP32-mixed storage) in launch shape HEOM_SHAPE: the unit is
// compiled once per shape it provides.
#include "stage_kernels.h"

namespace heom {

StageKernel HEOM_SHAPED(tile_kernel_part_12)(int N, int KP, bool mixed) {
  constexpr int S = HEOM_SHAPE;
  if (N == 12 && KP == 1)
    return mixed ? &stage_tile<12, 1, float, S> : &stage_tile<12, 1, double, S>;
  return nullptr;
}

}  // namespace heom
