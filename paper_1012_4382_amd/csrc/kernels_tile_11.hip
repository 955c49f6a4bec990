// kernels_tile_11.hip -- instances of the tile stage kernel for
// N=11 K+1=1
// (FP64 and FP32-mixed storage) in launch shape HEOM_SHAPE: the unit is
// compiled once per shape it provides.
#include "stage_kernels.h"

namespace heom {

StageKernel HEOM_SHAPED(tile_kernel_part_11)(int N, int KP, bool mixed) {
  constexpr int S = HEOM_SHAPE;
  if (N == 11 && KP == 1)
    return mixed ? &stage_tile<11, 1, float, S> : &stage_tile<11, 1, double, S>;
  return nullptr;
}

}  // namespace heom
