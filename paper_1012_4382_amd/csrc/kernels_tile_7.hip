// kernels_tile_7.hip -- instances of the tile stage kernel for
// N=7 K+1=1, N=7 K+1=2
// (FP64 and FP32-mixed storage) in launch shape HEOM_SHAPE: the unit is
// compiled once per shape it provides.
#include "stage_kernels.h"

namespace heom {

StageKernel HEOM_SHAPED(tile_kernel_part_7)(int N, int KP, bool mixed) {
  constexpr int S = HEOM_SHAPE;
  if (N == 7 && KP == 1)
    return mixed ? &stage_tile<7, 1, float, S> : &stage_tile<7, 1, double, S>;
  if (N == 7 && KP == 2)
    return mixed ? &stage_tile<7, 2, float, S> : &stage_tile<7, 2, double, S>;
  return nullptr;
}

}  // namespace heom
