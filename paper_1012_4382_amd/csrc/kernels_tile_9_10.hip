// kernels_tile_9_10.hip -- instances of the tile stage kernel for
// N=9 K+1=1, N=10 K+1=1
// (FP64 and FP32-mixed storage) in launch shape HEOM_SHAPE: the unit is
// compiled once per shape it provides.
#include "stage_kernels.h"

namespace heom {

StageKernel HEOM_SHAPED(tile_kernel_part_9_10)(int N, int KP, bool mixed) {
  constexpr int S = HEOM_SHAPE;
  if (N == 9 && KP == 1)
    return mixed ? &stage_tile<9, 1, float, S> : &stage_tile<9, 1, double, S>;
  if (N == 10 && KP == 1)
    return mixed ? &stage_tile<10, 1, float, S> : &stage_tile<10, 1, double, S>;
  return nullptr;
}

}  // namespace heom
