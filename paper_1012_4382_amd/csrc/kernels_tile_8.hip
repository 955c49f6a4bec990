// kernels_tile_8.hip -- instances of the tile stage kernel for
// N=8 K+1=1, N=8 K+1=2
// (FP64 and FP32-mixed storage) in launch shape HEOM_SHAPE: the unit is
// compiled once per shape it provides.
#include "stage_kernels.h"

namespace heom {

StageKernel HEOM_SHAPED(tile_kernel_part_8)(int N, int KP, bool mixed) {
  constexpr int S = HEOM_SHAPE;
  if (N == 8 && KP == 1)
    return mixed ? &stage_tile<8, 1, float, S> : &stage_tile<8, 1, double, S>;
  if (N == 8 && KP == 2)
    return mixed ? &stage_tile<8, 2, float, S> : &stage_tile<8, 2, double, S>;
  return nullptr;
}

}  // namespace heom
