// kernels_tile_small.hip -- instances of the tile stage kernel for
// N=1 K+1=1, N=2 K+1=1, N=3 K+1=1, N=4 K+1=1, N=5 K+1=1, N=6 K+1=1, N=1 K+1=2, N=2 K+1=2, N=3 K+1=2, N=4 K+1=2, N=5 K+1=2, N=6 K+1=2
// (FP64 and FP32-mixed storage) in launch shape HEOM_SHAPE: the unit is
// compiled once per shape it provides.
#include "stage_kernels.h"

namespace heom {

StageKernel HEOM_SHAPED(tile_kernel_part_small)(int N, int KP, bool mixed) {
  constexpr int S = HEOM_SHAPE;
  if (N == 1 && KP == 1)
    return mixed ? &stage_tile<1, 1, float, S> : &stage_tile<1, 1, double, S>;
  if (N == 2 && KP == 1)
    return mixed ? &stage_tile<2, 1, float, S> : &stage_tile<2, 1, double, S>;
  if (N == 3 && KP == 1)
    return mixed ? &stage_tile<3, 1, float, S> : &stage_tile<3, 1, double, S>;
  if (N == 4 && KP == 1)
    return mixed ? &stage_tile<4, 1, float, S> : &stage_tile<4, 1, double, S>;
  if (N == 5 && KP == 1)
    return mixed ? &stage_tile<5, 1, float, S> : &stage_tile<5, 1, double, S>;
  if (N == 6 && KP == 1)
    return mixed ? &stage_tile<6, 1, float, S> : &stage_tile<6, 1, double, S>;
  if (N == 1 && KP == 2)
    return mixed ? &stage_tile<1, 2, float, S> : &stage_tile<1, 2, double, S>;
  if (N == 2 && KP == 2)
    return mixed ? &stage_tile<2, 2, float, S> : &stage_tile<2, 2, double, S>;
  if (N == 3 && KP == 2)
    return mixed ? &stage_tile<3, 2, float, S> : &stage_tile<3, 2, double, S>;
  if (N == 4 && KP == 2)
    return mixed ? &stage_tile<4, 2, float, S> : &stage_tile<4, 2, double, S>;
  if (N == 5 && KP == 2)
    return mixed ? &stage_tile<5, 2, float, S> : &stage_tile<5, 2, double, S>;
  if (N == 6 && KP == 2)
    return mixed ? &stage_tile<6, 2, float, S> : &stage_tile<6, 2, double, S>;
  return nullptr;
}

}  // namespace heom
