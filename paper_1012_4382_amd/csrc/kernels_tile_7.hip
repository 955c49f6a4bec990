// kernels_tile_7.hip -- instances of the tile stage kernel for
// N=7 K+1=1, N=7 K+1=2 (FP64 and FP32-mixed storage).
#include "stage_kernels.h"

namespace heom {

StageKernel tile_kernel_part_7(int N, int KP, bool mixed) {
  if (N == 7 && KP == 1)
    return mixed ? &stage_tile<7, 1, float> : &stage_tile<7, 1, double>;
  if (N == 7 && KP == 2)
    return mixed ? &stage_tile<7, 2, float> : &stage_tile<7, 2, double>;
  return nullptr;
}

}  // namespace heom
