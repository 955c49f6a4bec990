// kernels_tile_11.hip -- instances of the tile stage kernel for
// N=11 K+1=1 (FP64 and FP32-mixed storage).
#include "stage_kernels.h"

namespace heom {

StageKernel tile_kernel_part_11(int N, int KP, bool mixed) {
  if (N == 11 && KP == 1)
    return mixed ? &stage_tile<11, 1, float> : &stage_tile<11, 1, double>;
  return nullptr;
}

}  // namespace heom
