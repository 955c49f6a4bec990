// kernels_tile_12.hip -- instances of the tile stage kernel for
// N=12 K+1=1 (FP64 and FP32-mixed storage).
#include "stage_kernels.h"

namespace heom {

StageKernel tile_kernel_part_12(int N, int KP, bool mixed) {
  if (N == 12 && KP == 1)
    return mixed ? &stage_tile<12, 1, float> : &stage_tile<12, 1, double>;
  return nullptr;
}

}  // namespace heom
