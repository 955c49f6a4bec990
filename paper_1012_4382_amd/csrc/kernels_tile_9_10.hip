// kernels_tile_9_10.hip -- instances of the tile stage kernel for
// N=9 K+1=1, N=10 K+1=1 (FP64 and FP32-mixed storage).
#include "stage_kernels.h"

namespace heom {

StageKernel tile_kernel_part_9_10(int N, int KP, bool mixed) {
  if (N == 9 && KP == 1)
    return mixed ? &stage_tile<9, 1, float> : &stage_tile<9, 1, double>;
  if (N == 10 && KP == 1)
    return mixed ? &stage_tile<10, 1, float> : &stage_tile<10, 1, double>;
  return nullptr;
}

}  // namespace heom
