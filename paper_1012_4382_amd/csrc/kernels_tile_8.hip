// kernels_tile_8.hip -- instances of the tile stage kernel for
// N=8 K+1=1, N=8 K+1=2 (FP64 and FP32-mixed storage).
#include "stage_kernels.h"

namespace heom {

StageKernel tile_kernel_part_8(int N, int KP, bool mixed) {
  if (N == 8 && KP == 1)
    return mixed ? &stage_tile<8, 1, float> : &stage_tile<8, 1, double>;
  if (N == 8 && KP == 2)
    return mixed ? &stage_tile<8, 2, float> : &stage_tile<8, 2, double>;
  return nullptr;
}

}  // namespace heom
