// kernels_lane.hip -- instances of the one-lane-per-ADO stage kernel (N <= 8,
// K+1 <= 2; FP64 and FP32-mixed storage).
#include "stage_kernels.h"

namespace heom {

StageKernel lane_kernel_ptr(int N, int KP, bool mixed) {
  if (N == 1 && KP == 1)
    return mixed ? &stage_fixed<1, 1, float> : &stage_fixed<1, 1, double>;
  if (N == 2 && KP == 1)
    return mixed ? &stage_fixed<2, 1, float> : &stage_fixed<2, 1, double>;
  if (N == 3 && KP == 1)
    return mixed ? &stage_fixed<3, 1, float> : &stage_fixed<3, 1, double>;
  if (N == 4 && KP == 1)
    return mixed ? &stage_fixed<4, 1, float> : &stage_fixed<4, 1, double>;
  if (N == 5 && KP == 1)
    return mixed ? &stage_fixed<5, 1, float> : &stage_fixed<5, 1, double>;
  if (N == 6 && KP == 1)
    return mixed ? &stage_fixed<6, 1, float> : &stage_fixed<6, 1, double>;
  if (N == 7 && KP == 1)
    return mixed ? &stage_fixed<7, 1, float> : &stage_fixed<7, 1, double>;
  if (N == 8 && KP == 1)
    return mixed ? &stage_fixed<8, 1, float> : &stage_fixed<8, 1, double>;
  if (N == 1 && KP == 2)
    return mixed ? &stage_fixed<1, 2, float> : &stage_fixed<1, 2, double>;
  if (N == 2 && KP == 2)
    return mixed ? &stage_fixed<2, 2, float> : &stage_fixed<2, 2, double>;
  if (N == 3 && KP == 2)
    return mixed ? &stage_fixed<3, 2, float> : &stage_fixed<3, 2, double>;
  if (N == 4 && KP == 2)
    return mixed ? &stage_fixed<4, 2, float> : &stage_fixed<4, 2, double>;
  if (N == 5 && KP == 2)
    return mixed ? &stage_fixed<5, 2, float> : &stage_fixed<5, 2, double>;
  if (N == 6 && KP == 2)
    return mixed ? &stage_fixed<6, 2, float> : &stage_fixed<6, 2, double>;
  if (N == 7 && KP == 2)
    return mixed ? &stage_fixed<7, 2, float> : &stage_fixed<7, 2, double>;
  if (N == 8 && KP == 2)
    return mixed ? &stage_fixed<8, 2, float> : &stage_fixed<8, 2, double>;
  return nullptr;
}

}  // namespace heom
