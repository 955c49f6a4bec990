// kernels_tile_8.hip -- instances of the tile stage kernel for
// N=8 K+1=1, N=8 K+1=2
// in launch shape HEOM_SHAPE and storage precision HEOM_TILE_F64 (FP64, with
// plain and streaming stores, or FP32-mixed): the unit is compiled once per
// shape it provides and per precision.
#include "stage_kernels.h"

namespace heom {

StageKernel HEOM_SHAPED(tile_kernel_part_8)(int N, int KP, bool mixed, bool streaming,
                                            bool scaled) {
  constexpr int S = HEOM_SHAPE;
  if (N == 8 && KP == 1)
    return tile_instance<8, 1, S>(mixed, streaming, scaled);
  if (N == 8 && KP == 2)
    return tile_instance<8, 2, S>(mixed, streaming, scaled);
  return nullptr;
}

}  // namespace heom
