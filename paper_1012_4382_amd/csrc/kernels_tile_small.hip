// kernels_tile_small.hip -- instances of the tile stage kernel for
// N=1 K+1=1, N=2 K+1=1, N=3 K+1=1, N=4 K+1=1, N=5 K+1=1, N=6 K+1=1, N=1 K+1=2, N=2 K+1=2, N=3 K+1=2, N=4 K+1=2, N=5 K+1=2, N=6 K+1=2
// in launch shape HEOM_SHAPE and storage precision HEOM_TILE_F64 (FP64, with
// plain and streaming stores, or FP32-mixed): the unit is compiled once per
// shape it provides and per precision.
#include "stage_kernels.h"

namespace heom {

StageKernel HEOM_SHAPED(tile_kernel_part_small)(int N, int KP, bool mixed, bool streaming,
                                                bool scaled) {
  constexpr int S = HEOM_SHAPE;
  if (N == 1 && KP == 1)
    return tile_instance<1, 1, S>(mixed, streaming, scaled);
  if (N == 2 && KP == 1)
    return tile_instance<2, 1, S>(mixed, streaming, scaled);
  if (N == 3 && KP == 1)
    return tile_instance<3, 1, S>(mixed, streaming, scaled);
  if (N == 4 && KP == 1)
    return tile_instance<4, 1, S>(mixed, streaming, scaled);
  if (N == 5 && KP == 1)
    return tile_instance<5, 1, S>(mixed, streaming, scaled);
  if (N == 6 && KP == 1)
    return tile_instance<6, 1, S>(mixed, streaming, scaled);
  if (N == 1 && KP == 2)
    return tile_instance<1, 2, S>(mixed, streaming, scaled);
  if (N == 2 && KP == 2)
    return tile_instance<2, 2, S>(mixed, streaming, scaled);
  if (N == 3 && KP == 2)
    return tile_instance<3, 2, S>(mixed, streaming, scaled);
  if (N == 4 && KP == 2)
    return tile_instance<4, 2, S>(mixed, streaming, scaled);
  if (N == 5 && KP == 2)
    return tile_instance<5, 2, S>(mixed, streaming, scaled);
  if (N == 6 && KP == 2)
    return tile_instance<6, 2, S>(mixed, streaming, scaled);
  return nullptr;
}

}  // namespace heom
