// kernels_dispatch.hip -- launch entry points of the stage, initialisation and
// snapshot kernels used by the host runtime (runtime.cpp).  The tile and lane
// kernel instances live in the kernels_tile_*.hip and kernels_lane.hip units.
#include "stage_kernels.h"

namespace heom {

typedef StageKernel (*TilePart)(int N, int KP, bool mixed);
// Tile instances by shape: N <= 8 in every shape, N = 9..12 in shape 0 only.
StageKernel tile_kernel_part_small_s0(int, int, bool);
StageKernel tile_kernel_part_small_s1(int, int, bool);
StageKernel tile_kernel_part_small_s2(int, int, bool);
StageKernel tile_kernel_part_7_s0(int, int, bool);
StageKernel tile_kernel_part_7_s1(int, int, bool);
StageKernel tile_kernel_part_7_s2(int, int, bool);
StageKernel tile_kernel_part_8_s0(int, int, bool);
StageKernel tile_kernel_part_8_s1(int, int, bool);
StageKernel tile_kernel_part_8_s2(int, int, bool);
StageKernel tile_kernel_part_small_s3(int, int, bool);
StageKernel tile_kernel_part_7_s3(int, int, bool);
StageKernel tile_kernel_part_8_s3(int, int, bool);
StageKernel tile_kernel_part_small_s4(int, int, bool);
StageKernel tile_kernel_part_7_s4(int, int, bool);
StageKernel tile_kernel_part_8_s4(int, int, bool);
StageKernel tile_kernel_part_9_10_s0(int, int, bool);
StageKernel tile_kernel_part_11_s0(int, int, bool);
StageKernel tile_kernel_part_12_s0(int, int, bool);
StageKernel lane_kernel_ptr(int N, int KP, bool mixed);

namespace {

static_assert(kTileShapes == 5, "one row of tile parts per shape");
constexpr TilePart kTileParts[kTileShapes][6] = {
    {&tile_kernel_part_small_s0, &tile_kernel_part_7_s0, &tile_kernel_part_8_s0,
     &tile_kernel_part_9_10_s0, &tile_kernel_part_11_s0, &tile_kernel_part_12_s0},
    {&tile_kernel_part_small_s1, &tile_kernel_part_7_s1, &tile_kernel_part_8_s1, nullptr, nullptr,
     nullptr},
    {&tile_kernel_part_small_s2, &tile_kernel_part_7_s2, &tile_kernel_part_8_s2, nullptr, nullptr,
     nullptr},
    {&tile_kernel_part_small_s3, &tile_kernel_part_7_s3, &tile_kernel_part_8_s3, nullptr, nullptr,
     nullptr},
    {&tile_kernel_part_small_s4, &tile_kernel_part_7_s4, &tile_kernel_part_8_s4, nullptr, nullptr,
     nullptr},
};

StageKernel tile_kernel(int N, int KP, bool mixed, int shape) {
  if (shape < 0 || shape >= kTileShapes) return nullptr;
  for (TilePart part : kTileParts[shape]) {
    StageKernel k = part ? part(N, KP, mixed) : nullptr;
    if (k) return k;
  }
  return nullptr;
}

}  // namespace

bool has_fixed_kernel(int N, int KP) { return lane_kernel_ptr(N, KP, false) != nullptr; }

bool has_tile_kernel(int N, int KP) { return tile_kernel(N, KP, false, 0) != nullptr; }

bool tile_shape_info(int N, int KP, bool mixed, int shape, int *threads, int *elems_per_wave,
                     int *chunk, int *min_waves) {
  if (!tile_kernel(N, KP, mixed, shape)) return false;
  const TileShape sh = tile_shape(!mixed, shape);
  if (threads) *threads = 64 * tile_waves(N, !mixed, shape);
  if (elems_per_wave) *elems_per_wave = sh.elems_per_wave;
  if (chunk) *chunk = sh.chunk;
  if (min_waves) *min_waves = sh.min_waves;
  return true;
}

hipError_t launch_stage(KernelKind kind, bool mixed, int N, int KP, int shape,
                        const InstDesc *descs, const WorkItem *work, int n_items, int block,
                        int stage, double coef, int hist_slot, hipStream_t stream) {
  StageKernel k = nullptr;
  switch (kind) {
    case KernelKind::kTile:
      k = tile_kernel(N, KP, mixed, shape);
      break;
    case KernelKind::kLane:
      k = lane_kernel_ptr(N, KP, mixed);
      break;
    case KernelKind::kGeneric:
      k = mixed ? &stage_generic<float> : &stage_generic<double>;
      break;
  }
  if (!k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3(n_items), dim3(block), 0, stream, descs, work, stage, coef, hist_slot);
  return hipGetLastError();
}

hipError_t launch_init(bool mixed, const InstDesc *descs, const WorkItem *work, int n_items,
                       int block, hipStream_t stream) {
  if (mixed)
    hipLaunchKernelGGL(init_state<float>, dim3(n_items), dim3(block), 0, stream, descs, work);
  else
    hipLaunchKernelGGL(init_state<double>, dim3(n_items), dim3(block), 0, stream, descs, work);
  return hipGetLastError();
}

hipError_t launch_snapshot(bool mixed, const InstDesc *descs, int n_inst, int slot,
                           hipStream_t stream) {
  if (mixed)
    hipLaunchKernelGGL(snapshot<float>, dim3(n_inst), dim3(64), 0, stream, descs, n_inst, slot);
  else
    hipLaunchKernelGGL(snapshot<double>, dim3(n_inst), dim3(64), 0, stream, descs, n_inst, slot);
  return hipGetLastError();
}

}  // namespace heom
