// kernels_dispatch.hip -- launch entry points of the stage, initialisation and
// snapshot kernels used by the host runtime (runtime.cpp).  The tile and lane
// kernel instances live in the kernels_tile_*.hip and kernels_lane.hip units.
#include "stage_kernels.h"

namespace heom {

StageKernel tile_kernel_part_small(int N, int KP, bool mixed);
StageKernel tile_kernel_part_7(int N, int KP, bool mixed);
StageKernel tile_kernel_part_8(int N, int KP, bool mixed);
StageKernel tile_kernel_part_9_10(int N, int KP, bool mixed);
StageKernel tile_kernel_part_11(int N, int KP, bool mixed);
StageKernel tile_kernel_part_12(int N, int KP, bool mixed);
StageKernel lane_kernel_ptr(int N, int KP, bool mixed);

namespace {

StageKernel tile_kernel(int N, int KP, bool mixed) {
  StageKernel k = nullptr;
  if (!k) k = tile_kernel_part_small(N, KP, mixed);
  if (!k) k = tile_kernel_part_7(N, KP, mixed);
  if (!k) k = tile_kernel_part_8(N, KP, mixed);
  if (!k) k = tile_kernel_part_9_10(N, KP, mixed);
  if (!k) k = tile_kernel_part_11(N, KP, mixed);
  if (!k) k = tile_kernel_part_12(N, KP, mixed);
  return k;
}

}  // namespace

bool has_fixed_kernel(int N, int KP) { return lane_kernel_ptr(N, KP, false) != nullptr; }

bool has_tile_kernel(int N, int KP) { return tile_kernel(N, KP, false) != nullptr; }

int tile_threads(int N, bool mixed) { return 64 * tile_waves_for(N, !mixed); }

hipError_t launch_stage(KernelKind kind, bool mixed, int N, int KP, const InstDesc *descs,
                        const WorkItem *work, int n_items, int block, int stage, double coef,
                        int hist_slot, hipStream_t stream) {
  StageKernel k = nullptr;
  switch (kind) {
    case KernelKind::kTile:
      k = tile_kernel(N, KP, mixed);
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
