// kernels_dispatch.hip -- launch entry points of the stage, initialisation and
// snapshot kernels used by the host runtime (runtime.cpp).  The tile and lane
// kernel instances live in the kernels_tile_*.hip and kernels_lane.hip units.
#include <map>
#include <mutex>

#include "stage_kernels.h"
#include "resident_kernel.h"

namespace heom {

typedef StageKernel (*TilePart)(int N, int KP, bool mixed, bool streaming, bool scaled);
// Tile instances by shape and storage precision (_f1: FP64, _f0: FP32-mixed):
// N <= 8 in every shape, N = 9..12 in shape 0 only.
StageKernel tile_kernel_part_small_s0_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_small_s0_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_7_s0_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_7_s0_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_8_s0_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_8_s0_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_9_10_s0_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_9_10_s0_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_11_s0_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_11_s0_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_12_s0_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_12_s0_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_small_s1_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_small_s1_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_7_s1_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_7_s1_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_8_s1_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_8_s1_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_small_s2_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_small_s2_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_7_s2_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_7_s2_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_8_s2_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_8_s2_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_small_s3_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_small_s3_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_7_s3_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_7_s3_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_8_s3_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_8_s3_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_small_s4_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_small_s4_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_7_s4_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_7_s4_f0(int, int, bool, bool, bool);
StageKernel tile_kernel_part_8_s4_f1(int, int, bool, bool, bool);
StageKernel tile_kernel_part_8_s4_f0(int, int, bool, bool, bool);
StageKernel lane_kernel_ptr(int N, int KP, bool mixed);

namespace {

static_assert(kTileShapes == 5, "one row of tile parts per shape");
constexpr TilePart kTileParts[kTileShapes][12] = {
    {&tile_kernel_part_small_s0_f1, &tile_kernel_part_small_s0_f0, &tile_kernel_part_7_s0_f1,
     &tile_kernel_part_7_s0_f0, &tile_kernel_part_8_s0_f1, &tile_kernel_part_8_s0_f0,
     &tile_kernel_part_9_10_s0_f1, &tile_kernel_part_9_10_s0_f0, &tile_kernel_part_11_s0_f1,
     &tile_kernel_part_11_s0_f0, &tile_kernel_part_12_s0_f1, &tile_kernel_part_12_s0_f0},
    {&tile_kernel_part_small_s1_f1, &tile_kernel_part_small_s1_f0, &tile_kernel_part_7_s1_f1,
     &tile_kernel_part_7_s1_f0, &tile_kernel_part_8_s1_f1, &tile_kernel_part_8_s1_f0, nullptr,
     nullptr, nullptr, nullptr, nullptr, nullptr},
    {&tile_kernel_part_small_s2_f1, &tile_kernel_part_small_s2_f0, &tile_kernel_part_7_s2_f1,
     &tile_kernel_part_7_s2_f0, &tile_kernel_part_8_s2_f1, &tile_kernel_part_8_s2_f0, nullptr,
     nullptr, nullptr, nullptr, nullptr, nullptr},
    {&tile_kernel_part_small_s3_f1, &tile_kernel_part_small_s3_f0, &tile_kernel_part_7_s3_f1,
     &tile_kernel_part_7_s3_f0, &tile_kernel_part_8_s3_f1, &tile_kernel_part_8_s3_f0, nullptr,
     nullptr, nullptr, nullptr, nullptr, nullptr},
    {&tile_kernel_part_small_s4_f1, &tile_kernel_part_small_s4_f0, &tile_kernel_part_7_s4_f1,
     &tile_kernel_part_7_s4_f0, &tile_kernel_part_8_s4_f1, &tile_kernel_part_8_s4_f0, nullptr,
     nullptr, nullptr, nullptr, nullptr, nullptr},
};

StageKernel tile_kernel(int N, int KP, bool mixed, int shape, bool streaming = false,
                        bool scaled = false) {
  if (shape < 0 || shape >= kTileShapes) return nullptr;
  for (TilePart part : kTileParts[shape]) {
    StageKernel k = part ? part(N, KP, mixed, streaming, scaled) : nullptr;
    if (k) return k;
  }
  return nullptr;
}

}  // namespace

bool has_streaming_stores(int N, int KP, bool mixed, int shape) {
  return shape != kWideShape && tile_kernel(N, KP, mixed, shape, true) != nullptr;
}

bool has_fixed_kernel(int N, int KP) { return lane_kernel_ptr(N, KP, false) != nullptr; }

bool has_tile_kernel(int N, int KP) { return tile_kernel(N, KP, false, 0) != nullptr; }

// Whether the tile kernel runs scaled hierarchies of (N, K+1) (shape 0, plain
// stores: the one scaled instance).
bool has_scaled_tile_kernel(int N, int KP, bool mixed) {
  return tile_kernel(N, KP, mixed, 0, false, true) != nullptr;
}

// The wide kernel's LDS (tile, Hamiltonian, tables, and for scaled
// hierarchies `levels` weights per mode) must fit the 160 KB of a gfx950 CU.
bool has_wide_kernel(int N, int M, bool mixed, int levels) {
  constexpr int kLdsBytes = 160 * 1024;
  return N >= 1 && N <= kWideMaxN && M % N == 0 && M / N <= kWideMaxKP &&
         wide_lds(N, M, mixed ? 4 : 8, levels).total <= kLdsBytes;
}

namespace {
template <typename T, bool SCALED>
const void *wide_kernel_of(int KP) {
  static_assert(kWideMaxKP == 4, "one instance per K+1");
  switch (KP) {
    case 1: return reinterpret_cast<const void *>(&stage_wide<T, 1, SCALED>);
    case 2: return reinterpret_cast<const void *>(&stage_wide<T, 2, SCALED>);
    case 3: return reinterpret_cast<const void *>(&stage_wide<T, 3, SCALED>);
    case 4: return reinterpret_cast<const void *>(&stage_wide<T, 4, SCALED>);
  }
  return nullptr;
}
const void *wide_kernel(bool mixed, int KP, bool scaled) {
  if (mixed) return scaled ? wide_kernel_of<float, true>(KP) : wide_kernel_of<float, false>(KP);
  return scaled ? wide_kernel_of<double, true>(KP) : wide_kernel_of<double, false>(KP);
}
}  // namespace

bool tile_shape_info(int N, int KP, bool mixed, int shape, int *ados, int *threads,
                     int *elems_per_wave, int *chunk, int *min_waves) {
  int a, t, e, c, w;
  if (shape == kWideShape) {
    if (!has_wide_kernel(N, N * KP, mixed, 0)) return false;
    const int P = N * (N + 1) / 2;
    a = kWideAdos;
    t = 64 * kWideWaves;
    e = (P + kWideSlots - 1) / kWideSlots * (64 / kWideAdos);  // per wave, per ADO of the tile
    c = 1;
    w = 1;
  } else {
    if (!tile_kernel(N, KP, mixed, shape)) return false;
    const TileShape sh = tile_shape(!mixed, shape);
    a = kTile;
    t = 64 * tile_waves(N, !mixed, shape);
    e = sh.elems_per_wave;
    c = sh.chunk;
    w = sh.min_waves;
  }
  if (ados) *ados = a;
  if (threads) *threads = t;
  if (elems_per_wave) *elems_per_wave = e;
  if (chunk) *chunk = c;
  if (min_waves) *min_waves = w;
  return true;
}

// Dynamic LDS beyond the default limit has to be allowed per kernel; done
// once per configuration before any launch (and before graph capture).
hipError_t prepare_wide(int N, int M, bool mixed, int levels) {
  const int bytes = wide_lds(N, M, mixed ? 4 : 8, levels).total;
  const void *k = wide_kernel(mixed, M / N, levels > 0);
  if (!k) return hipErrorInvalidValue;
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// LDS bytes the resident kernel needs for an instance of n ADOs: the
// run-time-N kernel (fixed = false) or the compile-time one.
int resident_lds_bytes(int N, int M, int64_t n_ados, bool fixed) {
  const int n = static_cast<int>(n_ados);
  return fixed ? fixed_lds_bytes(N, n) : resident_lds(N, M, n).total;
}

// Threads per workgroup of the compile-time resident kernel with R items per
// thread: 1024 for one or two, 768 for three, 512 for four (the registers of
// the items).
int resident_threads(int R) { return R >= 4 ? 512 : (R == 3 ? 768 : 1024); }

// Cost of the compile-time resident kernel's LDS accesses for an instance of
// n ADOs with R items per thread: R passes over the 16-lane groups that hold
// items, each group that spans two elements weighted 11/8 for its bank
// conflicts (a count of LDS cycles per access up to a constant).  0 where
// the instance does not fit the workgroup.
int64_t resident_fixed_cost(int N, int64_t n_ados, int R) {
  const int64_t P = static_cast<int64_t>(N) * (N + 1) / 2;
  const int threads = resident_threads(R);
  const int64_t W = (n_ados + R - 1) / R;
  if (R < 1 || n_ados < 1 || P * W > threads) return 0;
  const int L = fixed_lanes(static_cast<int>(P), static_cast<int>(W), threads);
  return L % 16 == 0 ? R * P * (L / 16) * 8 : R * ((P * W + 15) / 16) * 11;
}

// The resident kernel with compile-time N, K+1 and items per thread R, or
// nullptr where not built (N <= 8, K+1 <= 2, 1 <= R <= 4).
template <int N, int KP>
const void *resident_fixed_r(int R) {
  switch (R) {
    case 1: return reinterpret_cast<const void *>(&stage_resident_fixed<N, KP, 1, 1024>);
    case 2: return reinterpret_cast<const void *>(&stage_resident_fixed<N, KP, 2, 1024>);
    case 3: return reinterpret_cast<const void *>(&stage_resident_fixed<N, KP, 3, 768>);
    case 4: return reinterpret_cast<const void *>(&stage_resident_fixed<N, KP, 4, 512>);
    default: return nullptr;
  }
}
template <int KP>
const void *resident_fixed_n(int N, int R) {
  switch (N) {
    case 1: return resident_fixed_r<1, KP>(R);
    case 2: return resident_fixed_r<2, KP>(R);
    case 3: return resident_fixed_r<3, KP>(R);
    case 4: return resident_fixed_r<4, KP>(R);
    case 5: return resident_fixed_r<5, KP>(R);
    case 6: return resident_fixed_r<6, KP>(R);
    case 7: return resident_fixed_r<7, KP>(R);
    case 8: return resident_fixed_r<8, KP>(R);
    default: return nullptr;
  }
}
const void *resident_kernel(int N, int KP, int R) {
  if (R == 0) return reinterpret_cast<const void *>(&stage_resident);
  if (KP == 1) return resident_fixed_n<1>(N, R);
  if (KP == 2) return resident_fixed_n<2>(N, R);
  return nullptr;
}

// Whether the compile-time resident kernel for (N, K+1, R) is built and
// keeps every value in registers (no scratch memory: a spilled operand would
// cost a memory round trip per stage).  A property of the code object, so
// each instance is asked once per process (a failed query is not kept).
bool resident_fixed_usable(int N, int KP, int R) {
  const void *k = R > 0 ? resident_kernel(N, KP, R) : nullptr;
  if (!k) return false;
  static std::mutex mu;
  static std::map<const void *, bool> known;
  {
    std::lock_guard<std::mutex> lock(mu);
    const auto it = known.find(k);
    if (it != known.end()) return it->second;
  }
  hipFuncAttributes attr{};
  if (hipFuncGetAttributes(&attr, k) != hipSuccess) return false;
  const bool usable = attr.localSizeBytes == 0;
  std::lock_guard<std::mutex> lock(mu);
  known[k] = usable;
  return usable;
}

// Lets the resident kernel (R = 0: run-time N; else the compile-time
// instance for N, K+1 and R items per thread) take `bytes` of dynamic LDS.
hipError_t prepare_resident(int N, int KP, int R, int bytes) {
  const void *k = resident_kernel(N, KP, R);
  if (!k) return hipErrorInvalidValue;
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// Steps step0 + 1 ... step0 + n_steps of n_inst resident instances, one
// workgroup each (descs[0 .. n_inst - 1]), on the kernel prepare_resident
// names for (N, KP, R).
hipError_t launch_resident(int N, int KP, int R, const InstDesc *descs, int n_inst,
                           int64_t step0, int64_t n_steps, int64_t record_every, int slot0,
                           double dt, int lds_bytes, hipStream_t stream) {
  const void *k = resident_kernel(N, KP, R);
  if (!k) return hipErrorInvalidValue;
  void *args[] = {&descs, &step0, &n_steps, &record_every, &slot0, &dt};
  const int threads = R == 0 ? kResidentThreads : resident_threads(R);
  return hipLaunchKernel(k, dim3(n_inst), dim3(threads), args, static_cast<size_t>(lds_bytes),
                         stream);
}

// `streaming` selects the tile kernel instance with non-temporal output
// stores (built for FP64 storage; the wide, lane and generic kernels always
// store plainly).  `levels` > 0: the group holds scaled hierarchies (wide
// kernel only) with weight tables of that many occupations per mode.
hipError_t launch_stage(KernelKind kind, bool mixed, int N, int KP, int shape,
                        const InstDesc *descs, const WorkItem *work, int n_items, int block,
                        int stage, double coef, int hist_slot, bool streaming, int levels,
                        hipStream_t stream) {
  if (kind == KernelKind::kTile && shape == kWideShape) {
    const size_t lds = static_cast<size_t>(wide_lds(N, N * KP, mixed ? 4 : 8, levels).total);
    const StageKernel k =
        reinterpret_cast<StageKernel>(const_cast<void *>(wide_kernel(mixed, KP, levels > 0)));
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(n_items), dim3(block), lds, stream, descs, work, stage, coef,
                       hist_slot);
    return hipGetLastError();
  }
  StageKernel k = nullptr;
  if (levels > 0 && kind != KernelKind::kTile) return hipErrorInvalidValue;
  switch (kind) {
    case KernelKind::kTile:
      // Scaled hierarchies: shape 0 with plain stores only.
      k = levels > 0 ? tile_kernel(N, KP, mixed, shape, false, true)
                     : tile_kernel(N, KP, mixed, shape, streaming);
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

// Scratch of the allocation-free entry point (heom_advance_slots_noalloc):
// the descriptors and work list of its launches, rewritten in full by every
// call (nothing in it needs to start at zero).  Each GPU the library runs on
// holds its own copy until the process ends.  Host code never uses the name
// `scratch` as an address: it takes the device address that
// hipGetSymbolAddress returns for the current device, once per device.
namespace {
__device__ __align__(256) char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;
}  // namespace

hipError_t static_scratch(int device, void **ptr) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) {
    *ptr = it->second;
    return hipSuccess;
  }
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  *ptr = p;
  return hipSuccess;
}

hipError_t launch_init(bool mixed, const InstDesc *descs, const WorkItem *work, int n_items,
                       int block, hipStream_t stream) {
  if (mixed)
    hipLaunchKernelGGL(init_state<float>, dim3(n_items), dim3(block), 0, stream, descs, work);
  else
    hipLaunchKernelGGL(init_state<double>, dim3(n_items), dim3(block), 0, stream, descs, work);
  return hipGetLastError();
}

hipError_t launch_filter(bool mixed, const InstDesc *descs, const WorkItem *work, int n_items,
                         hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  if (mixed)
    hipLaunchKernelGGL(filter_ados<float>, dim3(n_items), dim3(64), 0, stream, descs, work);
  else
    hipLaunchKernelGGL(filter_ados<double>, dim3(n_items), dim3(64), 0, stream, descs, work);
  return hipGetLastError();
}

hipError_t launch_halo(bool mixed, const InstDesc *descs, const HaloEntry *list, int n,
                       int stage, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((n + 255) / 256);
  if (mixed)
    hipLaunchKernelGGL(halo_fill<float>, grid, dim3(256), 0, stream, descs, list, n, stage);
  else
    hipLaunchKernelGGL(halo_fill<double>, grid, dim3(256), 0, stream, descs, list, n, stage);
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
