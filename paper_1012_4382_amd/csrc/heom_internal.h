// heom_internal.h -- structures shared by the host sources and the HIP kernels
// of libheom.so.  Not part of the public interface (include/heom.h).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "heom.h"

#ifdef __HIP__
#define HEOM_HD __host__ __device__
#else
#define HEOM_HD
#endif

namespace heom {

constexpr int kMaxSites = 64;
// Records of sigma_0 held on the device between copies to the host.
constexpr int64_t kRingRecords = 512;
// ADOs are padded to a multiple of this in every plane (one wave of lanes).
constexpr int64_t kPlanePad = 64;

// Layout of one ADO ("packed Hermitian", N*N reals): element e < N is the
// real diagonal entry (e, e); for each pair a < b in row-major order, with pair
// index p, element N + 2p is Re sigma_ab and element N + 2p + 1 is Im sigma_ab.
// In device memory each element has a plane of `stride` values (structure of
// arrays, so lanes that handle consecutive ADOs read consecutive addresses):
// diagonal element e of ADO i lives at e * stride + i, and the two planes of
// pair p form one block of (Re, Im) pairs, ADO i at (N + 2p) * stride + 2i and
// + 1, so one 16-byte access (8 in FP32 storage) moves both parts.
HEOM_HD inline int pair_index(int N, int a, int b) {  // a < b
  return a * N - a * (a + 1) / 2 + (b - a - 1);
}
// Index of packed element e of ADO i in planes of stride S.
HEOM_HD inline int64_t elem_index(int N, int e, int64_t S, int64_t i) {
  if (e < N) return e * S + i;
  const int q = (e - N) & 1;
  return (e - q) * S + 2 * i + q;
}

// Per-instance parameters, all converted to rad/fs (energies) and 1/fs
// (rates), laid out as one array of doubles in the workspace:
//   [0, N^2)           H_re (diagonal offset removed)
//   [N^2, 2N^2)        H_im
//   [2N^2, +N)         decay: (trap_a + rec_a) / 2
//   [.., +N)           delta_a (low-temperature correction residual)
//   [.., +N)           trap_a
//   [.., +N)           rec_a
//   [.., +M)           Re c_m
//   [.., +M)           Im c_m
//   [.., +M)           nu_m
//   [.., +N*N)         packed rho0 (used by the initialisation kernel)
//   [.., +ceil(R/2))   FP32 copy of the first R = rho0 entries, two floats
//                      per double (read by the FP32 stage kernels)
// and, for a scaled hierarchy (ADOs held divided by
// w_n = sqrt(prod_m n_m! |c_m|^n_m)), from `total` on, with L = depth + 1:
//   [total, +M*L)      up-coupling weight of mode m at occupation v,
//                      sqrt((v + 1)|c_m|), at m * L + v
//   [.., +M*L)         down-coupling weight, sqrt(v / |c_m|) (n_m's place)
struct ParamOffsets {
  int h_re, h_im, half_gamma, delta, trap, rec, c_re, c_im, nu, rho0, f32, total;
};
HEOM_HD inline ParamOffsets param_offsets(int N, int M) {
  ParamOffsets o;
  o.h_re = 0;
  o.h_im = N * N;
  o.half_gamma = 2 * N * N;
  o.delta = o.half_gamma + N;
  o.trap = o.delta + N;
  o.rec = o.trap + N;
  o.c_re = o.rec + N;
  o.c_im = o.c_re + M;
  o.nu = o.c_im + M;
  o.rho0 = o.nu + M;
  o.f32 = o.rho0 + N * N;
  o.total = o.f32 + (o.rho0 + 1) / 2;
  return o;
}

// Scalars carried with each state buffer: P_trap, P_rec, Q = int P_trap dt.
constexpr int kScalars = 4;  // padded

// InstDesc::flags: the instance's ADO 0 is not sigma_0 (one rank's share of
// a hierarchy split over ranks: sigma_0, the sinks and the records live on the
// rank that holds the first ADOs).
constexpr int32_t kInstNoSigma0 = 1;
// The instance holds the scaled ADOs (coupling weights after the parameters).
constexpr int32_t kInstScaled = 2;

// Device descriptor of one instance (lives in the workspace).
struct InstDesc {
  void *y, *a, *b;            // planes of the state and the two stage buffers (T*)
  double *y0, *a0, *b0;       // FP64 sigma_0 copies (mixed precision only)
  double *sc_y, *sc_a, *sc_b; // kScalars each
  double *hist;               // kRingRecords x (N*N + kScalars)
  const double *params;       // see ParamOffsets
  const int32_t *up, *down;   // [M][stride]
  const uint8_t *occ;         // [M][stride]
  int64_t n_ados, stride;
  int32_t N, M, KP, flags;
  int32_t levels, pad_;  // scaled: occupations 0 .. levels - 1 in the weight tables
  double filter_tol;     // > 0: ADOs below it are zeroed after every step
  // The neighbour tables as 16-bit offsets from the ADO's own index (0: no
  // neighbour), [M][stride], or null where an offset does not fit.
  const int16_t *up16, *down16;
};

// One halo ADO of a split hierarchy: before each stage, ADO src_index of
// instance src (its owner) is copied to slot dst_index of instance dst, in the
// stage's input buffer; only the rows and columns of the sites in `sites`
// (bit s for site s), the only entries the stage reads of it: element (a, b)
// of a neighbour along a mode of site s is used only where s is a or b.
struct HaloEntry {
  int32_t dst, dst_index, src, src_index;
  uint64_t sites;
};

// Stage kernel variants.
//  kTile:    real H, N <= 32; ADO tiles staged in LDS, in one of the launch
//            shapes below (default where built)
//  kLane:    N <= 8, real H; one lane per ADO, ADO held in registers
//  kGeneric: any N, complex H; one lane per ADO, reads from the planes
enum class KernelKind { kTile, kLane, kGeneric };

// Launch shapes of the LDS-tiled kernels, the autotuner's candidates:
// shapes 0 .. kWideShape - 1 are the 64-ADO tile kernel (N <= 12), shape
// kWideShape the 16-ADO wide kernel (N <= 32, LDS permitting).
constexpr int kWideShape = 5;
constexpr int kMaxTileShapes = kWideShape + 1;

// Size of the static device scratch of the allocation-free entry point
// (descriptors and work list of one call).
constexpr size_t kStaticScratchBytes = size_t{2} << 20;

// A block of ADOs of one instance: blockIdx.x -> (instance, first ADO).
// first = -1 marks the sigma_0 item of an FP32-mixed tile launch.
struct WorkItem {
  int32_t inst;
  int32_t first;
};

// Host-side handle of a stage kernel: (descriptors, work list, stage index,
// stage coefficient dt/4, dt/3, dt/2 or dt, history slot or -1).
typedef void (*StageKernel)(const InstDesc *, const WorkItem *, int, double, int);

}  // namespace heom

// Host-side hierarchy handle.
struct heom_hierarchy {
  int N = 0, K = 0, KP = 1, M = 0, depth = 0;
  int64_t n_ados = 0, stride = 0;
  bool h_real = true;
  bool scaled = false;      // ADOs held divided by w_n; weights after the parameters
  double filter_tol = 0.0;  // > 0: filter after every step (scaled hierarchies)
  double energy_offset = 0.0;  // removed mean site energy, rad/fs
  std::vector<double> params;  // ParamOffsets layout without rho0 filled
  std::vector<int32_t> site;   // [M]
  std::vector<double> c_re, c_im, nu, delta;
  std::vector<int32_t> multi;  // [n_ados][M]
  std::vector<int32_t> up, down;  // [M][stride] (device layout)
  std::vector<uint8_t> occ;       // [M][stride]
  // Device copies of the tables, per device ordinal.
  struct DeviceTables {
    int device = -1;
    int32_t *up = nullptr, *down = nullptr;
    uint8_t *occ = nullptr;
    int16_t *up16 = nullptr, *down16 = nullptr;  // null where an offset does not fit
  };
  mutable std::mutex mu;
  mutable std::vector<DeviceTables> dev;
};

// A hierarchy split over ranks: rank r owns the contiguous range
// [first[r], first[r + 1]) of the ADO order and is an instance of its own,
// whose tables point at its own ADOs (local index i - first[r]) and at halo
// slots n_local, n_local + 1, ... that hold copies of the other ranks' ADOs it
// couples to.  Rank 0 holds sigma_0.
struct heom_shard {
  int n_ranks = 0;
  int N = 0, M = 0;
  int64_t n_ados = 0;
  std::vector<heom_hierarchy *> rank;  // owned; n_ados = local ADOs, stride covers the halo
  std::vector<int64_t> first;          // [n_ranks + 1]
  std::vector<heom::HaloEntry> halo;   // every rank's halo, rank by rank
  struct Stats {
    int64_t n_halo = 0, cut_links = 0, halo_reals_min = 0;
  };
  std::vector<Stats> stats;
};

namespace heom {

// Thread-local error text.
void set_error(const std::string &msg);
int fail(int status, const std::string &msg);

// params.cpp
int build_params(const heom_system *sys, heom_hierarchy *h);
// hierarchy.cpp
int build_tables(heom_hierarchy *h);
// shard.cpp
int build_shard(const heom_hierarchy *h, int n_ranks, heom_shard *s);
// kernels_dispatch.hip: whether launch shape `shape` exists for (N, K+1,
// storage), and its ADOs per work item, threads per workgroup, elements per
// wave, load chunk and minimum waves per SIMD (any output may be NULL).
bool tile_shape_info(int N, int KP, bool mixed, int shape, int *ados, int *threads,
                     int *elems_per_wave, int *chunk, int *min_waves);
// kernels_dispatch.hip: whether launch shape `shape` also has an instance
// with non-temporal (streaming) output stores.
bool has_streaming_stores(int N, int KP, bool mixed, int shape);
// autotune.cpp: the launch shape and store policy of a tile group of n_tiles
// tiles, from the cache or, for a new key, by timing each candidate shape that
// available(shape) admits with time_shape(shape, streaming = false,
// &microseconds_per_launch), then the fastest one with streaming stores.
int autotune_choose(int device, bool mixed, int N, int KP, int64_t n_tiles,
                    const std::function<bool(int)> &available,
                    const std::function<int(int, bool, double *)> &time_shape, int *shape_out,
                    bool *streaming_out);
int autotune_lookup(int device, bool mixed, int N, int KP, int64_t n_tiles, int *shape,
                    int *streaming, double *us, double *us_streaming);
void autotune_clear();

}  // namespace heom
