// runtime.cpp -- C-ABI entry points of libheom.so (host side).
//
// Builds hierarchies (params.cpp, hierarchy.cpp), lays out caller-owned device
// workspaces, uploads per-instance parameters and neighbour tables, and
// sequences the RK4 stage kernels (stage_kernels.h) with the sigma_0
// history ring that is copied to the host in chunks (the paper keeps every
// ADO on the device and moves only the N x N reduced density matrix,
// Appendix B).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "heom_internal.h"

namespace heom {

// kernels_dispatch.hip
bool has_fixed_kernel(int N, int KP);
hipError_t prepare_wide(int N, int M, bool mixed, int levels);
bool has_wide_kernel(int N, int M, bool mixed, int levels);
bool has_scaled_tile_kernel(int N, int KP, bool mixed);
hipError_t launch_stage(KernelKind kind, bool mixed, int N, int KP, int shape,
                        const InstDesc *descs, const WorkItem *work, int n_items, int block,
                        int stage, double coef, int hist_slot, bool streaming, int levels,
                        hipStream_t stream);
hipError_t launch_filter(bool mixed, const InstDesc *descs, const WorkItem *work, int n_items,
                         hipStream_t stream);
hipError_t launch_init(bool mixed, const InstDesc *descs, const WorkItem *work, int n_items,
                       int block, hipStream_t stream);
hipError_t launch_snapshot(bool mixed, const InstDesc *descs, int n_inst, int slot,
                           hipStream_t stream);
hipError_t static_scratch(int device, void **ptr);
int resident_lds_bytes(int N, int M, int64_t n_ados, bool fixed);
bool resident_fixed_usable(int N, int KP, int R);
int64_t resident_fixed_cost(int N, int64_t n_ados, int R);
hipError_t prepare_resident(int N, int KP, int R, int bytes);
hipError_t launch_resident(int N, int KP, int R, const InstDesc *descs, int n_inst,
                           int64_t step0, int64_t n_steps, int64_t record_every, int slot0,
                           double dt, int lds_bytes, hipStream_t stream);
hipError_t launch_halo(bool mixed, const InstDesc *descs, const HaloEntry *list, int n,
                       int stage, hipStream_t stream);

namespace {

thread_local std::string g_last_error;

constexpr uint64_t kMagic = 0x48454f4d57530001ull;  // "HEOMWS" v1
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int dev_fail(hipError_t e, const char *what) {
  return fail(HEOM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HEOM_HIP(call, what)                      \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return dev_fail(e_, what); \
  } while (0)

// ADOs handled by one workgroup of the lane-per-ADO kernels.
int block_ados() {
  static int v = [] {
    const char *s = std::getenv("HEOM_BLOCK_ADOS");
    int b = s ? std::atoi(s) : 128;
    if (b != 64 && b != 128 && b != 256) b = 128;
    return b;
  }();
  return v;
}

struct Header {
  uint64_t magic;
  int64_t n_inst;
  int64_t precision;
  int64_t total_ados;
};

struct InstLayout {
  size_t params, y, a, b, y0, a0, b0, sc_y, sc_a, sc_b, hist;
};

struct Layout {
  size_t header = 0, descs = 0, work = 0;
  int64_t work_cap = 0;
  std::vector<InstLayout> inst;
  size_t total = 0;
};

// Work-list entries an instance of n_ados ADOs can need: its stage items in
// 16-ADO and in 64-ADO tiles (a group may carry both lists), the sigma_0 item
// of an FP32-mixed tile list, its initialisation and filter items (one per 64
// ADOs each) and the padding of each list to a multiple of the XCD count.
int64_t work_items_cap(int64_t n_ados) {
  return (n_ados + 15) / 16 + 3 * ((n_ados + kPlanePad - 1) / kPlanePad) + 16;
}

// Occupations per mode in the weight tables of a scaled hierarchy (0: not scaled).
int weight_levels(const heom_hierarchy *h) { return h->scaled ? h->depth + 1 : 0; }

Layout make_layout(heom_hierarchy *const *hs, int n, int precision) {
  Layout L;
  size_t off = 0;
  L.header = off;
  off = align_up(off + sizeof(Header));
  L.descs = off;
  off = align_up(off + sizeof(InstDesc) * n);
  int64_t cap = 0;
  for (int k = 0; k < n; ++k) cap += work_items_cap(hs[k]->n_ados);
  L.work = off;
  L.work_cap = cap;
  off = align_up(off + sizeof(WorkItem) * cap);
  const size_t elt = (precision == HEOM_FP32_MIXED) ? 4 : 8;
  L.inst.resize(n);
  for (int k = 0; k < n; ++k) {
    const heom_hierarchy *h = hs[k];
    const size_t N2 = static_cast<size_t>(h->N) * h->N;
    InstLayout &I = L.inst[k];
    I.params = off;
    off = align_up(off + sizeof(double) * h->params.size());
    const size_t plane_bytes = elt * N2 * static_cast<size_t>(h->stride);
    I.y = off;
    off = align_up(off + plane_bytes);
    I.a = off;
    off = align_up(off + plane_bytes);
    I.b = off;
    off = align_up(off + plane_bytes);
    I.y0 = off;
    off = align_up(off + sizeof(double) * N2);
    I.a0 = off;
    off = align_up(off + sizeof(double) * N2);
    I.b0 = off;
    off = align_up(off + sizeof(double) * N2);
    I.sc_y = off;
    off = align_up(off + sizeof(double) * kScalars);
    I.sc_a = off;
    off = align_up(off + sizeof(double) * kScalars);
    I.sc_b = off;
    off = align_up(off + sizeof(double) * kScalars);
    I.hist = off;
    off = align_up(off + sizeof(double) * (N2 + kScalars) * kRingRecords);
  }
  L.total = off;
  return L;
}

// h's neighbour tables as offsets from each ADO's own index (0 where there is
// no neighbour: no ADO is its own neighbour), or false where an offset does
// not fit 16 bits.
bool tables16(const heom_hierarchy *h, std::vector<int16_t> *u16, std::vector<int16_t> *d16) {
  const size_t n = h->up.size();
  const int64_t S = h->stride;
  if (S <= 0 || n == 0) return false;
  u16->assign(n, 0);
  d16->assign(n, 0);
  for (size_t q = 0; q < n; ++q) {
    const int64_t i = static_cast<int64_t>(q % static_cast<size_t>(S));
    const int32_t ju = h->up[q], jd = h->down[q];
    for (int side = 0; side < 2; ++side) {
      const int32_t j = side ? jd : ju;
      if (j < 0) continue;
      const int64_t delta = j - i;
      if (delta == 0 || delta < -32767 || delta > 32767) return false;
      (side ? *d16 : *u16)[q] = static_cast<int16_t>(delta);
    }
  }
  return true;
}

// The device copy of h's neighbour tables on `device`, uploaded on first use
// (with upload = false a missing copy is an error: nothing is allocated).
int ensure_device_tables(const heom_hierarchy *h, int device, heom_hierarchy::DeviceTables *out,
                         bool upload = true) {
  std::lock_guard<std::mutex> lock(h->mu);
  for (const auto &t : h->dev)
    if (t.device == device) {
      *out = t;
      return HEOM_OK;
    }
  if (!upload)
    return fail(HEOM_E_UNSUPPORTED,
                "the neighbour tables of a hierarchy are not on this device yet (an allocating "
                "call with that hierarchy on this device uploads them)");
  heom_hierarchy::DeviceTables t;
  t.device = device;
  const size_t n32 = h->up.size() * sizeof(int32_t);
  const size_t n8 = h->occ.size();
  hipError_t e;
  if ((e = hipMalloc(reinterpret_cast<void **>(&t.up), n32)) != hipSuccess)
    return dev_fail(e, "hipMalloc(tables)");
  if ((e = hipMalloc(reinterpret_cast<void **>(&t.down), n32)) != hipSuccess) {
    (void)hipFree(t.up);
    return dev_fail(e, "hipMalloc(tables)");
  }
  if ((e = hipMalloc(reinterpret_cast<void **>(&t.occ), n8)) != hipSuccess) {
    (void)hipFree(t.up);
    (void)hipFree(t.down);
    return dev_fail(e, "hipMalloc(tables)");
  }
  if ((e = hipMemcpy(t.up, h->up.data(), n32, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(t.down, h->down.data(), n32, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(t.occ, h->occ.data(), n8, hipMemcpyHostToDevice)) != hipSuccess) {
    (void)hipFree(t.up);
    (void)hipFree(t.down);
    (void)hipFree(t.occ);
    return dev_fail(e, "hipMemcpy(tables)");
  }
  // The 16-bit form, where every neighbour lies within 32767 ADOs: the stage
  // kernels stage it instead, 4 bytes per mode and ADO instead of 8.
  std::vector<int16_t> u16, d16;
  if (tables16(h, &u16, &d16)) {
    const size_t n16 = u16.size() * sizeof(int16_t);
    bool ok = hipMalloc(reinterpret_cast<void **>(&t.up16), n16) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void **>(&t.down16), n16) == hipSuccess;
    ok = ok && hipMemcpy(t.up16, u16.data(), n16, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(t.down16, d16.data(), n16, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
      // An optional copy: without it the kernels stage the 32-bit tables.
      (void)hipGetLastError();
      if (t.up16) (void)hipFree(t.up16);
      if (t.down16) (void)hipFree(t.down16);
      t.up16 = t.down16 = nullptr;
    }
  }
  h->dev.push_back(t);
  *out = t;
  return HEOM_OK;
}

// Packs a Hermitian N x N complex matrix into N*N reals (plane order).
int pack_hermitian(int N, const double *rho, double *packed) {
  double mx = 0.0;
  for (int k = 0; k < 2 * N * N; ++k) {
    if (!std::isfinite(rho[k])) return fail(HEOM_E_INVALID, "rho0 has a non-finite entry");
    mx = std::fmax(mx, std::fabs(rho[k]));
  }
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) {
      const double dr = rho[2 * (a * N + b)] - rho[2 * (b * N + a)];
      const double di = rho[2 * (a * N + b) + 1] + rho[2 * (b * N + a) + 1];
      if (std::fabs(dr) > 1e-12 * mx || std::fabs(di) > 1e-12 * mx)
        return fail(HEOM_E_INVALID, "rho0 is not Hermitian");
    }
  for (int a = 0; a < N; ++a) packed[a] = rho[2 * (a * N + a)];
  for (int a = 0; a < N; ++a)
    for (int b = a + 1; b < N; ++b) {
      const int e = N + 2 * pair_index(N, a, b);
      packed[e] = rho[2 * (a * N + b)];
      packed[e + 1] = rho[2 * (a * N + b) + 1];
    }
  return HEOM_OK;
}

void unpack_hermitian(int N, const double *packed, double *rho) {
  for (int a = 0; a < N; ++a) {
    rho[2 * (a * N + a)] = packed[a];
    rho[2 * (a * N + a) + 1] = 0.0;
    for (int b = a + 1; b < N; ++b) {
      const int e = N + 2 * pair_index(N, a, b);
      rho[2 * (a * N + b)] = packed[e];
      rho[2 * (a * N + b) + 1] = packed[e + 1];
      rho[2 * (b * N + a)] = packed[e];
      rho[2 * (b * N + a) + 1] = -packed[e + 1];
    }
  }
}

// Steps captured in one graph.
constexpr int64_t kGraphSteps = 32;

// Tolerance of the population health check (relative to the conserved
// value); HEOM_DRIFT_TOL overrides it.
double population_drift_tol() {
  const char *s = std::getenv("HEOM_DRIFT_TOL");
  if (s && s[0]) {
    const double v = std::atof(s);
    if (v > 0.0) return v;
  }
  return 1e-7;
}

// MI355X has 8 XCDs, each with its own L2; workgroups are dispatched to them
// round-robin by workgroup index.
constexpr int64_t kXcds = 8;

// XCD-aware ordering of the work list (HEOM_XCD_REMAP=0 turns it off).
bool xcd_remap() {
  static bool v = [] {
    const char *s = std::getenv("HEOM_XCD_REMAP");
    return !(s && s[0] == '0');
  }();
  return v;
}

// A private stream per device and host thread, used only to capture graphs
// (capture on the caller's stream is not possible when it is the legacy
// default stream).  Default priority.
int capture_stream(int device, hipStream_t *out) {
  thread_local std::map<int, hipStream_t> streams;
  auto it = streams.find(device);
  if (it != streams.end()) {
    *out = it->second;
    return HEOM_OK;
  }
  hipStream_t s;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return dev_fail(e, "hipStreamCreateWithFlags");
  streams[device] = s;
  *out = s;
  return HEOM_OK;
}

// Streams and events that let the kernel groups of one RK4 stage run side by
// side: each group's launch touches only its own instances, so only the
// stages must follow each other.  One set per device and host thread, kept
// for the life of the process; default priority.
struct ForkJoin {
  hipEvent_t fork = nullptr;
  std::vector<hipStream_t> aux;  // aux[g], g >= 1: stream of group g
  std::vector<hipEvent_t> join;  // join[g]: group g's launch is done
};

int fork_join(int device, size_t n_groups, ForkJoin **out) {
  thread_local std::map<int, ForkJoin> sets;
  ForkJoin &f = sets[device];
  if (!f.fork) {
    hipError_t e = hipEventCreateWithFlags(&f.fork, hipEventDisableTiming);
    if (e != hipSuccess) {
      f.fork = nullptr;
      return dev_fail(e, "hipEventCreateWithFlags");
    }
    f.aux.push_back(nullptr);  // group 0 runs on the caller's stream
    f.join.push_back(nullptr);
  }
  while (f.aux.size() < n_groups) {
    hipStream_t st;
    hipEvent_t ev;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return dev_fail(e, "hipStreamCreateWithFlags");
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipStreamDestroy(st);
      return dev_fail(e, "hipEventCreateWithFlags");
    }
    f.aux.push_back(st);
    f.join.push_back(ev);
  }
  *out = &f;
  return HEOM_OK;
}

// A graph of k RK4 steps, destroyed with the object.
struct StepGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  template <typename Enqueue>
  int build(int device, int64_t k, Enqueue enqueue_step) {
    hipStream_t cap;
    int rc = capture_stream(device, &cap);
    if (rc) return rc;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return dev_fail(e, "hipStreamBeginCapture");
    hipError_t launch_err = hipSuccess;
    for (int64_t i = 0; i < k && launch_err == hipSuccess; ++i) launch_err = enqueue_step(cap);
    e = hipStreamEndCapture(cap, &graph);
    if (launch_err != hipSuccess) return dev_fail(launch_err, "stage kernel (capture)");
    if (e != hipSuccess) return dev_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return dev_fail(e, "hipGraphInstantiate");
    return HEOM_OK;
  }
  ~StepGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

// The instances of one launch per stage.  A kTile group carries a work list
// for each item size its launch shapes use (64-ADO tiles, 16-ADO wide tiles);
// the chosen shape selects one.
struct Group {
  KernelKind kind;
  int N, KP;
  int levels = 0;  // scaled hierarchies: weight levels (wide kernel only)
  int shape;    // launch shape (kTile only)
  bool streaming = false;  // non-temporal output stores (kTile only)
  int threads;  // of the chosen shape
  int64_t n_tiles;  // 64-ADO tiles of the group (the autotuner's size key)
  int64_t begin[2] = {0, 0}, count[2] = {0, 0};  // work lists: [0] 64-ADO, [1] 16-ADO items
  int list(int s) const { return (kind == KernelKind::kTile && s == kWideShape) ? 1 : 0; }
};

// Whether launch shape s can run hierarchy h: built for its N and K+1, and
// for the wide kernel, whose loads use 32-bit byte offsets from the buffer
// bases, state buffers below 4 GiB.
bool shape_ok(const heom_hierarchy *h, bool mixed, int s) {
  if (h->scaled) {  // tile shape 0 or the wide kernel (with its weight tables in LDS)
    if (s == 0) return has_scaled_tile_kernel(h->N, h->KP, mixed);
    if (s != kWideShape || !has_wide_kernel(h->N, h->M, mixed, weight_levels(h))) return false;
  } else if (!tile_shape_info(h->N, h->KP, mixed, s, nullptr, nullptr, nullptr, nullptr,
                              nullptr)) {
    return false;
  }
  if (s != kWideShape) return true;
  const uint64_t bytes = static_cast<uint64_t>(h->N) * h->N * h->stride * (mixed ? 4 : 8);
  return bytes < (uint64_t{1} << 32);
}

// Whether h has any LDS-tiled launch shape.
bool has_tiled(const heom_hierarchy *h, bool mixed) {
  for (int s = 0; s < kMaxTileShapes; ++s)
    if (shape_ok(h, mixed, s)) return true;
  return false;
}

// Stage sequences timed per candidate shape by the autotuner (after one
// untimed sequence).
constexpr int kTuneReps = 5;

// Tile launch shape forced by the flags (HEOM_TILE_SHAPE(s)), or -1.
int forced_shape(int flags) { return ((flags >> 8) & 0xf) - 1; }

// Store policy of the tile kernels forced by the flags: 1 streaming (where
// such an instance is built), 0 plain, -1 not forced.
int forced_streaming(int flags) {
  if (flags & HEOM_STREAMING_STORES) return 1;
  if (flags & HEOM_PLAIN_STORES) return 0;
  return -1;
}

constexpr int kShapeFlagMask = 0xf00;

// LDS of one CU that the resident kernel may take, and its longest launch in
// steps (a launch of a long run is cut into chunks of this many steps).
constexpr int kResidentMaxLds = 160 * 1024;
constexpr int64_t kResidentChunkSteps = 4096;
// Where one workgroup runs a stage faster than a stage launch.  The
// compile-time kernel (every instance of the call with the same N <= 8 and
// K+1 <= 2) holds each thread's element operands in registers and takes R
// items (packed element x ADO) per thread: one or two on 1024 threads, three
// on 768, four on 512, each only where that instance needs no scratch
// memory; measured 1.6-6x faster than stage launches from the dimer to 8
// sites at depth 2.  The run-time-N
// kernel, for calls that mix hierarchies, takes one item per thread and few
// sites (its per-element chain grows with N: the dimer 2.3x faster, 7 sites
// at depth 2 0.86x).
constexpr int64_t kResidentMaxItems = 1024;  // the run-time kernel's threads: one item each
constexpr int kResidentMaxSites = 4;
constexpr int kResidentFixedSites = 8;
constexpr int kResidentMaxR = 4;

// The resident kernel of a call: its LDS bytes (0: the call does not fit a
// resident kernel) and which one, R = 0 for the run-time-N kernel, else the
// compile-time instance for (N, KP) with R items per thread.
struct ResidentPlan {
  int bytes = 0;
  int N = 0, KP = 0, R = 0;
};

// FP64 storage, hierarchies the LDS-tiled kernels run (real H), unscaled and
// unfiltered, no split, small enough, and no flag that asks for another
// kernel.  A call whose instances share N and K+1 takes the compile-time
// kernel, with the items per thread whose LDS accesses cost least on its
// costliest instance (more items only where that saves over a tenth: fewer
// items per thread leave more waves to hide latency with).
ResidentPlan resident_plan(heom_hierarchy *const *hs, int n, bool mixed, int flags, bool split) {
  const ResidentPlan none;
  if (mixed || split || n < 1) return none;
  if (flags & (HEOM_NO_RESIDENT | HEOM_GENERIC_KERNEL | HEOM_LANE_KERNEL)) return none;
  if (forced_shape(flags) >= 0) return none;
  int bytes_rt = 0, bytes_fx = 0;
  bool same = true, small = true;
  for (int k = 0; k < n; ++k) {
    const heom_hierarchy *h = hs[k];
    // The LDS-tiled kernels' domain (real H, N and K+1 they are built for):
    // there the two paths agree bitwise.
    if (!h->h_real || h->scaled || h->filter_tol > 0.0 || !has_tiled(h, false)) return none;
    const int64_t P = static_cast<int64_t>(h->N) * (h->N + 1) / 2;
    if (h->n_ados > (1 << 20)) return none;
    bytes_rt = std::max(bytes_rt, resident_lds_bytes(h->N, h->M, h->n_ados, false));
    bytes_fx = std::max(bytes_fx, resident_lds_bytes(h->N, h->M, h->n_ados, true));
    same = same && h->N == hs[0]->N && h->KP == hs[0]->KP;
    small = small && h->N <= kResidentMaxSites && h->n_ados * P <= kResidentMaxItems;
  }
  ResidentPlan plan;
  if (same && hs[0]->N <= kResidentFixedSites && hs[0]->KP <= 2 && bytes_fx <= kResidentMaxLds) {
    int64_t best = 0;
    for (int r = 1; r <= kResidentMaxR; ++r) {
      int64_t cost = 0;
      for (int k = 0; k < n; ++k) {
        const int64_t c = resident_fixed_cost(hs[0]->N, hs[k]->n_ados, r);
        if (c == 0) {
          cost = 0;
          break;
        }
        cost = std::max(cost, c);
      }
      if (cost == 0 || (plan.R > 0 && 10 * cost >= 9 * best)) continue;
      if (!resident_fixed_usable(hs[0]->N, hs[0]->KP, r)) continue;
      plan.R = r;
      best = cost;
    }
    if (plan.R > 0) {
      plan.bytes = bytes_fx;
      plan.N = hs[0]->N;
      plan.KP = hs[0]->KP;
      return plan;
    }
  }
  if (small && bytes_rt <= kResidentMaxLds) plan.bytes = bytes_rt;
  return plan;
}

// Where the device data of one call live: each instance's regions (offsets
// relative to its own base), the headers that identify the runs held there,
// and the descriptor array and work list of the launch.
struct RunPlace {
  std::vector<char *> base;       // per instance
  std::vector<InstLayout> inst;   // per instance, relative to base
  std::vector<char *> header;     // header regions
  std::vector<Header> want;       // their contents for this call
  std::vector<int> header_of;     // per instance: its header region
  char *descs = nullptr, *work = nullptr;
  int64_t work_cap = 0;
};

int check_common(heom_hierarchy *const *hs, int n, int precision, int flags, double dt_fs,
                 int64_t n_steps, int64_t record_every, int allowed_flags) {
  if (!hs || n < 1) return fail(HEOM_E_INVALID, "no hierarchies");
  for (int k = 0; k < n; ++k)
    if (!hs[k]) return fail(HEOM_E_INVALID, "NULL hierarchy handle");
  if (precision != HEOM_FP64 && precision != HEOM_FP32_MIXED)
    return fail(HEOM_E_UNSUPPORTED, "precision must be HEOM_FP64 or HEOM_FP32_MIXED");
  if (flags & ~allowed_flags) return fail(HEOM_E_INVALID, "unknown flags");
  if ((flags & HEOM_GENERIC_KERNEL) && (flags & HEOM_LANE_KERNEL))
    return fail(HEOM_E_INVALID, "HEOM_GENERIC_KERNEL and HEOM_LANE_KERNEL are exclusive");
  if ((flags & HEOM_STREAMING_STORES) && (flags & HEOM_PLAIN_STORES))
    return fail(HEOM_E_INVALID, "HEOM_STREAMING_STORES and HEOM_PLAIN_STORES are exclusive");
  if (!(dt_fs > 0.0) || !std::isfinite(dt_fs)) return fail(HEOM_E_INVALID, "dt_fs must be > 0");
  if (n_steps < 0) return fail(HEOM_E_INVALID, "n_steps must be >= 0");
  if (record_every < 1) return fail(HEOM_E_INVALID, "record_every must be >= 1");
  // A forced launch shape must exist for every instance the LDS-tiled
  // kernels will run.
  const int forced = forced_shape(flags);
  if (forced >= kMaxTileShapes) return fail(HEOM_E_INVALID, "tile launch shape out of range");
  const bool mixed = precision == HEOM_FP32_MIXED;
  for (int k = 0; k < n; ++k)
    if (hs[k]->scaled) {
      if (flags & (HEOM_GENERIC_KERNEL | HEOM_LANE_KERNEL))
        return fail(HEOM_E_UNSUPPORTED, "scaled hierarchies run on the LDS-tiled kernels only");
      if (!shape_ok(hs[k], mixed, 0) && !shape_ok(hs[k], mixed, kWideShape))
        return fail(HEOM_E_UNSUPPORTED,
                    "scaled hierarchies need the tile kernel (N <= 12, K + 1 <= 2) or the wide "
                    "kernel (real H, N <= 32, K + 1 <= 4, its LDS within 160 KB and state "
                    "buffers below 4 GiB)");
      if (forced >= 0 && !shape_ok(hs[k], mixed, forced))
        return fail(HEOM_E_UNSUPPORTED, "scaled hierarchies run in tile launch shape 0 or " +
                                            std::to_string(kWideShape) + " only");
    }
  if (forced >= 0 && !(flags & (HEOM_GENERIC_KERNEL | HEOM_LANE_KERNEL)))
    for (int k = 0; k < n; ++k) {
      const heom_hierarchy *h = hs[k];
      if (h->scaled) continue;  // checked above
      if (h->h_real && has_tiled(h, mixed) && !shape_ok(h, mixed, forced))
        return fail(HEOM_E_UNSUPPORTED, "tile launch shape " + std::to_string(forced) +
                                            " is not built for N=" + std::to_string(h->N) +
                                            ", K+1=" + std::to_string(h->KP));
    }
  return HEOM_OK;
}

// Propagates n instances placed as described by `place`.  start[k] = 1
// initialises instance k from rho0s[k]; 0 continues the run held there.
// How run_impl runs.
struct RunOptions {
  // Fail with HEOM_E_NUMERIC at the first non-finite record (otherwise the
  // records are returned as they are and the caller checks them).
  bool check_numeric = true;
  // Allocate nothing on the device (and create no stream, event or graph):
  // tables must already be resident, launch shapes come from the autotuner's
  // cache or the defaults, every launch goes directly to the caller's stream.
  bool no_alloc = false;
  // The instances are the ranks of one split hierarchy: instances after the
  // first do not hold sigma_0, and the n_halo entries at d_halo are copied
  // into each stage's input before the stage runs.
  bool shard = false;
  const HaloEntry *d_halo = nullptr;
  int n_halo = 0;
};

int run_impl(heom_hierarchy *const *hs, int n, int precision, int flags, const int32_t *start,
             const double *const *rho0s, double dt_fs, int64_t n_steps, int64_t record_every,
             const RunPlace &place, void *hip_stream, double *const *rho_outs,
             double *const *sinks_outs, const RunOptions &opt = RunOptions()) {
  const bool check_numeric = opt.check_numeric;
  const bool mixed = precision == HEOM_FP32_MIXED;
  // Packed initial states (validated before any device work).
  std::vector<std::vector<double>> params(n);
  for (int k = 0; k < n; ++k) {
    params[k] = hs[k]->params;
    if (start[k]) {
      if (!rho0s || !rho0s[k]) return fail(HEOM_E_INVALID, "rho0 is NULL");
      const ParamOffsets o = param_offsets(hs[k]->N, hs[k]->M);
      int rc = pack_hermitian(hs[k]->N, rho0s[k], params[k].data() + o.rho0);
      if (rc) return rc;
    }
  }
  // A header region is either started or continued as a whole.
  std::vector<int> hdr_start(place.header.size(), -1);
  for (int k = 0; k < n; ++k) {
    int &hs_ = hdr_start[place.header_of[k]];
    const int s = start[k] ? 1 : 0;
    if (hs_ >= 0 && hs_ != s)
      return fail(HEOM_E_INVALID, "instances sharing a workspace must all start or all resume");
    hs_ = s;
  }

  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  int device = 0;
  HEOM_HIP(hipGetDevice(&device), "hipGetDevice");

  // Descriptors and work list.
  std::vector<InstDesc> descs(n);
  for (int k = 0; k < n; ++k) {
    heom_hierarchy::DeviceTables t;
    int rc = ensure_device_tables(hs[k], device, &t, !opt.no_alloc);
    if (rc) return rc;
    char *ws = place.base[k];
    const InstLayout &I = place.inst[k];
    InstDesc &d = descs[k];
    d.y = ws + I.y;
    d.a = ws + I.a;
    d.b = ws + I.b;
    d.y0 = reinterpret_cast<double *>(ws + I.y0);
    d.a0 = reinterpret_cast<double *>(ws + I.a0);
    d.b0 = reinterpret_cast<double *>(ws + I.b0);
    d.sc_y = reinterpret_cast<double *>(ws + I.sc_y);
    d.sc_a = reinterpret_cast<double *>(ws + I.sc_a);
    d.sc_b = reinterpret_cast<double *>(ws + I.sc_b);
    d.hist = reinterpret_cast<double *>(ws + I.hist);
    d.params = reinterpret_cast<const double *>(ws + I.params);
    d.up = t.up;
    d.down = t.down;
    d.occ = t.occ;
    d.up16 = t.up16;
    d.down16 = t.down16;
    d.n_ados = hs[k]->n_ados;
    d.stride = hs[k]->stride;
    d.N = hs[k]->N;
    d.M = hs[k]->M;
    d.KP = hs[k]->KP;
    d.flags = ((opt.shard && k > 0) ? kInstNoSigma0 : 0) | (hs[k]->scaled ? kInstScaled : 0);
    d.levels = weight_levels(hs[k]);
    d.pad_ = 0;
    d.filter_tol = hs[k]->filter_tol;
  }
  std::map<std::tuple<int, int, int, int>, std::vector<int>> by_key;
  for (int k = 0; k < n; ++k) {
    const heom_hierarchy *h = hs[k];
    KernelKind kind = KernelKind::kGeneric;
    if (h->scaled) {
      kind = KernelKind::kTile;  // validated by check_common: tile shape 0 or wide
    } else if (!(flags & HEOM_GENERIC_KERNEL) && h->h_real) {
      if (flags & HEOM_LANE_KERNEL) {
        if (has_fixed_kernel(h->N, h->KP)) kind = KernelKind::kLane;
      } else if (has_tiled(h, mixed)) {
        kind = KernelKind::kTile;
      }
    }
    const int kp = (kind == KernelKind::kGeneric) ? 0 : h->KP;
    by_key[std::make_tuple(static_cast<int>(kind), h->N, kp, weight_levels(h))].push_back(k);
  }
  std::vector<WorkItem> items;
  std::vector<Group> groups;
  // Appends the work list of `members` in items of `ados` ADOs, XCD-ordered;
  // with `sigma0`, each instance's items are preceded by its sigma_0 item
  // (first = -1, the FP64 update of sigma_0 in FP32-mixed tile launches).
  auto add_list = [&](const std::vector<int> &members, int64_t ados, bool sigma0, int64_t *begin,
                      int64_t *count) {
    std::vector<WorkItem> mine;
    for (int k : members) {
      if (sigma0) mine.push_back({k, -1});
      for (int64_t first = 0; first < hs[k]->n_ados; first += ados)
        mine.push_back({k, static_cast<int32_t>(first)});
    }
    if (xcd_remap()) {
      // Workgroup b runs on XCD b % kXcds.  Give XCD x the x-th contiguous
      // eighth of the list (consecutive tiles of the same instance), so that
      // neighbour gathers hit the L2 of the XCD that staged their tiles.
      // Padding items start past the instance's last ADO and exit at once.
      const int64_t len = (static_cast<int64_t>(mine.size()) + kXcds - 1) / kXcds;
      const WorkItem pad = {mine.back().inst, static_cast<int32_t>(hs[mine.back().inst]->n_ados)};
      mine.resize(len * kXcds, pad);
      std::vector<WorkItem> perm(mine.size());
      for (int64_t b = 0; b < static_cast<int64_t>(perm.size()); ++b)
        perm[b] = mine[(b % kXcds) * len + b / kXcds];
      mine.swap(perm);
    }
    *begin = static_cast<int64_t>(items.size());
    *count = static_cast<int64_t>(mine.size());
    items.insert(items.end(), mine.begin(), mine.end());
  };
  for (const auto &kv : by_key) {
    Group g;
    g.kind = static_cast<KernelKind>(std::get<0>(kv.first));
    g.N = std::get<1>(kv.first);
    g.KP = std::get<2>(kv.first);
    g.levels = std::get<3>(kv.first);
    g.shape = 0;
    g.n_tiles = 0;
    for (int k : kv.second) g.n_tiles += (hs[k]->n_ados + kPlanePad - 1) / kPlanePad;
    if (g.kind == KernelKind::kTile) {
      bool tile = true, wide = true;
      for (int k : kv.second) {
        tile = tile && shape_ok(hs[k], mixed, 0);
        wide = wide && shape_ok(hs[k], mixed, kWideShape);
      }
      if (tile) add_list(kv.second, kPlanePad, mixed, &g.begin[0], &g.count[0]);
      if (wide) {
        add_list(kv.second, 16, false, &g.begin[1], &g.count[1]);
        HEOM_HIP(prepare_wide(g.N, g.N * g.KP, mixed, g.levels), "wide kernel attributes");
      }
      g.shape = tile ? 0 : kWideShape;
      tile_shape_info(g.N, g.KP, mixed, g.shape, nullptr, &g.threads, nullptr, nullptr, nullptr);
    } else {
      g.threads = block_ados();
      add_list(kv.second, g.threads, false, &g.begin[0], &g.count[0]);
    }
    groups.push_back(g);
  }
  // Initialisation items (64 ADOs each) of the instances that start here.
  const int64_t init_begin = static_cast<int64_t>(items.size());
  for (int k = 0; k < n; ++k)
    if (start[k])
      for (int64_t first = 0; first < hs[k]->n_ados; first += kPlanePad)
        items.push_back({k, static_cast<int32_t>(first)});
  const int64_t n_init = static_cast<int64_t>(items.size()) - init_begin;
  // Filter items (64 ADOs each) of the instances with a filter.
  const int64_t filter_begin = static_cast<int64_t>(items.size());
  for (int k = 0; k < n; ++k)
    if (hs[k]->filter_tol > 0.0)
      for (int64_t first = 0; first < hs[k]->n_ados; first += kPlanePad)
        items.push_back({k, static_cast<int32_t>(first)});
  const int64_t n_filter = static_cast<int64_t>(items.size()) - filter_begin;
  if (static_cast<int64_t>(items.size()) > place.work_cap)
    return fail(HEOM_E_WORKSPACE, "work list exceeds its workspace region");

  // Continued runs must be the runs these hierarchies left in the workspace.
  for (size_t r = 0; r < place.header.size(); ++r) {
    if (hdr_start[r] != 0) continue;
    Header cur;
    HEOM_HIP(hipMemcpyAsync(&cur, place.header[r], sizeof(Header), hipMemcpyDeviceToHost, stream),
             "hipMemcpyAsync(header)");
    HEOM_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (std::memcmp(&cur, &place.want[r], sizeof(Header)) != 0)
      return fail(HEOM_E_WORKSPACE, "workspace does not hold a run of these hierarchies");
  }
  HEOM_HIP(hipMemcpyAsync(place.descs, descs.data(), sizeof(InstDesc) * n, hipMemcpyHostToDevice,
                          stream),
           "hipMemcpyAsync(descs)");
  HEOM_HIP(hipMemcpyAsync(place.work, items.data(), sizeof(WorkItem) * items.size(),
                          hipMemcpyHostToDevice, stream),
           "hipMemcpyAsync(work)");
  for (int k = 0; k < n; ++k)
    HEOM_HIP(hipMemcpyAsync(place.base[k] + place.inst[k].params, params[k].data(),
                            sizeof(double) * params[k].size(), hipMemcpyHostToDevice, stream),
             "hipMemcpyAsync(params)");
  const InstDesc *d_descs = reinterpret_cast<const InstDesc *>(place.descs);
  const WorkItem *d_work = reinterpret_cast<const WorkItem *>(place.work);
  if (n_init > 0)
    HEOM_HIP(launch_init(mixed, d_descs, d_work + init_begin, static_cast<int>(n_init),
                         static_cast<int>(kPlanePad), stream),
             "init kernel");
  for (size_t r = 0; r < place.header.size(); ++r)
    if (hdr_start[r] == 1)
      HEOM_HIP(hipMemcpyAsync(place.header[r], &place.want[r], sizeof(Header),
                              hipMemcpyHostToDevice, stream),
               "hipMemcpyAsync(header)");

  bool want_rho = false;
  for (int k = 0; rho_outs && k < n; ++k) want_rho = want_rho || rho_outs[k] != nullptr;
  std::vector<std::vector<double>> host_ring(n);
  // Health check of every record: Tr sigma_0 + P_trap + P_rec is conserved
  // exactly by the equations and by RK4 (every term but the sinks is
  // traceless, and the sinks feed P_trap and P_rec), in both precisions (the
  // diagonal of sigma_0 and the scalars are FP64).  Its value at the first
  // record of the call is the reference; a drift beyond the tolerance means a
  // corrupted state.
  const double drift_tol = population_drift_tol();
  std::vector<double> pop_ref(n, std::nan(""));
  int slot = 0;
  int64_t rec_done = 0;
  auto drain = [&]() -> int {
    if (slot == 0) return HEOM_OK;
    for (int k = 0; k < n; ++k) {
      if (!rho_outs[k]) continue;
      const size_t rec_len = static_cast<size_t>(hs[k]->N) * hs[k]->N + kScalars;
      host_ring[k].resize(rec_len * slot);
      HEOM_HIP(hipMemcpyAsync(host_ring[k].data(), place.base[k] + place.inst[k].hist,
                              sizeof(double) * rec_len * slot, hipMemcpyDeviceToHost, stream),
               "hipMemcpyAsync(history)");
    }
    HEOM_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
    for (int k = 0; k < n; ++k) {
      if (!rho_outs[k]) continue;
      const int N = hs[k]->N;
      const size_t rec_len = static_cast<size_t>(N) * N + kScalars;
      for (int s = 0; s < slot; ++s) {
        const double *src = host_ring[k].data() + rec_len * s;
        for (size_t q = 0; check_numeric && q < rec_len - 1; ++q)
          if (!std::isfinite(src[q]))
            return fail(HEOM_E_NUMERIC, "non-finite reduced density matrix at record " +
                                            std::to_string(rec_done + s));
        if (check_numeric) {
          double pop = src[N * N] + src[N * N + 1];  // P_trap + P_rec
          for (int a = 0; a < N; ++a) pop += src[a];
          if (std::isnan(pop_ref[k])) pop_ref[k] = pop;
          if (std::fabs(pop - pop_ref[k]) > drift_tol * std::fmax(1.0, std::fabs(pop_ref[k])))
            return fail(HEOM_E_NUMERIC,
                        "population drift at record " + std::to_string(rec_done + s) +
                            ": Tr rho + P_trap + P_rec moved by " +
                            std::to_string(pop - pop_ref[k]) + " (instance " +
                            std::to_string(k) + ")");
        }
        unpack_hermitian(N, src, rho_outs[k] + 2 * static_cast<size_t>(N) * N * (rec_done + s));
      }
    }
    rec_done += slot;
    slot = 0;
    return HEOM_OK;
  };

  // End of a run: the last records, then the final sink populations.
  auto finish = [&]() -> int {
    if (want_rho) {
      int rc = drain();
      if (rc) return rc;
    }
    std::vector<double> sc(static_cast<size_t>(kScalars) * n);
    bool want_sinks = false;
    for (int k = 0; sinks_outs && k < n; ++k) want_sinks = want_sinks || sinks_outs[k] != nullptr;
    if (want_sinks)
      for (int k = 0; k < n; ++k)
        if (sinks_outs[k])
          HEOM_HIP(hipMemcpyAsync(sc.data() + kScalars * k, place.base[k] + place.inst[k].sc_y,
                                  sizeof(double) * kScalars, hipMemcpyDeviceToHost, stream),
                   "hipMemcpyAsync(scalars)");
    HEOM_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (want_sinks)
      for (int k = 0; k < n; ++k)
        if (sinks_outs[k])
          for (int q = 0; q < 3; ++q) sinks_outs[k][q] = sc[kScalars * k + q];
    return HEOM_OK;
  };

  if (want_rho) {
    HEOM_HIP(launch_snapshot(mixed, d_descs, n, slot, stream), "snapshot kernel");
    ++slot;
  }
  const double coef[4] = {dt_fs / 4.0, dt_fs / 3.0, dt_fs / 2.0, dt_fs};
  // Small hierarchies: every step of a chunk in one launch of the resident
  // kernel, one workgroup per instance, records written in place.
  const ResidentPlan res = resident_plan(hs, n, mixed, flags, opt.n_halo > 0 || opt.shard);
  if (res.bytes > 0) {
    HEOM_HIP(prepare_resident(res.N, res.KP, res.R, res.bytes), "resident kernel attributes");
    int64_t step = 0;
    while (step < n_steps) {
      int64_t run = std::min(n_steps - step, kResidentChunkSteps);
      if (want_rho) {
        // Records that fit the ring before the next drain.
        const int64_t room = kRingRecords - slot;
        run = std::min(run, (step / record_every + room) * record_every - step);
      }
      HEOM_HIP(launch_resident(res.N, res.KP, res.R, d_descs, n, step, run,
                               want_rho ? record_every : 0, static_cast<int>(slot), dt_fs,
                               res.bytes, stream),
               "resident kernel");
      if (want_rho) slot += static_cast<int>((step + run) / record_every - step / record_every);
      step += run;
      if (want_rho && slot == kRingRecords) {
        int rc = drain();
        if (rc) return rc;
      }
    }
    return finish();
  }
  // Launch shape and store policy of each tile group: forced by the flags,
  // the defaults (plain stores), or the autotuner's.  A store policy forced
  // by the flags overrides the tuner's.  The tuner times repeated stage
  // sequences 1, 2, 3, 2:
  // the same traffic as a step, but none of them writes the state y (only
  // the last stage does), and the run's first step rewrites the stage
  // buffers they leave behind before reading them, so the run is unchanged.
  for (Group &g : groups) {
    if (g.kind != KernelKind::kTile) continue;
    // Scaled groups: the forced shape, else tile shape 0 where every member
    // has it, else the wide kernel (no tuning; validated by check_common).
    int shape = forced_shape(flags);
    if (g.levels > 0 && shape < 0) shape = g.shape;
    bool streaming = false;
    if (shape < 0 && ((flags & HEOM_NO_AUTOTUNE) || n_steps == 0)) shape = g.shape;
    if (shape < 0 && opt.no_alloc) {
      // No timing runs (they create events): the tuned configuration if this
      // process has one for the key, else the default shape.
      int s = -1, nt = -1;
      int rc = autotune_lookup(device, mixed, g.N, g.KP, g.n_tiles, &s, &nt, nullptr, nullptr);
      if (rc) return rc;
      const bool ok = s >= 0 && s < kMaxTileShapes && g.count[g.list(s)] > 0;
      shape = ok ? s : g.shape;
      streaming = ok && nt == 1;
    }
    if (shape < 0) {
      auto time_shape = [&](int s, bool nt, double *us) -> int {
        if (nt && !has_streaming_stores(g.N, g.KP, mixed, s)) {
          *us = -1.0;  // not built
          return HEOM_OK;
        }
        int threads = 0;
        tile_shape_info(g.N, g.KP, mixed, s, nullptr, &threads, nullptr, nullptr, nullptr);
        const int l = g.list(s);
        hipEvent_t ev[2] = {nullptr, nullptr};
        int rc = HEOM_OK;
        auto pseudo_step = [&]() {
          hipError_t e = hipSuccess;
          for (int st : {0, 1, 2, 1})
            if (e == hipSuccess)
              e = launch_stage(g.kind, mixed, g.N, g.KP, s, d_descs, d_work + g.begin[l],
                               static_cast<int>(g.count[l]), threads, st, coef[st], -1, nt,
                               g.levels, stream);
          return e;
        };
        hipError_t e = hipEventCreate(&ev[0]);
        if (e == hipSuccess) e = hipEventCreate(&ev[1]);
        if (e == hipSuccess) e = pseudo_step();
        if (e == hipSuccess) e = hipEventRecord(ev[0], stream);
        for (int r = 0; r < kTuneReps && e == hipSuccess; ++r) e = pseudo_step();
        if (e == hipSuccess) e = hipEventRecord(ev[1], stream);
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (e != hipSuccess) rc = dev_fail(e, "autotune timing");
        for (hipEvent_t x : ev)
          if (x) (void)hipEventDestroy(x);
        *us = 1000.0 * static_cast<double>(ms) / (4 * kTuneReps);
        return rc;
      };
      // A shape is available when the group carries the work list it uses.
      auto available = [&](int s) { return g.count[g.list(s)] > 0; };
      int rc = autotune_choose(device, mixed, g.N, g.KP, g.n_tiles, available, time_shape, &shape,
                               &streaming);
      if (rc) return rc;
    }
    if (forced_streaming(flags) >= 0) streaming = forced_streaming(flags) == 1;
    g.shape = shape;
    g.streaming = streaming && g.levels == 0 && has_streaming_stores(g.N, g.KP, mixed, shape);
    tile_shape_info(g.N, g.KP, mixed, shape, nullptr, &g.threads, nullptr, nullptr, nullptr);
  }
  // Enqueues one RK4 step (4 stages x kernel groups) on stream `s`.  With
  // several groups, each stage forks: group 0 runs on `s`, group g on its own
  // stream, and `s` waits for all of them before the next stage.  (In a
  // graph capture this gives parallel branches.)
  ForkJoin *fj = nullptr;
  if (groups.size() > 1 && !opt.no_alloc) {
    int rc = fork_join(device, groups.size(), &fj);
    if (rc) return rc;
  }
  auto launch_group = [&](const Group &g, int st, hipStream_t s) -> hipError_t {
    const int l = g.list(g.shape);
    return launch_stage(g.kind, mixed, g.N, g.KP, g.shape, d_descs, d_work + g.begin[l],
                        static_cast<int>(g.count[l]), g.threads, st, coef[st], -1, g.streaming,
                        g.levels, s);
  };
  auto enqueue_step = [&](hipStream_t s) -> hipError_t {
    for (int st = 0; st < 4; ++st) {
      hipError_t e = launch_halo(mixed, d_descs, opt.d_halo, opt.n_halo, st, s);
      if (e != hipSuccess) return e;
      if (!fj) {
        for (const Group &g : groups)
          if (e == hipSuccess) e = launch_group(g, st, s);
        if (e != hipSuccess) return e;
        continue;
      }
      e = hipEventRecord(fj->fork, s);
      for (size_t gi = 1; gi < groups.size() && e == hipSuccess; ++gi) {
        e = hipStreamWaitEvent(fj->aux[gi], fj->fork, 0);
        if (e == hipSuccess) e = launch_group(groups[gi], st, fj->aux[gi]);
        if (e == hipSuccess) e = hipEventRecord(fj->join[gi], fj->aux[gi]);
      }
      if (e == hipSuccess) e = launch_group(groups[0], st, s);
      for (size_t gi = 1; gi < groups.size() && e == hipSuccess; ++gi)
        e = hipStreamWaitEvent(s, fj->join[gi], 0);
      if (e != hipSuccess) return e;
    }
    // The filter of scaled hierarchies, on the state the step produced.
    return launch_filter(mixed, d_descs, d_work + filter_begin, static_cast<int>(n_filter), s);
  };
  // Runs of kGraphSteps steps are replayed from one captured graph, which
  // removes the host launch cost of each stage kernel.
  StepGraph graph;
  const bool use_graph =
      (flags & HEOM_NO_GRAPH) == 0 && n_steps >= kGraphSteps && !opt.no_alloc;
  if (use_graph) {
    int rc = graph.build(device, kGraphSteps, enqueue_step);
    if (rc) return rc;
  }
  int64_t step = 0;
  while (step < n_steps) {
    // Steps until the next record (or the end).
    int64_t run = n_steps - step;
    if (want_rho) run = std::min(run, record_every - step % record_every);
    for (; use_graph && run >= kGraphSteps; run -= kGraphSteps, step += kGraphSteps)
      HEOM_HIP(hipGraphLaunch(graph.exec, stream), "hipGraphLaunch");
    for (; run > 0; --run, ++step) HEOM_HIP(enqueue_step(stream), "stage kernel");
    if (want_rho && step % record_every == 0) {
      HEOM_HIP(launch_snapshot(mixed, d_descs, n, slot, stream), "snapshot kernel");
      ++slot;
      if (slot == kRingRecords) {
        int rc = drain();
        if (rc) return rc;
      }
    }
  }
  return finish();
}

Header header_for(heom_hierarchy *const *hs, int n, int precision) {
  int64_t total = 0;
  for (int k = 0; k < n; ++k) total += hs[k]->n_ados;
  return Header{kMagic, n, precision, total};
}

// All instances in one workspace (heom_propagate, heom_propagate_batch).
int propagate_impl(heom_hierarchy *const *hs, int n, int precision, int flags,
                   const double *const *rho0s, double dt_fs, int64_t n_steps, int64_t record_every,
                   void *d_ws, size_t ws_bytes, void *hip_stream, double *const *rho_outs,
                   double *const *sinks_outs) {
  int rc = check_common(hs, n, precision, flags, dt_fs, n_steps, record_every,
                        HEOM_RESUME | HEOM_GENERIC_KERNEL | HEOM_LANE_KERNEL | HEOM_NO_GRAPH |
                            HEOM_NO_AUTOTUNE | HEOM_STREAMING_STORES | HEOM_PLAIN_STORES |
                            HEOM_NO_RESIDENT | kShapeFlagMask);
  if (rc) return rc;
  const Layout L = make_layout(hs, n, precision);
  if (!d_ws) return fail(HEOM_E_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign)
    return fail(HEOM_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(HEOM_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total) + " bytes");
  char *ws = static_cast<char *>(d_ws);
  RunPlace P;
  P.base.assign(n, ws);
  P.inst = L.inst;
  P.header = {ws + L.header};
  P.want = {header_for(hs, n, precision)};
  P.header_of.assign(n, 0);
  P.descs = ws + L.descs;
  P.work = ws + L.work;
  P.work_cap = L.work_cap;
  const std::vector<int32_t> start(n, (flags & HEOM_RESUME) ? 0 : 1);
  return run_impl(hs, n, precision, flags & ~HEOM_RESUME, start.data(), rho0s, dt_fs, n_steps,
                  record_every, P, hip_stream, rho_outs, sinks_outs);
}

// Scratch of a multi-workspace launch: descriptors and work list.
struct SlotScratch {
  size_t descs = 0, work = 0, total = 0;
  int64_t work_cap = 0;
};
SlotScratch slot_scratch(heom_hierarchy *const *hs, int n) {
  SlotScratch s;
  s.descs = 0;
  size_t off = align_up(sizeof(InstDesc) * n);
  for (int k = 0; k < n; ++k) s.work_cap += work_items_cap(hs[k]->n_ados);
  s.work = off;
  s.total = align_up(off + sizeof(WorkItem) * s.work_cap);
  return s;
}

// heom_advance_slots and its allocation-free variant (no_alloc: the scratch
// is the library's static device array, nothing is allocated or created).
int advance_slots_impl(heom_hierarchy *const *hs, int n, int precision, int flags,
                       void *const *d_workspaces, const size_t *workspace_bytes,
                       const int32_t *start, const double *const *rho0s, double dt_fs,
                       int64_t n_steps, void *d_scratch, size_t scratch_bytes, void *hip_stream,
                       double *const *rho_out, double *const *sinks_out, bool no_alloc) {
  int rc = check_common(hs, n, precision, flags, dt_fs, n_steps, 1,
                        HEOM_GENERIC_KERNEL | HEOM_LANE_KERNEL | HEOM_NO_GRAPH |
                            HEOM_NO_AUTOTUNE | HEOM_STREAMING_STORES | HEOM_PLAIN_STORES |
                            HEOM_NO_RESIDENT | kShapeFlagMask);
  if (rc) return rc;
  if (!d_workspaces || !workspace_bytes || !start)
    return fail(HEOM_E_INVALID, "workspaces, sizes and start flags are required");
  const SlotScratch sc = slot_scratch(hs, n);
  if (no_alloc && sc.total > scratch_bytes)
    return fail(HEOM_E_WORKSPACE, "these slots need " + std::to_string(sc.total) +
                                      " bytes of launch scratch; the static scratch holds " +
                                      std::to_string(scratch_bytes));
  if (!d_scratch || reinterpret_cast<uintptr_t>(d_scratch) % kAlign || scratch_bytes < sc.total)
    return fail(HEOM_E_WORKSPACE, "scratch missing, misaligned or too small: need " +
                                      std::to_string(sc.total) + " bytes");
  RunPlace P;
  for (int k = 0; k < n; ++k) {
    heom_hierarchy *h = hs[k];
    const Layout L1 = make_layout(&h, 1, precision);
    char *ws = static_cast<char *>(d_workspaces[k]);
    if (!ws || reinterpret_cast<uintptr_t>(ws) % kAlign || workspace_bytes[k] < L1.total)
      return fail(HEOM_E_WORKSPACE, "workspace " + std::to_string(k) +
                                        " missing, misaligned or too small");
    for (int j = 0; j < k; ++j)
      if (d_workspaces[j] == d_workspaces[k])
        return fail(HEOM_E_INVALID, "two slots share one workspace");
    P.base.push_back(ws);
    P.inst.push_back(L1.inst[0]);
    P.header.push_back(ws + L1.header);
    P.want.push_back(header_for(&h, 1, precision));
    P.header_of.push_back(k);
  }
  char *s = static_cast<char *>(d_scratch);
  P.descs = s + sc.descs;
  P.work = s + sc.work;
  P.work_cap = sc.work_cap;
  // Records of every slot (the state at the start and after the last step)
  // and its sinks, checked per slot below: a slot with a non-finite result
  // fails alone, and every slot's output is written either way.
  const int64_t rec_every = n_steps > 0 ? n_steps : 1;
  std::vector<std::vector<double>> rec(n);
  std::vector<double> sk(3 * static_cast<size_t>(n), 0.0);
  std::vector<double *> ro(n, nullptr), so(n, nullptr);
  for (int k = 0; k < n; ++k) {
    rec[k].assign(4 * static_cast<size_t>(hs[k]->N) * hs[k]->N, 0.0);
    ro[k] = rec[k].data();
    so[k] = sk.data() + 3 * k;
  }
  RunOptions opt;
  opt.check_numeric = false;
  opt.no_alloc = no_alloc;
  rc = run_impl(hs, n, precision, flags, start, rho0s, dt_fs, n_steps, rec_every, P, hip_stream,
                ro.data(), so.data(), opt);
  if (rc) return rc;
  std::string bad;
  for (int k = 0; k < n; ++k) {
    const size_t len = 2 * static_cast<size_t>(hs[k]->N) * hs[k]->N;
    const double *fin = rec[k].data() + (n_steps > 0 ? len : 0);
    bool ok = std::isfinite(so[k][0]) && std::isfinite(so[k][1]) && std::isfinite(so[k][2]);
    for (size_t q = 0; ok && q < len; ++q) ok = std::isfinite(fin[q]);
    if (!ok) bad += (bad.empty() ? "" : ", ") + std::to_string(k);
    if (rho_out && rho_out[k]) std::memcpy(rho_out[k], fin, sizeof(double) * len);
    if (sinks_out && sinks_out[k]) std::memcpy(sinks_out[k], so[k], sizeof(double) * 3);
  }
  if (!bad.empty())
    return fail(HEOM_E_NUMERIC, "non-finite result in slot(s) " + bad +
                                    " (every slot was advanced; the others are valid)");
  return HEOM_OK;
}

}  // namespace

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int status, const std::string &msg) {
  g_last_error = msg;
  return status;
}

}  // namespace heom

using namespace heom;

extern "C" {

const char *heom_status_string(int status) {
  switch (status) {
    case HEOM_OK: return "ok";
    case HEOM_E_INVALID: return "invalid argument";
    case HEOM_E_NOMEM: return "out of memory";
    case HEOM_E_DEVICE: return "device error";
    case HEOM_E_NUMERIC: return "numerical failure";
    case HEOM_E_WORKSPACE: return "workspace error";
    case HEOM_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char *heom_last_error(void) { return g_last_error.c_str(); }

int heom_build_hierarchy(const heom_system *sys, int32_t depth, heom_hierarchy **out) {
  if (!out) return fail(HEOM_E_INVALID, "out is NULL");
  *out = nullptr;
  heom_hierarchy *h = new (std::nothrow) heom_hierarchy();
  if (!h) return fail(HEOM_E_NOMEM, "host allocation failed");
  try {
    int rc = build_params(sys, h);
    if (rc == HEOM_OK) {
      h->depth = depth;
      rc = build_tables(h);
    }
    if (rc != HEOM_OK) {
      delete h;
      return rc;
    }
  } catch (const std::bad_alloc &) {
    delete h;
    return fail(HEOM_E_NOMEM, "host allocation failed");
  } catch (...) {
    delete h;
    return fail(HEOM_E_INVALID, "unexpected failure while building the hierarchy");
  }
  g_last_error.clear();
  *out = h;
  return HEOM_OK;
}

int heom_build_hierarchy_scaled(const heom_system *sys, int32_t depth, double filter_tol,
                                heom_hierarchy **out) {
  if (!out) return fail(HEOM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!(filter_tol >= 0.0) || !std::isfinite(filter_tol))
    return fail(HEOM_E_INVALID, "filter_tol must be finite and >= 0");
  heom_hierarchy *h = nullptr;
  int rc = heom_build_hierarchy(sys, depth, &h);
  if (rc) return rc;
  // Coupling weights by mode and occupation: the ADO n is held divided by
  // w_n = sqrt(prod_m n_m! |c_m|^n_m), so the coupling to n + e_m carries
  // w_{n+e_m} / w_n = sqrt((n_m + 1)|c_m|) and the one to n - e_m carries
  // n_m w_{n-e_m} / w_n = sqrt(n_m / |c_m|).
  const int M = h->M, L = depth + 1;
  for (int m = 0; m < M; ++m)
    if (!(std::hypot(h->c_re[m], h->c_im[m]) > 0.0)) {
      heom_destroy(h);
      return fail(HEOM_E_INVALID, "a scaled hierarchy needs nonzero bath amplitudes (lambda > 0)");
    }
  try {
    const size_t base = h->params.size();
    h->params.resize(base + 2 * static_cast<size_t>(M) * L);
    for (int m = 0; m < M; ++m) {
      const double absc = std::hypot(h->c_re[m], h->c_im[m]);
      for (int v = 0; v < L; ++v) {
        h->params[base + m * L + v] = std::sqrt((v + 1.0) * absc);
        h->params[base + M * L + m * L + v] = std::sqrt(v / absc);
      }
    }
  } catch (...) {
    heom_destroy(h);
    return fail(HEOM_E_NOMEM, "host allocation failed");
  }
  h->scaled = true;
  h->filter_tol = filter_tol;
  *out = h;
  return HEOM_OK;
}

int heom_hierarchy_info(const heom_hierarchy *h, int64_t *n_ados, int32_t *n_modes,
                        size_t *workspace_bytes_fp64, size_t *workspace_bytes_fp32) {
  if (!h) return fail(HEOM_E_INVALID, "hierarchy is NULL");
  heom_hierarchy *hh = const_cast<heom_hierarchy *>(h);
  if (n_ados) *n_ados = h->n_ados;
  if (n_modes) *n_modes = h->M;
  if (workspace_bytes_fp64) *workspace_bytes_fp64 = make_layout(&hh, 1, HEOM_FP64).total;
  if (workspace_bytes_fp32) *workspace_bytes_fp32 = make_layout(&hh, 1, HEOM_FP32_MIXED).total;
  return HEOM_OK;
}

int heom_hierarchy_tables(const heom_hierarchy *h, int32_t *multi, int32_t *up, int32_t *down) {
  if (!h) return fail(HEOM_E_INVALID, "hierarchy is NULL");
  const int M = h->M;
  if (multi) std::memcpy(multi, h->multi.data(), sizeof(int32_t) * h->multi.size());
  for (int64_t i = 0; i < h->n_ados; ++i)
    for (int m = 0; m < M; ++m) {
      if (up) up[i * M + m] = h->up[static_cast<size_t>(m) * h->stride + i];
      if (down) down[i * M + m] = h->down[static_cast<size_t>(m) * h->stride + i];
    }
  return HEOM_OK;
}

int heom_hierarchy_modes(const heom_hierarchy *h, int32_t *site, double *c_re, double *c_im,
                         double *nu, double *delta) {
  if (!h) return fail(HEOM_E_INVALID, "hierarchy is NULL");
  for (int m = 0; m < h->M; ++m) {
    if (site) site[m] = h->site[m];
    if (c_re) c_re[m] = h->c_re[m];
    if (c_im) c_im[m] = h->c_im[m];
    if (nu) nu[m] = h->nu[m];
  }
  if (delta)
    for (int a = 0; a < h->N; ++a) delta[a] = h->delta[a];
  return HEOM_OK;
}

int heom_max_stable_dt(const heom_hierarchy *h, double *dt_fs) {
  if (!h || !dt_fs) return fail(HEOM_E_INVALID, "hierarchy or output is NULL");
  double nu_max = 0.0;
  for (int m = 0; m < h->M; ++m) nu_max = std::max(nu_max, h->nu[m]);
  const double rate = h->depth * nu_max;  // the deepest ADO on the fastest mode
  *dt_fs = rate > 0.0 ? 2.5 / rate : std::numeric_limits<double>::infinity();
  return HEOM_OK;
}

int heom_batch_workspace_bytes(heom_hierarchy *const *hs, int32_t n, int precision, size_t *bytes) {
  if (!hs || n < 1 || !bytes) return fail(HEOM_E_INVALID, "bad arguments");
  for (int k = 0; k < n; ++k)
    if (!hs[k]) return fail(HEOM_E_INVALID, "NULL hierarchy handle");
  if (precision != HEOM_FP64 && precision != HEOM_FP32_MIXED)
    return fail(HEOM_E_UNSUPPORTED, "precision must be HEOM_FP64 or HEOM_FP32_MIXED");
  *bytes = make_layout(hs, n, precision).total;
  return HEOM_OK;
}

int heom_propagate(heom_hierarchy *h, int precision, int flags, const double *rho0, double dt_fs,
                   int64_t n_steps, int64_t record_every, void *d_workspace,
                   size_t workspace_bytes, void *hip_stream, double *rho_out, double *sinks_out) {
  try {
    return propagate_impl(&h, 1, precision, flags, &rho0, dt_fs, n_steps, record_every,
                          d_workspace, workspace_bytes, hip_stream, &rho_out, &sinks_out);
  } catch (...) {
    return fail(HEOM_E_NOMEM, "host allocation failed");
  }
}

int heom_propagate_batch(heom_hierarchy *const *hs, int32_t n, int precision, int flags,
                         const double *const *rho0s, double dt_fs, int64_t n_steps,
                         int64_t record_every, void *d_workspace, size_t workspace_bytes,
                         void *hip_stream, double *const *rho_outs, double *const *sinks_outs) {
  try {
    std::vector<double *> ro(n > 0 ? n : 0, nullptr), so(n > 0 ? n : 0, nullptr);
    for (int k = 0; k < n; ++k) {
      if (rho_outs) ro[k] = rho_outs[k];
      if (sinks_outs) so[k] = sinks_outs[k];
    }
    return propagate_impl(hs, n, precision, flags, rho0s, dt_fs, n_steps, record_every,
                          d_workspace, workspace_bytes, hip_stream, ro.data(), so.data());
  } catch (...) {
    return fail(HEOM_E_NOMEM, "host allocation failed");
  }
}

int heom_slots_scratch_bytes(heom_hierarchy *const *hs, int32_t n, size_t *bytes) {
  if (!hs || n < 1 || !bytes) return fail(HEOM_E_INVALID, "bad arguments");
  for (int k = 0; k < n; ++k)
    if (!hs[k]) return fail(HEOM_E_INVALID, "NULL hierarchy handle");
  *bytes = slot_scratch(hs, n).total;
  return HEOM_OK;
}

int heom_advance_slots(heom_hierarchy *const *hs, int32_t n, int precision, int flags,
                       void *const *d_workspaces, const size_t *workspace_bytes,
                       const int32_t *start, const double *const *rho0s, double dt_fs,
                       int64_t n_steps, void *d_scratch, size_t scratch_bytes, void *hip_stream,
                       double *const *rho_out, double *const *sinks_out) {
  try {
    return advance_slots_impl(hs, n, precision, flags, d_workspaces, workspace_bytes, start,
                              rho0s, dt_fs, n_steps, d_scratch, scratch_bytes, hip_stream, rho_out,
                              sinks_out, false);
  } catch (...) {
    return fail(HEOM_E_NOMEM, "host allocation failed");
  }
}

int heom_advance_slots_noalloc(heom_hierarchy *const *hs, int32_t n, int precision, int flags,
                               void *const *d_workspaces, const size_t *workspace_bytes,
                               const int32_t *start, const double *const *rho0s, double dt_fs,
                               int64_t n_steps, void *hip_stream, double *const *rho_out,
                               double *const *sinks_out) {
  try {
    int device = 0;
    HEOM_HIP(hipGetDevice(&device), "hipGetDevice");
    void *scratch = nullptr;
    HEOM_HIP(static_scratch(device, &scratch), "hipGetSymbolAddress(scratch)");
    return advance_slots_impl(hs, n, precision, flags, d_workspaces, workspace_bytes, start,
                              rho0s, dt_fs, n_steps, scratch, kStaticScratchBytes, hip_stream,
                              rho_out, sinks_out, true);
  } catch (...) {
    return fail(HEOM_E_NOMEM, "host allocation failed");
  }
}

int heom_efficiency(heom_hierarchy *h, int precision, const double *rho0, double dt_fs,
                    double t_end_fs, double pop_tol, void *d_workspace, size_t workspace_bytes,
                    void *hip_stream, heom_eff_result *out) {
  if (!h || !out) return fail(HEOM_E_INVALID, "hierarchy or out is NULL");
  if (!(dt_fs > 0.0)) return fail(HEOM_E_INVALID, "dt_fs must be > 0");
  if (!std::isfinite(t_end_fs)) return fail(HEOM_E_INVALID, "t_end_fs must be finite");
  if (t_end_fs <= 0.0 && !(pop_tol > 0.0 && pop_tol < 1.0))
    return fail(HEOM_E_INVALID, "pop_tol must be in (0, 1) when t_end_fs <= 0");
  const int N = h->N;
  std::vector<double> rho(2 * static_cast<size_t>(N) * N * 2);
  double sinks[3] = {0, 0, 0};
  int64_t steps_done = 0;
  try {
    if (t_end_fs > 0.0) {
      const int64_t steps = static_cast<int64_t>(std::llround(t_end_fs / dt_fs));
      int rc = heom_propagate(h, precision, 0, rho0, dt_fs, steps, steps > 0 ? steps : 1,
                              d_workspace, workspace_bytes, hip_stream, rho.data(), sinks);
      if (rc) return rc;
      steps_done = steps;
    } else {
      const int64_t chunk = 500;
      const int64_t max_steps = 100000000;
      int flags = 0;
      for (;;) {
        int rc = heom_propagate(h, precision, flags, rho0, dt_fs, chunk, chunk, d_workspace,
                                workspace_bytes, hip_stream, rho.data(), sinks);
        if (rc) return rc;
        flags = HEOM_RESUME;
        steps_done += chunk;
        double tr = 0.0;
        const double *last = rho.data() + 2 * static_cast<size_t>(N) * N;
        for (int a = 0; a < N; ++a) tr += last[2 * (a * N + a)];
        if (tr < pop_tol) break;
        if (steps_done >= max_steps)
          return fail(HEOM_E_NUMERIC, "population criterion not met within 1e8 steps");
      }
    }
  } catch (...) {
    return fail(HEOM_E_NOMEM, "host allocation failed");
  }
  const double *last = rho.data() + 2 * static_cast<size_t>(N) * N;
  double tr = 0.0;
  for (int a = 0; a < N; ++a) tr += last[2 * (a * N + a)];
  const double t = steps_done * dt_fs;
  out->eta = sinks[0];
  out->p_recomb = sinks[1];
  out->p_remaining = tr;
  out->t_end_fs = t;
  out->mean_trap_time_fs = t * sinks[0] - sinks[2];
  return HEOM_OK;
}

int heom_read_state(const heom_hierarchy *h, int precision, const void *d_workspace,
                    size_t workspace_bytes, void *hip_stream, double *state_out) {
  if (!h || !state_out) return fail(HEOM_E_INVALID, "hierarchy or state_out is NULL");
  if (precision != HEOM_FP64 && precision != HEOM_FP32_MIXED)
    return fail(HEOM_E_UNSUPPORTED, "precision must be HEOM_FP64 or HEOM_FP32_MIXED");
  heom_hierarchy *hh = const_cast<heom_hierarchy *>(h);
  const Layout L = make_layout(&hh, 1, precision);
  if (!d_workspace || workspace_bytes < L.total)
    return fail(HEOM_E_WORKSPACE, "workspace missing or too small");
  const char *ws = static_cast<const char *>(d_workspace);
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  const int N = h->N;
  const size_t N2 = static_cast<size_t>(N) * N;
  const size_t planes = N2 * static_cast<size_t>(h->stride);
  const bool mixed = precision == HEOM_FP32_MIXED;
  std::vector<double> p64;
  std::vector<float> p32;
  std::vector<double> y0(N2), sc(kScalars);
  Header cur;
  try {
    if (mixed)
      p32.resize(planes);
    else
      p64.resize(planes);
  } catch (...) {
    return fail(HEOM_E_NOMEM, "host allocation failed");
  }
  HEOM_HIP(hipMemcpyAsync(&cur, ws + L.header, sizeof(Header), hipMemcpyDeviceToHost, stream),
           "hipMemcpyAsync(header)");
  HEOM_HIP(hipMemcpyAsync(mixed ? static_cast<void *>(p32.data()) : static_cast<void *>(p64.data()),
                          ws + L.inst[0].y, planes * (mixed ? 4 : 8), hipMemcpyDeviceToHost, stream),
           "hipMemcpyAsync(state)");
  HEOM_HIP(hipMemcpyAsync(y0.data(), ws + L.inst[0].y0, sizeof(double) * N2, hipMemcpyDeviceToHost,
                          stream),
           "hipMemcpyAsync(sigma0)");
  HEOM_HIP(hipMemcpyAsync(sc.data(), ws + L.inst[0].sc_y, sizeof(double) * kScalars,
                          hipMemcpyDeviceToHost, stream),
           "hipMemcpyAsync(scalars)");
  HEOM_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
  if (cur.magic != kMagic || cur.n_inst != 1 || cur.precision != precision ||
      cur.total_ados != h->n_ados)
    return fail(HEOM_E_WORKSPACE, "workspace does not hold a run of this hierarchy");
  std::vector<double> packed(N2);
  for (int64_t i = 0; i < h->n_ados; ++i) {
    for (size_t e = 0; e < N2; ++e) {
      const size_t idx = static_cast<size_t>(elem_index(N, static_cast<int>(e), h->stride, i));
      packed[e] = (mixed && i == 0) ? y0[e] : (mixed ? p32[idx] : p64[idx]);
    }
    unpack_hermitian(N, packed.data(), state_out + 2 * N2 * i);
  }
  double *tail = state_out + 2 * N2 * h->n_ados;
  tail[0] = sc[0];
  tail[1] = sc[1];
  tail[2] = sc[2];
  return HEOM_OK;
}

// --- a hierarchy split over ranks (its one-GPU part) -------------------------

int heom_shard_build(const heom_hierarchy *h, int32_t n_ranks, heom_shard **out) {
  if (!h || !out) return fail(HEOM_E_INVALID, "hierarchy or out is NULL");
  *out = nullptr;
  if (h->scaled) return fail(HEOM_E_UNSUPPORTED, "scaled hierarchies are not split over ranks");
  heom_shard *s = new (std::nothrow) heom_shard();
  if (!s) return fail(HEOM_E_NOMEM, "host allocation failed");
  int rc = HEOM_OK;
  try {
    rc = build_shard(h, n_ranks, s);
  } catch (...) {
    rc = fail(HEOM_E_NOMEM, "host allocation failed");
  }
  if (rc != HEOM_OK) {
    heom_shard_destroy(s);
    return rc;
  }
  *out = s;
  return HEOM_OK;
}

int heom_shard_info(const heom_shard *s, int32_t rank, heom_shard_rank_info *out) {
  if (!s || !out) return fail(HEOM_E_INVALID, "shard or out is NULL");
  if (rank < 0 || rank >= s->n_ranks) return fail(HEOM_E_INVALID, "rank out of range");
  const heom_shard::Stats &st = s->stats[rank];
  out->first_ado = s->first[rank];
  out->n_local = s->first[rank + 1] - s->first[rank];
  out->n_halo = st.n_halo;
  out->cut_links = st.cut_links;
  out->halo_reals = st.n_halo * static_cast<int64_t>(s->N) * s->N;
  out->halo_reals_min = st.halo_reals_min;
  return HEOM_OK;
}

namespace {

// Workspace of a split hierarchy: every rank laid out as an instance of a
// batch, then the halo list.
struct ShardLayout {
  Layout L;
  size_t halo = 0, total = 0;
};
ShardLayout shard_layout(const heom_shard *s, int precision) {
  ShardLayout S;
  S.L = make_layout(s->rank.data(), s->n_ranks, precision);
  S.halo = S.L.total;
  S.total = align_up(S.halo + sizeof(HaloEntry) * s->halo.size());
  return S;
}

}  // namespace

int heom_shard_workspace_bytes(const heom_shard *s, int precision, size_t *bytes) {
  if (!s || !bytes) return fail(HEOM_E_INVALID, "shard or bytes is NULL");
  if (precision != HEOM_FP64) return fail(HEOM_E_UNSUPPORTED, "split hierarchies run in FP64");
  *bytes = shard_layout(s, precision).total;
  return HEOM_OK;
}

int heom_propagate_sharded(heom_shard *s, int precision, int flags, const double *rho0,
                           double dt_fs, int64_t n_steps, int64_t record_every, void *d_workspace,
                           size_t workspace_bytes, void *hip_stream, double *rho_out,
                           double *sinks_out) {
  try {
    if (!s) return fail(HEOM_E_INVALID, "shard is NULL");
    if (precision != HEOM_FP64) return fail(HEOM_E_UNSUPPORTED, "split hierarchies run in FP64");
    const int n = s->n_ranks;
    heom_hierarchy *const *hs = s->rank.data();
    int rc = check_common(hs, n, precision, flags, dt_fs, n_steps, record_every,
                          HEOM_RESUME | HEOM_GENERIC_KERNEL | HEOM_LANE_KERNEL | HEOM_NO_GRAPH |
                              HEOM_NO_AUTOTUNE | HEOM_STREAMING_STORES | HEOM_PLAIN_STORES |
                              HEOM_NO_RESIDENT | kShapeFlagMask);
    if (rc) return rc;
    const ShardLayout S = shard_layout(s, precision);
    if (!d_workspace) return fail(HEOM_E_WORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
      return fail(HEOM_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (workspace_bytes < S.total)
      return fail(HEOM_E_WORKSPACE,
                  "workspace too small: need " + std::to_string(S.total) + " bytes");
    char *ws = static_cast<char *>(d_workspace);
    RunPlace P;
    P.base.assign(n, ws);
    P.inst = S.L.inst;
    P.header = {ws + S.L.header};
    P.want = {header_for(hs, n, precision)};
    P.header_of.assign(n, 0);
    P.descs = ws + S.L.descs;
    P.work = ws + S.L.work;
    P.work_cap = S.L.work_cap;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    if (!s->halo.empty())
      HEOM_HIP(hipMemcpyAsync(ws + S.halo, s->halo.data(), sizeof(HaloEntry) * s->halo.size(),
                              hipMemcpyHostToDevice, stream),
               "hipMemcpyAsync(halo list)");
    const std::vector<int32_t> start(n, (flags & HEOM_RESUME) ? 0 : 1);
    const std::vector<const double *> rho0s(n, rho0);
    std::vector<double *> ro(n, nullptr), so(n, nullptr);
    ro[0] = rho_out;
    so[0] = sinks_out;
    RunOptions opt;
    opt.shard = true;
    opt.d_halo = reinterpret_cast<const HaloEntry *>(ws + S.halo);
    opt.n_halo = static_cast<int>(s->halo.size());
    return run_impl(hs, n, precision, flags & ~HEOM_RESUME, start.data(), rho0s.data(), dt_fs,
                    n_steps, record_every, P, hip_stream, ro.data(), so.data(), opt);
  } catch (...) {
    return fail(HEOM_E_NOMEM, "host allocation failed");
  }
}

int heom_read_state_sharded(const heom_shard *s, int precision, const void *d_workspace,
                            size_t workspace_bytes, void *hip_stream, double *state_out) {
  if (!s || !state_out) return fail(HEOM_E_INVALID, "shard or state_out is NULL");
  if (precision != HEOM_FP64) return fail(HEOM_E_UNSUPPORTED, "split hierarchies run in FP64");
  const ShardLayout S = shard_layout(s, precision);
  if (!d_workspace || workspace_bytes < S.total)
    return fail(HEOM_E_WORKSPACE, "workspace missing or too small");
  const char *ws = static_cast<const char *>(d_workspace);
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  const int N = s->N;
  const size_t N2 = static_cast<size_t>(N) * N;
  Header cur;
  std::vector<double> sc(kScalars);
  std::vector<std::vector<double>> planes(s->n_ranks);
  try {
    for (int r = 0; r < s->n_ranks; ++r) planes[r].resize(N2 * s->rank[r]->stride);
  } catch (...) {
    return fail(HEOM_E_NOMEM, "host allocation failed");
  }
  HEOM_HIP(hipMemcpyAsync(&cur, ws + S.L.header, sizeof(Header), hipMemcpyDeviceToHost, stream),
           "hipMemcpyAsync(header)");
  for (int r = 0; r < s->n_ranks; ++r)
    HEOM_HIP(hipMemcpyAsync(planes[r].data(), ws + S.L.inst[r].y,
                            sizeof(double) * planes[r].size(), hipMemcpyDeviceToHost, stream),
             "hipMemcpyAsync(state)");
  HEOM_HIP(hipMemcpyAsync(sc.data(), ws + S.L.inst[0].sc_y, sizeof(double) * kScalars,
                          hipMemcpyDeviceToHost, stream),
           "hipMemcpyAsync(scalars)");
  HEOM_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
  heom_hierarchy *const *hs = s->rank.data();
  const Header want = header_for(hs, s->n_ranks, precision);
  if (std::memcmp(&cur, &want, sizeof(Header)) != 0)
    return fail(HEOM_E_WORKSPACE, "workspace does not hold a run of this split hierarchy");
  std::vector<double> packed(N2);
  for (int r = 0; r < s->n_ranks; ++r) {
    const heom_hierarchy *g = s->rank[r];
    for (int64_t li = 0; li < g->n_ados; ++li) {
      for (size_t e = 0; e < N2; ++e)
        packed[e] = planes[r][elem_index(N, static_cast<int>(e), g->stride, li)];
      unpack_hermitian(N, packed.data(), state_out + 2 * N2 * (s->first[r] + li));
    }
  }
  double *tail = state_out + 2 * N2 * s->n_ados;
  tail[0] = sc[0];
  tail[1] = sc[1];
  tail[2] = sc[2];
  return HEOM_OK;
}

void heom_shard_destroy(heom_shard *s) {
  if (!s) return;
  for (heom_hierarchy *h : s->rank) heom_destroy(h);
  delete s;
}

int heom_tile_shape_count(void) { return kMaxTileShapes; }

int heom_tile_shape_info(int32_t n_sites, int32_t modes_per_site, int precision, int32_t shape,
                         int32_t *ados_per_workgroup, int32_t *threads, int32_t *elems_per_wave,
                         int32_t *chunk, int32_t *min_waves_per_simd) {
  if (precision != HEOM_FP64 && precision != HEOM_FP32_MIXED)
    return fail(HEOM_E_UNSUPPORTED, "precision must be HEOM_FP64 or HEOM_FP32_MIXED");
  if (shape < 0 || shape >= kMaxTileShapes) return fail(HEOM_E_INVALID, "shape out of range");
  int a = 0, t = 0, e = 0, c = 0, w = 0;
  if (!tile_shape_info(n_sites, modes_per_site, precision == HEOM_FP32_MIXED, shape, &a, &t, &e,
                       &c, &w))
    return fail(HEOM_E_UNSUPPORTED, "no kernel is built for this N, K+1 and launch shape");
  if (ados_per_workgroup) *ados_per_workgroup = a;
  if (threads) *threads = t;
  if (elems_per_wave) *elems_per_wave = e;
  if (chunk) *chunk = c;
  if (min_waves_per_simd) *min_waves_per_simd = w;
  return HEOM_OK;
}

int heom_autotune_lookup(int32_t n_sites, int32_t modes_per_site, int precision, int64_t n_tiles,
                         int32_t *shape, double *us_per_shape, int32_t *streaming,
                         double *us_streaming) {
  if (!shape) return fail(HEOM_E_INVALID, "shape is NULL");
  if (precision != HEOM_FP64 && precision != HEOM_FP32_MIXED)
    return fail(HEOM_E_UNSUPPORTED, "precision must be HEOM_FP64 or HEOM_FP32_MIXED");
  if (n_tiles < 1) return fail(HEOM_E_INVALID, "n_tiles must be >= 1");
  int device = 0;
  HEOM_HIP(hipGetDevice(&device), "hipGetDevice");
  int s = -1, nt = -1;
  int rc = autotune_lookup(device, precision == HEOM_FP32_MIXED, n_sites, modes_per_site, n_tiles,
                           &s, &nt, us_per_shape, us_streaming);
  if (rc) return rc;
  *shape = s;
  if (streaming) *streaming = nt;
  return HEOM_OK;
}

void heom_autotune_clear(void) { autotune_clear(); }

void heom_destroy(heom_hierarchy *h) {
  if (!h) return;
  for (auto &t : h->dev) {
    (void)hipFree(t.up);
    (void)hipFree(t.down);
    (void)hipFree(t.occ);
    if (t.up16) (void)hipFree(t.up16);
    if (t.down16) (void)hipFree(t.down16);
  }
  delete h;
}

}  // extern "C"
