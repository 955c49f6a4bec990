// autotune.cpp -- launch-shape autotuner of the tile stage kernel.
//
// The tile kernel is compiled in several launch shapes (waves per workgroup,
// packed elements per wave, elements whose gathers are in flight together,
// register budget; tile_shape in stage_kernels.h).  Which one is fastest depends on the size of
// the launch: a launch of a few hundred tiles is latency-bound and prefers
// long load batches, a launch of thousands of tiles is bandwidth-bound and
// prefers shapes that keep more workgroups resident.  The tuner keys its
// choice on (GPU architecture, precision, N, K+1, floor(log2(tiles))), times
// every candidate once per key on the caller's own launch (see run_impl),
// then the fastest one again with non-temporal (streaming) output stores, and
// remembers the faster configuration for the life of the process.  If
// HEOM_AUTOTUNE_CACHE names a file, its entries are read on first use and new
// entries are appended to it, one JSON object per line.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "heom_internal.h"

namespace heom {

namespace {

struct Entry {
  int shape = -1;
  int streaming = 0;          // non-temporal output stores
  double us[kMaxTileShapes];  // per shape, plain stores
  double us_streaming = -1.0;  // the chosen shape with streaming stores
};

// (arch, mixed, N, K+1, floor(log2(tiles)))
typedef std::tuple<std::string, int, int, int, int> Key;

std::mutex g_mu;
std::map<Key, Entry> g_cache;
bool g_file_read = false;

const char *cache_path() {
  const char *p = std::getenv("HEOM_AUTOTUNE_CACHE");
  return (p && p[0]) ? p : nullptr;
}

int log2_floor(int64_t x) {
  int r = 0;
  while (x > 1) {
    x >>= 1;
    ++r;
  }
  return r;
}

std::string arch_of(int device) {
  static std::mutex mu;
  static std::map<int, std::string> names;
  std::lock_guard<std::mutex> lock(mu);
  auto it = names.find(device);
  if (it != names.end()) return it->second;
  hipDeviceProp_t prop;
  std::string name = "unknown";
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    name = prop.gcnArchName;
    const size_t colon = name.find(':');  // drop target features
    if (colon != std::string::npos) name.resize(colon);
  }
  names[device] = name;
  return name;
}

// One line of the cache file (one timing per shape slot, -1 where untimed):
// {"arch": "gfx950", "precision": 0, "N": 7, "KP": 1, "tiles_log2": 8, "shape": 1,
//  "streaming": 0, "us": [10.6, 9.8, 12.0, -1.0, 11.1, 30.2], "us_streaming": 10.1}
bool parse_line(const char *line, Key *key, Entry *e) {
  char arch[64] = {0};
  int prec, N, KP, tl, shape, streaming, used = 0;
  const int got = std::sscanf(line,
                              " {\"arch\": \"%63[^\"]\", \"precision\": %d, \"N\": %d, \"KP\": %d, "
                              "\"tiles_log2\": %d, \"shape\": %d, \"streaming\": %d, \"us\": [%n",
                              arch, &prec, &N, &KP, &tl, &shape, &streaming, &used);
  if (got != 7 || used == 0 || shape < 0 || shape >= kMaxTileShapes) return false;
  if (streaming != 0 && streaming != 1) return false;
  const char *p = line + used;
  for (int s = 0; s < kMaxTileShapes; ++s) {
    char *end = nullptr;
    e->us[s] = std::strtod(p, &end);
    if (end == p) return false;
    p = end;
    while (*p == ',' || *p == ' ') ++p;
  }
  if (*p != ']') return false;
  int tail = 0;
  if (std::sscanf(p, "], \"us_streaming\": %lf}%n", &e->us_streaming, &tail) != 1 || tail == 0)
    return false;
  e->shape = shape;
  e->streaming = streaming;
  *key = Key(arch, prec, N, KP, tl);
  return true;
}

void read_file_locked() {
  if (g_file_read) return;
  g_file_read = true;
  const char *path = cache_path();
  if (!path) return;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  char line[1024];
  while (std::fgets(line, sizeof(line), f)) {
    Key k;
    Entry e;
    if (parse_line(line, &k, &e)) g_cache[k] = e;  // other lines are ignored
  }
  std::fclose(f);
}

void append_file_locked(const Key &k, const Entry &e) {
  const char *path = cache_path();
  if (!path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;  // the in-memory entry still holds
  std::fprintf(f,
               "{\"arch\": \"%s\", \"precision\": %d, \"N\": %d, \"KP\": %d, \"tiles_log2\": %d, "
               "\"shape\": %d, \"streaming\": %d, \"us\": [",
               std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k), std::get<3>(k),
               std::get<4>(k), e.shape, e.streaming);
  for (int s = 0; s < kMaxTileShapes; ++s)
    std::fprintf(f, s ? ", %.3f" : "%.3f", e.us[s]);
  std::fprintf(f, "], \"us_streaming\": %.3f}\n", e.us_streaming);
  std::fclose(f);
}

}  // namespace

int autotune_choose(int device, bool mixed, int N, int KP, int64_t n_tiles,
                    const std::function<bool(int)> &available,
                    const std::function<int(int, bool, double *)> &time_shape, int *shape_out,
                    bool *streaming_out) {
  const Key key(arch_of(device), mixed ? 1 : 0, N, KP, log2_floor(n_tiles));
  {
    std::lock_guard<std::mutex> lock(g_mu);
    read_file_locked();
    auto it = g_cache.find(key);
    if (it != g_cache.end() && available(it->second.shape)) {
      *shape_out = it->second.shape;
      *streaming_out = it->second.streaming != 0;
      return HEOM_OK;
    }
  }
  // Time the distinct candidates (shapes with the same launch configuration
  // as an earlier one are the same kernel in effect and are skipped).
  Entry e;
  for (double &u : e.us) u = -1.0;
  int seen[kMaxTileShapes][4], n_seen = 0;
  int cand[kMaxTileShapes], n_cand = 0;
  for (int s = 0; s < kMaxTileShapes; ++s) {
    int ados = 0, threads = 0, epw = 0, chunk = 0, waves = 0;
    if (!available(s) || !tile_shape_info(N, KP, mixed, s, &ados, &threads, &epw, &chunk, &waves))
      continue;
    bool dup = false;
    for (int q = 0; q < n_seen; ++q)
      dup = dup || (seen[q][0] == ados && seen[q][1] == threads && seen[q][2] == chunk &&
                    seen[q][3] == waves);
    if (dup) continue;
    seen[n_seen][0] = ados;
    seen[n_seen][1] = threads;
    seen[n_seen][2] = chunk;
    seen[n_seen][3] = waves;
    ++n_seen;
    cand[n_cand++] = s;
  }
  if (n_cand == 0) return fail(HEOM_E_UNSUPPORTED, "no tile launch shape for this hierarchy");
  double best = 0.0;
  for (int q = 0; q < n_cand; ++q) {
    const int s = cand[q];
    double us = 0.0;
    int rc = time_shape(s, false, &us);
    if (rc) return rc;
    e.us[s] = us;
    if (e.shape < 0 || us < best) {
      e.shape = s;
      best = us;
    }
  }
  if (e.shape < 0) return fail(HEOM_E_UNSUPPORTED, "no tile launch shape for this hierarchy");
  int rc = time_shape(e.shape, true, &e.us_streaming);  // -1: no such instance
  if (rc) return rc;
  e.streaming = e.us_streaming > 0.0 && e.us_streaming < best ? 1 : 0;
  std::lock_guard<std::mutex> lock(g_mu);
  auto ins = g_cache.emplace(key, e);
  if (ins.second) append_file_locked(key, e);
  const Entry &use = available(ins.first->second.shape) ? ins.first->second : e;
  *shape_out = use.shape;
  *streaming_out = use.streaming != 0;
  return HEOM_OK;
}

int autotune_lookup(int device, bool mixed, int N, int KP, int64_t n_tiles, int *shape,
                    int *streaming, double *us, double *us_streaming) {
  const Key key(arch_of(device), mixed ? 1 : 0, N, KP, log2_floor(n_tiles));
  std::lock_guard<std::mutex> lock(g_mu);
  read_file_locked();
  auto it = g_cache.find(key);
  const bool found = it != g_cache.end();
  *shape = found ? it->second.shape : -1;
  if (streaming) *streaming = found ? it->second.streaming : -1;
  if (us)
    for (int s = 0; s < kMaxTileShapes; ++s) us[s] = found ? it->second.us[s] : -1.0;
  if (us_streaming) *us_streaming = found ? it->second.us_streaming : -1.0;
  return HEOM_OK;
}

void autotune_clear() {
  std::lock_guard<std::mutex> lock(g_mu);
  g_cache.clear();
  g_file_read = false;
}

}  // namespace heom
