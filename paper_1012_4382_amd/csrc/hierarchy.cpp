// hierarchy.cpp -- enumeration of the ADO hierarchy and its neighbour tables
// (host).
//
// The ADOs are all multi-indices n over the M bath modes with |n| <= D (paper,
// eq:M and the truncation after eq:lab8); there are C(M + D, D) of them
// (Appendix B gives this count for one mode per site).  They are ordered
// lexicographically with the last mode varying fastest.  In this order the map
// n -> n + e_m sends consecutive ADOs (those that have the neighbour) to
// consecutive ADOs, and n -> n - e_m sends consecutive ADOs to an increasing
// sequence with small gaps, so that lanes handling consecutive ADOs gather
// their neighbours from nearly contiguous addresses.
//
// Each ADO is linked to its neighbours n +- e_m (Appendix B keeps these links
// in device memory as linked lists); here the links are
// dense int32 tables [M][stride] (-1 where the neighbour does not exist) plus
// the occupation n_m as uint8, laid out so that consecutive lanes read
// consecutive entries.
#include <cstring>
#include <limits>

#include "heom_internal.h"

namespace heom {
namespace {

// count[k][r] = number of k-tuples of non-negative integers with sum <= r
//             = C(k + r, r); saturates at a large sentinel on overflow.
struct Counts {
  int K = 0, R = 0;
  std::vector<int64_t> v;
  int64_t operator()(int k, int r) const { return v[static_cast<size_t>(k) * (R + 1) + r]; }
};

constexpr int64_t kSaturated = std::numeric_limits<int64_t>::max() / 4;

Counts make_counts(int K, int R) {
  Counts c;
  c.K = K;
  c.R = R;
  c.v.assign(static_cast<size_t>(K + 1) * (R + 1), 0);
  for (int r = 0; r <= R; ++r) c.v[r] = 1;  // k = 0: only the empty tuple
  for (int k = 1; k <= K; ++k) {
    int64_t acc = 0;
    for (int r = 0; r <= R; ++r) {
      // tuples of length k with sum <= r: sum over the first entry's value.
      // count(k, r) = count(k, r - 1) + count(k - 1, r)
      const int64_t prev = (r > 0) ? acc : 0;
      int64_t val = prev + c(k - 1, r);
      if (val > kSaturated) val = kSaturated;
      c.v[static_cast<size_t>(k) * (R + 1) + r] = val;
      acc = val;
    }
  }
  return c;
}

// Rank of multi-index n (length M, |n| <= D) in lexicographic order.
int64_t rank_of(const int32_t *n, int M, int D, const Counts &cnt) {
  int64_t r = 0;
  int rem = D;
  for (int j = 0; j < M; ++j) {
    // every tuple whose entry j is smaller (with the same prefix) comes first
    for (int v = 0; v < n[j]; ++v) r += cnt(M - 1 - j, rem - v);
    rem -= n[j];
  }
  return r;
}

}  // namespace

int build_tables(heom_hierarchy *h) {
  const int M = h->M;
  const int D = h->depth;
  if (D < 0) return fail(HEOM_E_INVALID, "depth must be >= 0");
  if (D > 255) return fail(HEOM_E_INVALID, "depth must be <= 255");
  const Counts cnt = make_counts(M, D);
  const int64_t n = cnt(M, D);
  if (n > std::numeric_limits<int32_t>::max() - kPlanePad)
    return fail(HEOM_E_INVALID, "hierarchy has more than 2^31 - 1 ADOs");
  const int64_t stride = (n + kPlanePad - 1) / kPlanePad * kPlanePad;
  h->n_ados = n;
  h->stride = stride;
  try {
    h->multi.assign(static_cast<size_t>(n) * M, 0);
    h->up.assign(static_cast<size_t>(M) * stride, -1);
    h->down.assign(static_cast<size_t>(M) * stride, -1);
    h->occ.assign(static_cast<size_t>(M) * stride, 0);
  } catch (...) {
    return fail(HEOM_E_NOMEM, "host allocation of the hierarchy tables failed");
  }
  // Enumerate in lexicographic order (odometer with the sum constraint).
  std::vector<int32_t> cur(M, 0);
  int sum = 0;
  for (int64_t i = 0; i < n; ++i) {
    std::memcpy(&h->multi[static_cast<size_t>(i) * M], cur.data(), sizeof(int32_t) * M);
    // advance: increment the last position that can grow, zeroing those after
    for (int j = M - 1; j >= 0; --j) {
      if (sum < D) {
        ++cur[j];
        ++sum;
        break;
      }
      sum -= cur[j];
      cur[j] = 0;
    }
    if (M == 0) break;
  }
  std::vector<int32_t> nb(M);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t *ni = &h->multi[static_cast<size_t>(i) * M];
    int tot = 0;
    for (int m = 0; m < M; ++m) tot += ni[m];
    for (int m = 0; m < M; ++m) {
      h->occ[static_cast<size_t>(m) * stride + i] = static_cast<uint8_t>(ni[m]);
      std::memcpy(nb.data(), ni, sizeof(int32_t) * M);
      if (tot < D) {
        nb[m] = ni[m] + 1;
        h->up[static_cast<size_t>(m) * stride + i] = static_cast<int32_t>(rank_of(nb.data(), M, D, cnt));
      }
      if (ni[m] > 0) {
        nb[m] = ni[m] - 1;
        h->down[static_cast<size_t>(m) * stride + i] = static_cast<int32_t>(rank_of(nb.data(), M, D, cnt));
      }
    }
  }
  return HEOM_OK;
}

}  // namespace heom
