// shard.cpp -- one hierarchy split into contiguous ranges of its ADO order,
// one per rank (host).
//
// A hierarchy too large for one GPU is propagated by several, each holding one
// range.  Every RK4 stage couples each ADO to its neighbours n +- e_m (eq:lab8),
// so a rank needs, before each stage, the stage input of the other ranks' ADOs
// its own ADOs link to (its halo).  Here each rank becomes an instance of its
// own: its neighbour tables point at its own ADOs (local indices) and at halo
// slots after them, and a list names, for each halo slot, the owning rank and
// that rank's local index.  On one GPU the halo copy stands in for the
// exchange; the stage kernel runs each rank's share unchanged.
#include <algorithm>

#include "heom_internal.h"

namespace heom {

namespace {

// Packed reals of an ADO in the rows and columns of the sites in `sites`
// (diagonal entries count once, off-diagonal pairs twice).
int64_t reals_for_sites(int N, int n_sites) {
  const int64_t pairs = static_cast<int64_t>(N) * (N - 1) / 2 -
                        static_cast<int64_t>(N - n_sites) * (N - n_sites - 1) / 2;
  return n_sites + 2 * pairs;
}

}  // namespace

int build_shard(const heom_hierarchy *h, int n_ranks, heom_shard *s) {
  const int64_t n = h->n_ados;
  const int M = h->M, N = h->N;
  if (n_ranks < 1) return fail(HEOM_E_INVALID, "n_ranks must be >= 1");
  if (n < kPlanePad * static_cast<int64_t>(n_ranks))
    return fail(HEOM_E_INVALID, "fewer than 64 ADOs per rank");
  s->n_ranks = n_ranks;
  s->N = N;
  s->M = M;
  s->n_ados = n;
  // Ranges of equal size, rounded to whole 64-ADO tiles.
  s->first.assign(n_ranks + 1, n);
  for (int r = 0; r < n_ranks; ++r)
    s->first[r] = (n * r / n_ranks) / kPlanePad * kPlanePad;
  s->stats.assign(n_ranks, heom_shard::Stats());
  for (int r = 0; r < n_ranks; ++r) {
    const int64_t lo = s->first[r], hi = s->first[r + 1], nl = hi - lo;
    // Halo: every ADO outside [lo, hi) that a local ADO links to, ascending,
    // with the sites whose modes make the links.
    std::vector<int32_t> halo;
    for (int m = 0; m < M; ++m)
      for (int64_t i = lo; i < hi; ++i)
        for (const std::vector<int32_t> *t : {&h->up, &h->down}) {
          const int32_t j = (*t)[static_cast<size_t>(m) * h->stride + i];
          if (j >= 0 && (j < lo || j >= hi)) halo.push_back(j);
        }
    std::sort(halo.begin(), halo.end());
    halo.erase(std::unique(halo.begin(), halo.end()), halo.end());
    auto slot_of = [&](int32_t j) -> int32_t {
      if (j < 0) return -1;
      if (j >= lo && j < hi) return static_cast<int32_t>(j - lo);
      const auto it = std::lower_bound(halo.begin(), halo.end(), j);
      return static_cast<int32_t>(nl + (it - halo.begin()));
    };
    const int64_t nh = static_cast<int64_t>(halo.size());
    heom_hierarchy *g = new heom_hierarchy();
    s->rank.push_back(g);
    g->N = h->N;
    g->K = h->K;
    g->KP = h->KP;
    g->M = M;
    g->depth = h->depth;
    g->h_real = h->h_real;
    g->energy_offset = h->energy_offset;
    g->params = h->params;
    g->site = h->site;
    g->c_re = h->c_re;
    g->c_im = h->c_im;
    g->nu = h->nu;
    g->delta = h->delta;
    g->n_ados = nl;
    g->stride = (nl + nh + kPlanePad - 1) / kPlanePad * kPlanePad;
    g->multi.assign(h->multi.begin() + lo * M, h->multi.begin() + hi * M);
    g->up.assign(static_cast<size_t>(M) * g->stride, -1);
    g->down.assign(static_cast<size_t>(M) * g->stride, -1);
    g->occ.assign(static_cast<size_t>(M) * g->stride, 0);
    std::vector<uint64_t> sites_of(nh, 0);  // bit s: a link along a mode of site s
    heom_shard::Stats &st = s->stats[r];
    for (int m = 0; m < M; ++m)
      for (int64_t i = lo; i < hi; ++i) {
        const size_t src = static_cast<size_t>(m) * h->stride + i;
        const size_t dst = static_cast<size_t>(m) * g->stride + (i - lo);
        const int32_t ju = slot_of(h->up[src]), jd = slot_of(h->down[src]);
        g->up[dst] = ju;
        g->down[dst] = jd;
        g->occ[dst] = h->occ[src];
        for (int32_t j : {ju, jd})
          if (j >= nl) {
            ++st.cut_links;
            sites_of[j - nl] |= uint64_t{1} << h->site[m];
          }
      }
    st.n_halo = nh;
    for (int64_t q = 0; q < nh; ++q)
      st.halo_reals_min += reals_for_sites(N, __builtin_popcountll(sites_of[q]));
    // Owner of each halo ADO, its index there and the sites whose rows and
    // columns are read.
    for (int64_t q = 0; q < nh; ++q) {
      const int64_t j = halo[q];
      const int owner = static_cast<int>(
          std::upper_bound(s->first.begin(), s->first.end(), j) - s->first.begin() - 1);
      s->halo.push_back(HaloEntry{r, static_cast<int32_t>(nl + q), owner,
                                  static_cast<int32_t>(j - s->first[owner]), sites_of[q]});
    }
  }
  return HEOM_OK;
}

}  // namespace heom
