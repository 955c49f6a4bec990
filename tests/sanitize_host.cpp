// sanitize_host.cpp -- drives the host-side code of the library (parameter
// normalisation, hierarchy enumeration and neighbour tables, the split over
// ranks) and the FP64 oracle on small systems, for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).
// Checks of the results are structural (the link tables are mutual inverses,
// every halo entry points into its owner's range); the values themselves are
// tested elsewhere.  Prints "ok" on success.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "heom_internal.h"

// runtime.cpp (not linked here: it needs the HIP runtime) defines these.
namespace heom {
void set_error(const std::string &) {}
int fail(int status, const std::string &) { return status; }
}  // namespace heom

extern "C" {
typedef struct {
  int32_t n_sites;
  const double *hamiltonian_cm;
  const double *lambda_cm;
  const double *gamma_inv_fs;
  double temperature_K;
  int32_t n_matsubara;
  int32_t low_temp_correction;
  int32_t theta_form;
  const double *trap_rate_per_ps;
  const double *recomb_rate_per_ps;
} oracle_system;
int oracle_propagate_scaled(const oracle_system *s, int32_t depth, int32_t scaled,
                            double filter_tol, const double *rho0, double dt_fs, int64_t n_steps,
                            int64_t record_every, double *rho_out, double *scalars_out,
                            double *state_out, const double *state_in, int32_t n_threads);
int oracle_count(const oracle_system *s, int32_t depth, int64_t *n_ados, int32_t *n_modes);
}

#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::printf("failed: %s (line %d)\n", #c, __LINE__);            \
      std::exit(1);                                                   \
    }                                                                 \
  } while (0)

int main() {
  for (int N : {1, 2, 3, 7}) {
    for (int K : {0, 1, 2}) {
      for (int D : {0, 1, 3, 5}) {
        // Hierarchies of at most a few thousand ADOs (C(M + D, D)).
        double count = 1.0;
        for (int j = 1; j <= D; ++j) count = count * (N * (K + 1) + j) / j;
        if (count > 3000.0) continue;
        std::vector<double> H(2 * N * N, 0.0), lam(N, 35.0), gi(N, 50.0), trap(N, 0.0),
            rec(N, 1e-3);
        for (int a = 0; a < N; ++a) {
          H[2 * (a * N + a)] = 12400.0 + 37.0 * a;
          if (a + 1 < N) H[2 * (a * N + a + 1)] = H[2 * ((a + 1) * N + a)] = -80.0 + a;
        }
        trap[N - 1] = 1.0;
        heom_system sys = {N, H.data(), lam.data(), gi.data(), 300.0, K, 1, 0,
                           trap.data(), rec.data()};
        heom_hierarchy h;
        CHECK(heom::build_params(&sys, &h) == HEOM_OK);
        h.depth = D;
        CHECK(heom::build_tables(&h) == HEOM_OK);
        const int M = h.M;
        for (int m = 0; m < M; ++m)
          for (int64_t i = 0; i < h.n_ados; ++i) {
            const int32_t u = h.up[m * h.stride + i], d = h.down[m * h.stride + i];
            if (u >= 0) CHECK(h.down[m * h.stride + u] == i);
            if (d >= 0) CHECK(h.up[m * h.stride + d] == i);
          }
        const int ranks = static_cast<int>(h.n_ados / 64);
        if (ranks >= 2) {
          heom_shard s;
          CHECK(heom::build_shard(&h, ranks > 5 ? 5 : ranks, &s) == HEOM_OK);
          for (const heom::HaloEntry &e : s.halo) {
            CHECK(e.src >= 0 && e.src < s.n_ranks && e.dst != e.src);
            CHECK(e.src_index >= 0 && e.src_index < s.first[e.src + 1] - s.first[e.src]);
            CHECK(e.dst_index < s.rank[e.dst]->stride);
          }
          for (heom_hierarchy *g : s.rank) delete g;
        }
        // The oracle on the same system: plain, scaled, scaled with a filter.
        oracle_system os = {N, H.data(), lam.data(), gi.data(), 300.0, K, 1, 0, trap.data(),
                            rec.data()};
        int64_t n_ado = 0;
        int32_t n_modes = 0;
        CHECK(oracle_count(&os, D, &n_ado, &n_modes) == 0 && n_ado == h.n_ados);
        std::vector<double> rho0(2 * N * N, 0.0), rho((20 / 5 + 1) * 2 * N * N), sc(3),
            state(2 * n_ado * N * N + 3);
        rho0[0] = 1.0;
        for (int mode = 0; mode < 3; ++mode) {
          const int scaled = mode > 0 ? 1 : 0;
          const double tol = mode == 2 ? 1e-9 : 0.0;
          CHECK(oracle_propagate_scaled(&os, D, scaled, tol, rho0.data(), 1.0, 20, 5, rho.data(),
                                        sc.data(), state.data(), nullptr, 2) == 0);
          double tr = sc[0] + sc[1];
          for (int a = 0; a < N; ++a) tr += rho[(20 / 5) * 2 * N * N + 2 * (a * N + a)];
          CHECK(std::fabs(tr - 1.0) < 1e-12);
        }
      }
    }
  }
  std::printf("ok\n");
  return 0;
}
