/* A C program against include/heom.h and libheom.so, host functions only (no
 * GPU needed): builds the FMO Table 1 hierarchy at depth 4, checks its size
 * C(7 + 4, 4) = 330 (the paper's N_max = 4 count), its neighbour tables and
 * modes, and the argument validation of the device entry points.  Prints
 * "ok" and exits 0 on success.  Built and run by tests/test_c_abi.py. */
#include <stdio.h>
#include <stdlib.h>

#include "heom.h"

#define CHECK(cond)                                                         \
  do {                                                                      \
    if (!(cond)) {                                                          \
      printf("failed: %s (line %d): %s\n", #cond, __LINE__, heom_last_error()); \
      return 1;                                                             \
    }                                                                       \
  } while (0)

int main(void) {
  static const double h_cm[7][7] = {
      {12410, -87.7, 5.5, -5.9, 6.7, -13.7, -9.9},  {-87.7, 12530, 30.8, 8.2, 0.7, 11.8, 4.3},
      {5.5, 30.8, 12210, -53.5, -2.2, -9.6, 6.0},   {-5.9, 8.2, -53.5, 12320, -70.7, -17.0, -63.3},
      {6.7, 0.7, -2.2, -70.7, 12480, 81.1, -1.3},   {-13.7, 11.8, -9.6, -17.0, 81.1, 12630, 39.7},
      {-9.9, 4.3, 6.0, -63.3, -1.3, 39.7, 12440}};
  double hc[7 * 7 * 2], lam[7], ginv[7], trap[7] = {0, 0, 0.4, 0.4, 0, 0, 0}, rec[7];
  for (int i = 0; i < 7; ++i) {
    for (int j = 0; j < 7; ++j) {
      hc[2 * (i * 7 + j)] = h_cm[i][j];
      hc[2 * (i * 7 + j) + 1] = 0.0;
    }
    lam[i] = 35.0;
    ginv[i] = 166.0;
    rec[i] = 1.0 / 250.0;
  }
  heom_system sys = {7, hc, lam, ginv, 300.0, 0, 1, 0, trap, rec};
  heom_hierarchy *h = NULL;
  CHECK(heom_build_hierarchy(&sys, 4, &h) == HEOM_OK && h != NULL);
  int64_t n = 0;
  int32_t m = 0;
  size_t b64 = 0, b32 = 0;
  CHECK(heom_hierarchy_info(h, &n, &m, &b64, &b32) == HEOM_OK);
  CHECK(n == 330 && m == 7 && b32 < b64);
  int32_t *multi = malloc(sizeof(int32_t) * n * m), *up = malloc(sizeof(int32_t) * n * m),
          *down = malloc(sizeof(int32_t) * n * m);
  CHECK(heom_hierarchy_tables(h, multi, up, down) == HEOM_OK);
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < m; ++k) {
      if (up[i * m + k] >= 0) CHECK(down[up[i * m + k] * m + k] == i);
      if (down[i * m + k] >= 0) CHECK(multi[down[i * m + k] * m + k] == multi[i * m + k] - 1);
    }
  double cre[7], cim[7], nu[7], delta[7];
  int32_t site[7];
  CHECK(heom_hierarchy_modes(h, site, cre, cim, nu, delta) == HEOM_OK);
  for (int k = 0; k < 7; ++k) CHECK(site[k] == k && nu[k] > 0 && cim[k] < 0 && delta[k] > 0);
  /* Validation happens before any device work. */
  double rho0[7 * 7 * 2] = {0};
  rho0[0] = 1.0;
  CHECK(heom_propagate(h, 7, 0, rho0, 1.0, 10, 1, (void *)4096, b64, NULL, NULL, NULL) ==
        HEOM_E_UNSUPPORTED);
  CHECK(heom_propagate(h, HEOM_FP64, 0, rho0, -1.0, 10, 1, (void *)4096, b64, NULL, NULL, NULL) ==
        HEOM_E_INVALID);
  CHECK(heom_propagate(h, HEOM_FP64, 0, rho0, 1.0, 10, 1, NULL, b64, NULL, NULL, NULL) ==
        HEOM_E_WORKSPACE);
  CHECK(heom_propagate(h, HEOM_FP64, HEOM_TILE_SHAPE(9), rho0, 1.0, 10, 1, (void *)4096, b64, NULL,
                       NULL, NULL) == HEOM_E_INVALID);
  sys.n_sites = 0;
  heom_hierarchy *bad = NULL;
  CHECK(heom_build_hierarchy(&sys, 4, &bad) == HEOM_E_INVALID && bad == NULL);
  free(multi);
  free(up);
  free(down);
  heom_destroy(h);
  heom_destroy(NULL);
  printf("ok\n");
  return 0;
}
