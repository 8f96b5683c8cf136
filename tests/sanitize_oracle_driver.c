/* Host sanitizer run of the FP64 oracle (test infrastructure): the oracle's
 * translation unit is included whole and built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py).  Every radius,
 * the smallest and largest stride, both weight kinds, forward with saved
 * inputs and backward, on small ragged images; then the argument errors.
 * Exit status 0 when every call returned as expected. */
#include "../oracle/sgwls_oracle.c"

#include <math.h>
#include <stdio.h>

static double frand(unsigned* s) {
  *s = *s * 1664525u + 1013904223u;
  return (double)(*s >> 8) / 16777216.0;
}

int main(void) {
  unsigned seed = 12345u;
  int failures = 0;
  for (int r = 1; r <= 4; ++r)
    for (int si = 0; si < 2; ++si)
      for (int kind = 0; kind < 2; ++kind) {
        const int stride = si == 0 ? 1 : 2 * r + 1;
        const int C = 2, M = 2 * r + 4, N = 2 * r + 7;
        const size_t n = (size_t)C * M * N;
        orc_params p = {3.0, r, 2, stride, kind, (double)r, 0.2, 1.2, 1.2, 1e-2};
        double* F = malloc(sizeof(double) * n);
        double* U = malloc(sizeof(double) * n);
        double* g = malloc(sizeof(double) * M * N);
        double* saved = malloc(sizeof(double) * n * 2 * p.iters);
        double* Ub = malloc(sizeof(double) * n);
        double* Fb = malloc(sizeof(double) * n);
        double* gb = malloc(sizeof(double) * M * N);
        double lb = 0.0;
        for (size_t i = 0; i < n; ++i) { F[i] = frand(&seed); Ub[i] = frand(&seed) - 0.5; }
        for (int i = 0; i < M * N; ++i) g[i] = frand(&seed);
        int rc = orc_filter(C, M, N, F, g, U, &p, saved);
        if (rc == ORC_OK) rc = orc_filter_backward(C, M, N, g, saved, Ub, Fb, gb, &lb, &p);
        int finite = isfinite(lb);
        for (size_t i = 0; i < n; ++i) finite &= isfinite(U[i]) && isfinite(Fb[i]);
        if (rc != ORC_OK || !finite) {
          fprintf(stderr, "r=%d stride=%d kind=%d: rc %d finite %d\n", r, stride, kind, rc, finite);
          ++failures;
        }
        free(F); free(U); free(g); free(saved); free(Ub); free(Fb); free(gb);
      }
  /* argument errors return codes */
  double a[64], b[64], c[64];
  for (int i = 0; i < 64; ++i) a[i] = b[i] = 0.5;
  orc_params bad = {1.0, 0, 1, 1, 0, 1.0, 0.1, 1.2, 1.2, 1e-4};
  if (orc_filter(1, 8, 8, a, b, c, &bad, NULL) == ORC_OK) ++failures;
  bad.r = 1;
  bad.stride = 4;
  if (orc_filter(1, 8, 8, a, b, c, &bad, NULL) == ORC_OK) ++failures;
  bad.stride = 1;
  if (orc_filter(1, 8, 8, NULL, b, c, &bad, NULL) == ORC_OK) ++failures;
  if (orc_filter(1, 2, 8, a, b, c, &bad, NULL) == ORC_OK) ++failures;
  printf("sanitized oracle run: %d failures\n", failures);
  return failures ? 1 : 0;
}
