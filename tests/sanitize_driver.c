/* Driver for the sanitizer build of the C parts of the test infrastructure
 * (oracle/wilson.c and qcd_inputs/gen.c): generates links, gauge
 * transformations and sources, applies the Wilson operator in its four forms
 * and at listed sites on small lattices of odd and ragged extents, and checks
 * that D with kappa = 0 is the identity and that every output is finite.
 * Built and run by tests/test_sanitize.py with AddressSanitizer and
 * UndefinedBehaviorSanitizer; exit status 0 when every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void or_dslash(const int dims[4], const double *U, const double *phi, double *out, double kappa, int op);
void or_dslash_sites(const int dims[4], const double *U, const double *phi, double *out, double kappa,
                     const int64_t *sites, int64_t n);
void qi_gauge(double *U, int64_t volume, double eps, uint64_t seed);
void qi_gauge_transform(double *g, int64_t volume, double eps, uint64_t seed);
void qi_gaussian(double *psi, int64_t ncomplex, uint64_t seed);
void qi_uniform(double *out, int64_t n, uint64_t seed);
void qi_splitmix_raw(uint64_t state, uint64_t *out, int64_t n);

static int all_finite(const double *x, int64_t n) {
  for (int64_t i = 0; i < n; i++)
    if (!isfinite(x[i])) return 0;
  return 1;
}

int main(void) {
  const int shapes[][4] = {{2, 2, 2, 2}, {2, 4, 6, 10}, {3, 5, 1, 2}, {1, 1, 1, 1}, {4, 2, 2, 6}};
  int fails = 0;
  for (size_t c = 0; c < sizeof shapes / sizeof shapes[0]; c++) {
    const int *d = shapes[c];
    const int64_t V = (int64_t)d[0] * d[1] * d[2] * d[3];
    double *U = malloc(sizeof(double) * 2 * 36 * V), *G = malloc(sizeof(double) * 2 * 9 * V);
    const int64_t nout = V > 4 ? V : 4;  /* the site list below has 4 entries */
    double *psi = malloc(sizeof(double) * 2 * 12 * V), *out = malloc(sizeof(double) * 2 * 12 * nout);
    double *uni = malloc(sizeof(double) * 64);
    uint64_t raw[8];
    qi_gauge(U, V, 0.3, 11 + c);
    qi_gauge_transform(G, V, 1.0, 21 + c);
    qi_gaussian(psi, 12 * V, 31 + c);
    qi_uniform(uni, 64, 41 + c);
    qi_splitmix_raw(1234567 + c, raw, 8);
    fails += !all_finite(U, 72 * V) + !all_finite(G, 18 * V) + !all_finite(psi, 24 * V) + !all_finite(uni, 64);
    for (int op = 0; op < 4; op++) {
      or_dslash(d, U, psi, out, 0.124, op);
      fails += !all_finite(out, 24 * V);
    }
    or_dslash(d, U, psi, out, 0.0, 0);
    for (int64_t i = 0; i < 24 * V; i++) fails += out[i] != psi[i];
    int64_t sites[4] = {0, V - 1, V / 2, V > 1 ? 1 : 0};
    or_dslash_sites(d, U, psi, out, 0.124, sites, 4);
    fails += !all_finite(out, 24 * 4);
    free(U);
    free(G);
    free(psi);
    free(out);
    free(uni);
  }
  printf("sanitize driver: %d failed checks\n", fails);
  return fails != 0;
}
