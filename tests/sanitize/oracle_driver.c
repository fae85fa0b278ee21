/* Runs the oracle's whole FMM (tree, traversal, blank passes, every operator)
   and its direct sum on small clouds, for a build with AddressSanitizer and
   UndefinedBehaviorSanitizer.  Test infrastructure: built and run only by
   tests/test_host_sanitizers.py. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/defmm_oracle.h"

static double urand(unsigned long long* s) {
  *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
  return ((*s >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
}

static double run(int64_t n, double kappa, oracle_params prm, int sphere) {
  unsigned long long s = 1234567ULL + (unsigned long long)n;
  double* X = malloc(sizeof(double) * 3 * (size_t)(n + 1));
  double* q = malloc(sizeof(double) * 2 * (size_t)(n + 1));
  double* p = malloc(sizeof(double) * 2 * (size_t)(n + 1));
  for (int64_t i = 0; i < n; ++i) {
    double a = urand(&s), b = urand(&s), c = urand(&s);
    if (sphere) {
      double r = sqrt(a * a + b * b + c * c) + 1e-30;
      a /= r;
      b /= r;
      c /= r;
    }
    X[3 * i] = a;
    X[3 * i + 1] = b;
    X[3 * i + 2] = c;
    q[2 * i] = urand(&s);
    q[2 * i + 1] = urand(&s);
  }
  void* F = oracle_fmm_create(X, n, X, n, 1, kappa, &prm);
  oracle_fmm_apply(F, q, p);
  oracle_fmm_destroy(F);
  double acc = 0.0;
  for (int64_t i = 0; i < 2 * n; ++i) acc += fabs(p[i]);
  oracle_direct_sum(X, n, X, n, q, kappa, 1e-12, NULL, n, p, prm.kernel);
  free(X);
  free(q);
  free(p);
  return acc;
}

int main(void) {
  double acc = 0.0;
  oracle_params a = {4, 16, 1.0, 2.0, 0, ORACLE_HELMHOLTZ};
  acc += run(1500, 30.0, a, 1);
  oracle_params b = {5, 24, 0.5, 0.75, 1, ORACLE_HELMHOLTZ};
  acc += run(1200, 40.0, b, 1);
  oracle_params c = {3, 8, 0.7, 2.0, 0, ORACLE_YUKAWA};
  acc += run(1000, 5.0, c, 0);
  oracle_params d = {4, 64, 1.0, 2.0, 0, ORACLE_HELMHOLTZ};
  acc += run(40, 10.0, d, 1);
  printf("oracle driver: ok (%g)\n", acc);
  return 0;
}
