/* Drives the oracle's entry points on small seeded problems so that the
 * oracle can be built and run under AddressSanitizer and
 * UndefinedBehaviorSanitizer on the CPU (test infrastructure only). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/cfust_oracle.h"

static unsigned long long st = 88172645463325252ull;
static double unif(void) { /* xorshift64, mapped into (0, 1) */
  st ^= st << 13;
  st ^= st >> 7;
  st ^= st << 17;
  return ((double)(st >> 11) + 0.5) / 9007199254740992.0;
}

static int run_case(int n, int p, int q, int g, int N) {
  const int S = orc_stats_size(p, q);
  double *y = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * p);
  double *pi = malloc(sizeof(double) * g), *mu = malloc(sizeof(double) * g * p);
  double *Sg = malloc(sizeof(double) * g * p * p), *Dl = malloc(sizeof(double) * g * p * q);
  double *nu = malloc(sizeof(double) * g), *u = malloc(sizeof(double) * N * (q + 1));
  double *tau = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * g);
  double *logf = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * g);
  double *e1 = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * g);
  double *e2 = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * g);
  double *e3 = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * g * q);
  double *e4 = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * g * q * q);
  double *stats = malloc(sizeof(double) * g * S), ll = 0.0;
  double *trace = malloc(sizeof(double) * 4);
  int bad = -1, it = 0, rc = 0;
  for (int k = 0; k < n * p; ++k) y[k] = 4.0 * unif() - 2.0;
  for (int i = 0; i < g; ++i) {
    pi[i] = 1.0 / g;
    nu[i] = 4.0 + 6.0 * unif();
    for (int a = 0; a < p; ++a) {
      mu[i * p + a] = unif() - 0.5;
      for (int b = 0; b < p; ++b) Sg[(i * p + a) * p + b] = (a == b) ? 1.0 + unif() : 0.1;
      for (int l = 0; l < q; ++l) Dl[(i * p + a) * q + l] = unif() - 0.5;
    }
  }
  for (int k = 0; k < N * (q + 1); ++k) u[k] = unif();
  for (int mode = 0; mode < 3 && !rc; ++mode)
    for (int reorder = 0; reorder < 2 && !rc; ++reorder)
      rc = orc_estep(y, n, p, q, g, pi, mu, Sg, Dl, nu, u, N, mode, reorder, tau, logf, e1, e2, e3,
                     e4, stats, &ll, &bad);
  if (!rc) rc = orc_loglik(y, n, p, q, g, pi, mu, Sg, Dl, nu, u, N, 0, &ll, logf);
  if (!rc && n > 0)
    rc = orc_mstep(stats, n, p, q, g, mu, Dl, nu, 0, 0, 1.0, 200.0, pi, mu, Sg, Dl, nu, &bad);
  if (!rc && n > 0)
    rc = orc_em_fit(y, n, p, q, g, pi, mu, Sg, Dl, nu, u, N, 1, 0, 0, 2, 0.0, 1.0, 200.0, trace,
                    &it, &bad);
  printf("case n=%d p=%d q=%d g=%d N=%d: rc %d\n", n, p, q, g, N, rc);
  free(y); free(pi); free(mu); free(Sg); free(Dl); free(nu); free(u); free(tau); free(logf);
  free(e1); free(e2); free(e3); free(e4); free(stats); free(trace);
  /* ENOTPD from a random start is a valid outcome; memory errors abort */
  return (rc == ORC_OK || rc == ORC_ENOTPD) ? 0 : 1;
}

int main(void) {
  int fails = 0;
  fails += run_case(0, 2, 2, 2, 64);
  fails += run_case(9, 3, 2, 2, 65);
  fails += run_case(7, 2, 4, 3, 33);
  fails += run_case(5, 5, 5, 2, 17);
  fails += run_case(3, 12, 11, 2, 9);
  double EV[3], EVV[9], lT;
  const double h[3] = {0.3, -1.0, 2.0}, C[9] = {1, 0, 0, 0.3, 0.9, 0, -0.2, 0.1, 0.95};
  double u[64 * 4];
  for (int k = 0; k < 64 * 4; ++k) u[k] = unif();
  int perm[3];
  fails += orc_ghk(3, h, C, 7.0, u, 64, 1, &lT, EV, EVV) != 0;
  const double R[9] = {1, 0.3, -0.2, 0.3, 1, 0.1, -0.2, 0.1, 1};
  fails += orc_ghk_ordered(3, h, R, 7.0, u, 64, 1, &lT, EV, EVV, perm) != 0;
  printf("%s\n", fails ? "FAILED" : "SANITIZED_OK");
  return fails ? 1 : 0;
}
