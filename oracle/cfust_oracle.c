/*
 * cfust_oracle.c -- plain FP64 CPU oracle for the EM algorithm of a finite
 * mixture of canonical fundamental skew-t (CFUST) distributions.
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
 * CPU-baseline leg call it; the GPU product path does not.  It is slow on
 * purpose: every step is written the obvious way, in the order the method
 * states it, with no blocking, fusion or reordering.  It shares no code, no
 * header and no constant with the GPU library.
 *
 * What it follows (Lee, McLachlan & Leemaqz, "Multi-Node EM Algorithm for
 * Finite Mixture Models"):
 *   - section 2, eq. (1): mixture density; eq. (2): CFUST density
 *     2^q t_p(y; mu, Omega, nu) T_q(Delta^T Omega^{-1}(y-mu) sqrt((nu+p)/(nu+d)); 0, Lambda, nu+p)
 *     with Omega = Sigma + Delta Delta^T, Lambda = I - Delta^T Omega^{-1} Delta,
 *     d = Mahalanobis distance under Omega;
 *   - section 2, eq. (3): log-likelihood; eq. (4): posterior membership tau;
 *   - section 2 (latent gamma and truncated-normal variables) for the
 *     conditional expectations e1..e4, whose expressions the paper leaves to
 *     the CFUST-EM literature; they are re-derived from the hidden-variable
 *     model (see the E-step function below for the identities);
 *   - section 3.2, Algorithm 2: E-step with the per-component partial sums;
 *   - section 3.3, Algorithm 3: M-step per component;
 *   - section 3.4, Algorithm 4: Aitken stopping rule, read with the standard
 *     denominator 1 - a (the printed formula has a typo).
 *
 * The multivariate-t CDF T_q and the truncated moments are approximated with
 * the Genz-Bretz separation-of-variables (GHK) estimator over a given
 * quasi-Monte Carlo point set u[N][q+1]: column 0 picks the chi-square scale,
 * column m (1..q) the m-th sequential truncated-normal draw.
 *
 * Parity status: every function here is pinned by tests against closed forms,
 * scipy special functions, brute-force Monte Carlo or the textbook t-mixture
 * EM; none is marked "parity unpinned".
 */
#include "cfust_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define LN2_ 0.693147180559945309417232121458
#define LOG_SQRT_2PI_ 0.918938533204672741780329736406
#define SQRT1_2_ 0.707106781186547524400844362105
#define LOG_PI_ 1.14472988584940017414342735135

/* ------------------------------------------------------------------------- */
/* special functions                                                         */
/* ------------------------------------------------------------------------- */

/* Phi(x) = erfc(-x / sqrt 2) / 2. */
double orc_norm_cdf(double x) { return 0.5 * erfc(-x * SQRT1_2_); }

/* log Phi(x).  For x <= -30 erfc is near underflow, so Phi is written as
 * phi(t) * M(t), t = -x, with the Mills ratio M(t) = (1 - Phi(t)) / phi(t)
 * evaluated by Laplace's continued fraction
 * M(t) = 1 / (t + 1 / (t + 2 / (t + 3 / (t + ...)))). */
double orc_log_norm_cdf(double x) {
  if (x > 0.0) return log1p(-0.5 * erfc(x * SQRT1_2_));
  if (x > -30.0) return log(0.5 * erfc(-x * SQRT1_2_));
  double t = -x;
  double tail = t;
  for (int k = 400; k >= 1; --k) tail = t + (double)k / tail;
  return -0.5 * t * t - LOG_SQRT_2PI_ - log(tail);
}

/* Lower-half standard normal quantile from log p, log p <= log(1/2):
 * the root w <= 0 of log Phi(w) = log p by Newton's method on log Phi
 * (concave, so after the first step the iterates rise monotonically to the
 * root).  Start: Abramowitz & Stegun 26.2.23. */
double orc_norm_quantile_log(double log_p) {
  if (log_p >= -LN2_) return 0.0;
  double t = sqrt(-2.0 * log_p);
  double w = -(t - (2.515517 + 0.802853 * t + 0.010328 * t * t) /
                       (1.0 + 1.432788 * t + 0.189269 * t * t + 0.001308 * t * t * t));
  if (w > 0.0) w = 0.0;
  for (int it = 0; it < 200; ++it) {
    double lphi = orc_log_norm_cdf(w);
    double dlog = exp(-0.5 * w * w - LOG_SQRT_2PI_ - lphi); /* phi(w) / Phi(w) */
    double step = (lphi - log_p) / dlog;
    w -= step;
    if (fabs(step) <= 1e-15 * fmax(1.0, fabs(w))) break;
  }
  return w;
}

/* Standard normal quantile for p in (0,1). */
double orc_norm_quantile(double p) {
  if (!(p > 0.0 && p < 1.0)) return NAN;
  if (p <= 0.5) return orc_norm_quantile_log(log(p));
  return -orc_norm_quantile_log(log1p(-p));
}

/* Digamma for x > 0: upward recurrence psi(x) = psi(x+1) - 1/x to x >= 10,
 * then the asymptotic series ln x - 1/(2x) - sum B_2k / (2k x^2k). */
double orc_digamma(double x) {
  double r = 0.0;
  while (x < 10.0) {
    r -= 1.0 / x;
    x += 1.0;
  }
  double x2 = 1.0 / (x * x);
  r += log(x) - 0.5 / x -
       x2 * (1.0 / 12 -
             x2 * (1.0 / 120 -
                   x2 * (1.0 / 252 -
                         x2 * (1.0 / 240 - x2 * (1.0 / 132 - x2 * (691.0 / 32760 - x2 / 12))))));
  return r;
}

/* Regularised incomplete gamma functions P(a,x), Q(a,x) = 1 - P(a,x):
 * power series of P for x < a+1, continued fraction of Q otherwise
 * (evaluated with the modified Lentz method). */
static void gamma_pq(double a, double x, double* P, double* Q) {
  if (x <= 0.0) {
    *P = 0.0;
    *Q = 1.0;
    return;
  }
  double lpref = a * log(x) - x - lgamma(a); /* log(x^a e^-x / Gamma(a)) */
  if (x < a + 1.0) {
    /* P = x^a e^-x / Gamma(a) * sum_k x^k / (a (a+1) ... (a+k)) */
    double term = 1.0 / a, sum = term;
    for (int k = 1; k < 100000; ++k) {
      term *= x / (a + k);
      sum += term;
      if (term < sum * 1e-17) break;
    }
    *P = exp(lpref) * sum;
    *Q = 1.0 - *P;
  } else {
    /* Q = x^a e^-x / Gamma(a) * 1/(x+1-a- 1(1-a)/(x+3-a- 2(2-a)/(x+5-a- ...))) */
    const double tiny = 1e-300;
    double b = x + 1.0 - a;
    double c = 1.0 / tiny;
    double d = 1.0 / b;
    double h = d;
    for (int i = 1; i < 100000; ++i) {
      double an = -i * (i - a);
      b += 2.0;
      d = an * d + b;
      if (fabs(d) < tiny) d = tiny;
      c = b + an / c;
      if (fabs(c) < tiny) c = tiny;
      d = 1.0 / d;
      double del = d * c;
      h *= del;
      if (fabs(del - 1.0) < 1e-17) break;
    }
    *Q = exp(lpref) * h;
    *P = 1.0 - *Q;
  }
}

double orc_gamma_p(double a, double x) {
  double P, Q;
  gamma_pq(a, x, &P, &Q);
  return P;
}
double orc_gamma_q(double a, double x) {
  double P, Q;
  gamma_pq(a, x, &P, &Q);
  return Q;
}

/* Chi-square quantile: x with P(dof/2, x/2) = u.  Safeguarded Newton on
 * P - u (u <= 1/2) or (1-u) - Q (u > 1/2), bracketed, to a relative step
 * below 1e-15.  Start: Wilson-Hilferty. */
double orc_chi2_quantile(double u, double dof) {
  if (!(u > 0.0 && u < 1.0) || !(dof > 0.0)) return NAN;
  double a = 0.5 * dof;
  double z = orc_norm_quantile(u);
  double wh = 1.0 - 1.0 / (9.0 * a) + z / (3.0 * sqrt(a));
  double x = a * wh * wh * wh;
  if (!(x > 0.0)) x = 1e-3 * a;
  double lo = 0.0, hi = INFINITY;
  double lga = lgamma(a);
  for (int it = 0; it < 500; ++it) {
    double P, Q;
    gamma_pq(a, x, &P, &Q);
    double f = (u <= 0.5) ? (P - u) : ((1.0 - u) - Q);
    if (f < 0.0)
      lo = x;
    else
      hi = x;
    double dens = exp((a - 1.0) * log(x) - x - lga);
    double xn = x - f / dens;
    /* stop when the Newton step is at rounding level or the bracket has
     * closed to a few ulp (P, Q carry about 1e-15 absolute rounding) */
    if (fabs(xn - x) <= 1e-15 * x || hi - lo <= 4e-16 * x) {
      if (xn > lo && xn < hi) x = xn;
      break;
    }
    if (!(xn > lo && xn < hi)) xn = isinf(hi) ? 2.0 * x : 0.5 * (lo + hi);
    x = xn;
  }
  return 2.0 * x;
}

/* Derivative of the chi-square quantile with respect to the degrees of
 * freedom.  x = orc_chi2_quantile(u, dof) solves P(a, z) = u with a = dof/2,
 * z = x/2; differentiating, dz/da = -(dP/da) / (dP/dz), and since x = 2z and
 * dof = 2a, dx/d(dof) = dz/da.  Here dP/dz = z^(a-1) e^(-z) / Gamma(a) and,
 * term by term from the series P(a, z) = sum_{k>=0} e^(-z) z^(a+k) / Gamma(a+k+1),
 *   dP/da = sum_{k>=0} e^(-z) z^(a+k) / Gamma(a+k+1) * (log z - psi(a+k+1)).
 * Each term is evaluated on its own (log-gamma and digamma per term); the sum
 * stops once the terms, past their peak at a+k ~ z, fall below 1e-20. */
double orc_chi2_quantile_ddof(double u, double dof) {
  const double a = 0.5 * dof;
  const double z = 0.5 * orc_chi2_quantile(u, dof);
  const double lz = log(z);
  double dPda = 0.0;
  for (int k = 0; k < 100000; ++k) {
    const double w = exp((a + k) * lz - z - lgamma(a + k + 1.0));
    dPda += w * (lz - orc_digamma(a + k + 1.0));
    if (a + k > z && w < 1e-20) break;
  }
  const double dPdz = exp((a - 1.0) * lz - z - lgamma(a));
  return -dPda / dPdz;
}

/* ------------------------------------------------------------------------- */
/* small dense linear algebra                                                */
/* ------------------------------------------------------------------------- */

/* A = L L^T, L lower (m*m row-major).  Returns 0 on success, 1 when a
 * pivot (the squared diagonal entry of L) is not above min_pivot. */
static int cholesky_min(const double* A, int m, double* L, double min_pivot) {
  memset(L, 0, sizeof(double) * m * m);
  for (int j = 0; j < m; ++j) {
    double s = A[j * m + j];
    for (int k = 0; k < j; ++k) s -= L[j * m + k] * L[j * m + k];
    if (!(s > min_pivot) || !isfinite(s)) return 1;
    L[j * m + j] = sqrt(s);
    for (int i = j + 1; i < m; ++i) {
      double t = A[i * m + j];
      for (int k = 0; k < j; ++k) t -= L[i * m + k] * L[j * m + k];
      L[i * m + j] = t / L[j * m + j];
    }
  }
  return 0;
}

static int cholesky(const double* A, int m, double* L) { return cholesky_min(A, m, L, 0.0); }

/* A = L L^T with every pivot above rel times its diagonal entry A_jj (the
 * share of coordinate j's variance left after the earlier coordinates);
 * returns 1 otherwise. */
static int cholesky_rel(const double* A, int m, double* L, double rel) {
  memset(L, 0, sizeof(double) * m * m);
  for (int j = 0; j < m; ++j) {
    double s = A[j * m + j];
    for (int k = 0; k < j; ++k) s -= L[j * m + k] * L[j * m + k];
    if (!(s > rel * A[j * m + j]) || !isfinite(s)) return 1;
    L[j * m + j] = sqrt(s);
    for (int i = j + 1; i < m; ++i) {
      double t = A[i * m + j];
      for (int k = 0; k < j; ++k) t -= L[i * m + k] * L[j * m + k];
      L[i * m + j] = t / L[j * m + j];
    }
  }
  return 0;
}

/* solve L x = b (forward) */
static void fwd_solve(const double* L, int m, const double* b, double* x) {
  for (int i = 0; i < m; ++i) {
    double t = b[i];
    for (int k = 0; k < i; ++k) t -= L[i * m + k] * x[k];
    x[i] = t / L[i * m + i];
  }
}

/* solve L^T x = b (backward) */
static void bwd_solve(const double* L, int m, const double* b, double* x) {
  for (int i = m - 1; i >= 0; --i) {
    double t = b[i];
    for (int k = i + 1; k < m; ++k) t -= L[k * m + i] * x[k];
    x[i] = t / L[i * m + i];
  }
}

static int tri_idx(int a, int b, int m) {
  if (a > b) {
    int t = a;
    a = b;
    b = t;
  }
  return a * m - a * (a - 1) / 2 + (b - a);
}

int orc_stats_size(int p, int q) { return 3 + p + q + p * q + p * (p + 1) / 2 + q * (q + 1) / 2; }

/* offsets of s1..s8 inside one component's row of stats */
typedef struct {
  int s1, s2, s3, s4, s5, s6, s7, s8, S;
} offs_t;

static offs_t stat_offsets(int p, int q) {
  offs_t o;
  o.s1 = 0;
  o.s2 = 1;
  o.s3 = 2;
  o.s4 = o.s3 + p;
  o.s5 = o.s4 + q;
  o.s6 = o.s5 + q * (q + 1) / 2;
  o.s7 = o.s6 + p * q;
  o.s8 = o.s7 + p * (p + 1) / 2;
  o.S = o.s8 + 1;
  return o;
}

/* ------------------------------------------------------------------------- */
/* GHK estimator of the multivariate-t CDF and truncated moments             */
/* ------------------------------------------------------------------------- */

/* For V ~ t_q(0, R, dof), R = C C^T:  V = C eps / s, eps ~ N(0, I_q),
 * s = sqrt(chi2_dof / dof).  {V <= h} = {C eps <= s h}: eps_m is drawn in
 * turn from N(0,1) truncated above at
 *   ub_m = (s h_m - sum_{l<m} C_ml eps_l) / C_mm,
 * by inversion eps_m = Phi^{-1}(u_m Phi(ub_m)), and the point's weight is
 * prod_m Phi(ub_m).  Then
 *   P(V <= h)            ~ mean_k weight_k,
 *   E[V | V <= h]        ~ C sum_k weight_k epshat_k / sum_k weight_k,
 *   E[V V^T | V <= h]    ~ C (sum_k weight_k epshat_k epshat_k^T / sum_k weight_k) C^T,
 * with epshat = eps / s.  Weights are kept as logs and summed with a
 * two-pass log-sum-exp.  s[k] is the chi scale for point k.
 * When the draw probability u_m Phi(ub_m) exceeds 1/2 the quantile is taken
 * from the complement 1 - u_m Phi(ub_m) = (1 - u_m) + u_m Phi(-ub_m). */
static void ghk_core(int q, const double* h, const double* C, const double* s,
                     const double* u, int n_qmc, int moments, double* logw, double* ehat,
                     double* logT, double* EV, double* EVV) {
  double eps[64];
  for (int k = 0; k < n_qmc; ++k) {
    const double* uk = u + (size_t)k * (q + 1);
    double lw = 0.0;
    for (int m = 0; m < q; ++m) {
      double acc = s[k] * h[m];
      for (int l = 0; l < m; ++l) acc -= C[m * q + l] * eps[l];
      double ub = acc / C[m * q + m];
      double le = orc_log_norm_cdf(ub);
      lw += le;
      if (m < q - 1 || moments) {
        double um = uk[m + 1];
        double lp = log(um) + le;
        if (lp <= -LN2_) {
          eps[m] = orc_norm_quantile_log(lp);
        } else {
          double comp = (1.0 - um) + um * orc_norm_cdf(-ub);
          eps[m] = -orc_norm_quantile_log(log(comp));
        }
      }
    }
    logw[k] = lw;
    if (moments)
      for (int m = 0; m < q; ++m) ehat[(size_t)k * q + m] = eps[m] / s[k];
  }
  double M = -INFINITY;
  for (int k = 0; k < n_qmc; ++k)
    if (logw[k] > M) M = logw[k];
  if (!isfinite(M)) {
    *logT = -INFINITY;
    if (moments) {
      for (int a = 0; a < q; ++a) EV[a] = 0.0;
      for (int a = 0; a < q * q; ++a) EVV[a] = 0.0;
    }
    return;
  }
  double S0 = 0.0;
  double S1[64];
  double S2[64 * 64];
  if (moments) {
    for (int a = 0; a < q; ++a) S1[a] = 0.0;
    for (int a = 0; a < q * q; ++a) S2[a] = 0.0;
  }
  for (int k = 0; k < n_qmc; ++k) {
    double wk = exp(logw[k] - M);
    S0 += wk;
    if (moments) {
      const double* e = ehat + (size_t)k * q;
      for (int a = 0; a < q; ++a) {
        S1[a] += wk * e[a];
        for (int b = 0; b < q; ++b) S2[a * q + b] += wk * e[a] * e[b];
      }
    }
  }
  *logT = M + log(S0) - log((double)n_qmc);
  if (moments) {
    /* EV = C (S1/S0); EVV = C (S2/S0) C^T */
    double tmp[64 * 64];
    for (int a = 0; a < q; ++a) {
      double t = 0.0;
      for (int l = 0; l <= a; ++l) t += C[a * q + l] * S1[l] / S0;
      EV[a] = t;
    }
    for (int a = 0; a < q; ++a)
      for (int b = 0; b < q; ++b) {
        double t = 0.0;
        for (int l = 0; l <= a; ++l) t += C[a * q + l] * S2[l * q + b] / S0;
        tmp[a * q + b] = t;
      }
    for (int a = 0; a < q; ++a)
      for (int b = 0; b < q; ++b) {
        double t = 0.0;
        for (int l = 0; l <= b; ++l) t += tmp[a * q + l] * C[b * q + l];
        EVV[a * q + b] = t;
      }
  }
}

static void chi_scale_table(const double* u, int n_qmc, int q, double dof, double* s) {
  for (int k = 0; k < n_qmc; ++k) s[k] = sqrt(orc_chi2_quantile(u[(size_t)k * (q + 1)], dof) / dof);
}

/* Tangent of the scale of integral A with respect to a' = dof'/2 at a' = a:
 * the bounds of J(a') (see orc_estep) are s_k(a') h sqrt(a'/a), with
 * s_k(a') = sqrt(x_k(2a') / (2a')), so the factor multiplying h has
 *   t_k = d/da' [s_k(a') sqrt(a'/a)] at a' = a = 2 ds_k/d(dof) + s_k / (2a),
 *   ds_k/d(dof) = (dx_k/d(dof) / dof - x_k / dof^2) / (2 s_k),  dof = 2a. */
static void chi_tangent_table(const double* u, int n_qmc, int q, double a, const double* s,
                              double* t) {
  const double dof = 2.0 * a;
  for (int k = 0; k < n_qmc; ++k) {
    const double uk = u[(size_t)k * (q + 1)];
    const double x = orc_chi2_quantile(uk, dof);
    const double dx = orc_chi2_quantile_ddof(uk, dof);
    const double ds = (dx / dof - x / (dof * dof)) / (2.0 * s[k]);
    t[k] = 2.0 * ds + s[k] / (2.0 * a);
  }
}

/* log P(V <= h) of ghk_core (no moments) and its derivative along a
 * perturbation of the scale: the same estimator with the factor of h at
 * point k moving at rate t[k] (chi_tangent_table), differentiated step by
 * step through the sequential bounds and draws on the same points:
 *   ub_m' = (t_k h_m - sum_{l<m} C_ml eps_l') / C_mm,
 *   (log Phi(ub_m))' = phi(ub_m) / Phi(ub_m) * ub_m',
 *   eps_m' = u_m phi(ub_m) / phi(eps_m) * ub_m'   (from Phi(eps_m) = u_m Phi(ub_m)),
 *   (log weight_k)' = sum_m (log Phi(ub_m))',
 *   (log T)' = sum_k weight_k (log weight_k)' / sum_k weight_k.
 * Ratios of densities are taken in log space. */
static void ghk_tangent(int q, const double* h, const double* C, const double* s, const double* t,
                        const double* u, int n_qmc, double* logw, double* dlw, double* logT,
                        double* dlogT) {
  double eps[64], deps[64];
  for (int k = 0; k < n_qmc; ++k) {
    const double* uk = u + (size_t)k * (q + 1);
    double lw = 0.0, dl = 0.0;
    for (int m = 0; m < q; ++m) {
      double acc = s[k] * h[m], dacc = t[k] * h[m];
      for (int l = 0; l < m; ++l) {
        acc -= C[m * q + l] * eps[l];
        dacc -= C[m * q + l] * deps[l];
      }
      const double ub = acc / C[m * q + m];
      const double dub = dacc / C[m * q + m];
      const double le = orc_log_norm_cdf(ub);
      const double lphi_ub = -0.5 * ub * ub - LOG_SQRT_2PI_;
      lw += le;
      dl += exp(lphi_ub - le) * dub;
      if (m < q - 1) {
        double um = uk[m + 1];
        double lp = log(um) + le;
        if (lp <= -LN2_) {
          eps[m] = orc_norm_quantile_log(lp);
        } else {
          double comp = (1.0 - um) + um * orc_norm_cdf(-ub);
          eps[m] = -orc_norm_quantile_log(log(comp));
        }
        const double lphi_eps = -0.5 * eps[m] * eps[m] - LOG_SQRT_2PI_;
        deps[m] = exp(log(um) + lphi_ub - lphi_eps) * dub;
      }
    }
    logw[k] = lw;
    dlw[k] = dl;
  }
  double M = -INFINITY;
  for (int k = 0; k < n_qmc; ++k)
    if (logw[k] > M) M = logw[k];
  if (!isfinite(M)) {
    *logT = -INFINITY;
    *dlogT = 0.0;
    return;
  }
  double S0 = 0.0, S1 = 0.0;
  for (int k = 0; k < n_qmc; ++k) {
    const double wk = exp(logw[k] - M);
    S0 += wk;
    S1 += wk * dlw[k];
  }
  *logT = M + log(S0) - log((double)n_qmc);
  *dlogT = S1 / S0;
}

int orc_ghk(int q, const double* h, const double* C, double dof, const double* u, int n_qmc,
            int moments, double* logT, double* EV, double* EVV) {
  if (q < 1 || q > 64 || n_qmc < 1 || !(dof > 0.0)) return ORC_EINVAL;
  double* s = (double*)malloc(sizeof(double) * n_qmc);
  double* logw = (double*)malloc(sizeof(double) * n_qmc);
  double* ehat = (double*)malloc(sizeof(double) * (size_t)n_qmc * q);
  if (!s || !logw || !ehat) {
    free(s);
    free(logw);
    free(ehat);
    return ORC_ENOMEM;
  }
  chi_scale_table(u, n_qmc, q, dof, s);
  ghk_core(q, h, C, s, u, n_qmc, moments, logw, ehat, logT, EV, EVV);
  free(s);
  free(logw);
  free(ehat);
  return ORC_OK;
}

int orc_ghk_tangent(int q, const double* h, const double* C, double a, const double* u,
                    int n_qmc, double* logT, double* dlogT) {
  if (q < 1 || q > 64 || n_qmc < 1 || !(a > 0.0)) return ORC_EINVAL;
  double* s = (double*)malloc(sizeof(double) * n_qmc);
  double* t = (double*)malloc(sizeof(double) * n_qmc);
  double* logw = (double*)malloc(sizeof(double) * n_qmc);
  double* dlw = (double*)malloc(sizeof(double) * n_qmc);
  int rc = ORC_OK;
  if (!s || !t || !logw || !dlw) rc = ORC_ENOMEM;
  if (!rc) {
    chi_scale_table(u, n_qmc, q, 2.0 * a, s);
    chi_tangent_table(u, n_qmc, q, a, s, t);
    ghk_tangent(q, h, C, s, t, u, n_qmc, logw, dlw, logT, dlogT);
  }
  free(s);
  free(t);
  free(logw);
  free(dlw);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* variable ordering for the GHK estimator                                   */
/* ------------------------------------------------------------------------- */

/* Genz-Bretz variable prioritisation (Genz & Bretz, "Computation of
 * Multivariate Normal and t Probabilities", 2009, section 4.1.3) for the
 * upper-orthant probability P(Z <= h), Z ~ N(0, R), R a correlation matrix
 * (unit diagonal).  The variables are placed one at a time.  At step i every
 * variable j not yet placed has the standardised conditional bound
 *   b_j = (h_j - sum_{k<i} L_jk y_k) / sqrt(1 - sum_{k<i} L_jk^2),
 * where L_jk (k < i) are the entries of the Cholesky factor computed so far;
 * the variable with the smallest b_j (the smallest conditional probability
 * Phi(b_j); ties go to the lowest index) is placed at step i, the factor is
 * extended by its column, and y_i = E[Z | Z <= b_i] = -phi(b_i) / Phi(b_i).
 * On return perm[i] is the variable placed at step i and Cp (q*q row-major,
 * lower) is the Cholesky factor of R[perm][perm].  The multivariate-t
 * integrals use the order found for the normal one (scale s = 1).
 * Returns ORC_ENOTPD when a pivot is not positive. */
static int genz_order(int q, const double* h, const double* R, int* perm, double* Cp) {
  double Lr[64 * 64]; /* Lr[j][k]: variable j, step k */
  double y[64];
  int used[64];
  for (int j = 0; j < q; ++j) used[j] = 0;
  for (int i = 0; i < q; ++i) {
    int jb = -1;
    double best = 0.0;
    for (int j = 0; j < q; ++j) {
      if (used[j]) continue;
      double s2 = 1.0, num = h[j];
      for (int k = 0; k < i; ++k) {
        s2 -= Lr[j * 64 + k] * Lr[j * 64 + k];
        num -= Lr[j * 64 + k] * y[k];
      }
      double b = num / sqrt(s2);
      if (jb < 0 || b < best) {
        jb = j;
        best = b;
      }
    }
    perm[i] = jb;
    used[jb] = 1;
    double s2 = 1.0;
    for (int k = 0; k < i; ++k) s2 -= Lr[jb * 64 + k] * Lr[jb * 64 + k];
    if (!(s2 > 0.0)) return ORC_ENOTPD;
    double piv = sqrt(s2);
    Lr[jb * 64 + i] = piv;
    for (int j = 0; j < q; ++j) {
      if (used[j]) continue;
      double t = R[j * q + jb];
      for (int k = 0; k < i; ++k) t -= Lr[j * 64 + k] * Lr[jb * 64 + k];
      Lr[j * 64 + i] = t / piv;
    }
    y[i] = -exp(-0.5 * best * best - LOG_SQRT_2PI_ - orc_log_norm_cdf(best));
  }
  for (int i = 0; i < q; ++i)
    for (int k = 0; k < q; ++k) Cp[i * q + k] = (k <= i) ? Lr[perm[i] * 64 + k] : 0.0;
  return ORC_OK;
}

int orc_genz_order(int q, const double* h, const double* R, int* perm, double* Cp) {
  if (q < 1 || q > 64 || !h || !R || !perm || !Cp) return ORC_EINVAL;
  return genz_order(q, h, R, perm, Cp);
}

/* GHK over the variables taken in the order perm (perm NULL: natural order
 * with factor C; otherwise C is the factor of R[perm][perm]).  The bounds are
 * taken in that order, step m uses column m+1 of the points as in ghk_core,
 * and the moments come back in the original labelling. */
static void ghk_in_order(int q, const double* h, const double* C, const int* perm,
                         const double* s, const double* u, int n_qmc, int moments, double* logw,
                         double* ehat, double* logT, double* EV, double* EVV) {
  if (!perm) {
    ghk_core(q, h, C, s, u, n_qmc, moments, logw, ehat, logT, EV, EVV);
    return;
  }
  double hp[64], EVp[64], EVVp[64 * 64];
  for (int i = 0; i < q; ++i) hp[i] = h[perm[i]];
  ghk_core(q, hp, C, s, u, n_qmc, moments, logw, ehat, logT, EVp, EVVp);
  if (moments) {
    for (int i = 0; i < q; ++i) EV[perm[i]] = EVp[i];
    for (int i = 0; i < q; ++i)
      for (int k = 0; k < q; ++k) EVV[perm[i] * q + perm[k]] = EVVp[i * q + k];
  }
}

int orc_ghk_ordered(int q, const double* h, const double* R, double dof, const double* u,
                    int n_qmc, int moments, double* logT, double* EV, double* EVV, int* perm) {
  if (q < 1 || q > 64 || n_qmc < 1 || !(dof > 0.0) || !h || !R || !perm) return ORC_EINVAL;
  for (int j = 0; j < q; ++j)
    if (fabs(R[j * q + j] - 1.0) > 1e-12) return ORC_EINVAL;
  double* Cp = (double*)malloc(sizeof(double) * q * q);
  double* s = (double*)malloc(sizeof(double) * n_qmc);
  double* logw = (double*)malloc(sizeof(double) * n_qmc);
  double* ehat = (double*)malloc(sizeof(double) * (size_t)n_qmc * q);
  int rc = ORC_OK;
  if (!Cp || !s || !logw || !ehat) rc = ORC_ENOMEM;
  if (!rc) rc = genz_order(q, h, R, perm, Cp);
  if (!rc) {
    chi_scale_table(u, n_qmc, q, dof, s);
    ghk_in_order(q, h, Cp, perm, s, u, n_qmc, moments, logw, ehat, logT, EV, EVV);
  }
  free(Cp);
  free(s);
  free(logw);
  free(ehat);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* per-component quantities of eq. (2)                                       */
/* ------------------------------------------------------------------------- */

typedef struct {
  double* L;      /* chol(Omega), p*p */
  double* B;      /* Omega^{-1} Delta, p*q */
  double* D;      /* sqrt(diag Lambda), q */
  double* C;      /* chol(R), R = D^{-1} Lambda D^{-1}, q*q */
  double* R;      /* R itself, q*q (for the variable ordering) */
  double* sA;     /* chi scale table, dof nu+p, N */
  double* sB;     /* chi scale table, dof nu+p+2, N */
  double* sAp;    /* chi scale tables, dof (nu+p)(1 +- ORC_FD_REL) (exact e1 only) */
  double* sAm;
  double* tA;     /* tangent of integral A's scale in a = (nu+p)/2 (exact e1 only) */
  double kappa;   /* log pi + q log 2 + log of t_p's normaliser */
  double nu;
} comp_t;

static int validate_model(int64_t n, int p, int q, int g, const double* pi, const double* mu,
                          const double* Sigma, const double* Delta, const double* nu,
                          const double* y) {
  if (n < 0 || p < 1 || q < 1 || g < 1 || p > 64 || q > 64) return ORC_EINVAL;
  double psum = 0.0;
  for (int i = 0; i < g; ++i) {
    if (!isfinite(pi[i]) || !isfinite(nu[i])) return ORC_ENONFINITE;
    if (!(pi[i] > 0.0) || !(nu[i] > 0.0)) return ORC_EINVAL;
    psum += pi[i];
  }
  if (fabs(psum - 1.0) > 1e-12) return ORC_EINVAL;
  for (int a = 0; a < g * p; ++a)
    if (!isfinite(mu[a])) return ORC_ENONFINITE;
  for (int a = 0; a < g * p * p; ++a)
    if (!isfinite(Sigma[a])) return ORC_ENONFINITE;
  for (int a = 0; a < g * p * q; ++a)
    if (!isfinite(Delta[a])) return ORC_ENONFINITE;
  if (y)
    for (int64_t a = 0; a < n * p; ++a)
      if (!isfinite(y[a])) return ORC_ENONFINITE;
  return ORC_OK;
}

static void free_comps(comp_t* cp, int g) {
  if (!cp) return;
  for (int i = 0; i < g; ++i) {
    free(cp[i].L);
    free(cp[i].B);
    free(cp[i].D);
    free(cp[i].C);
    free(cp[i].R);
    free(cp[i].sA);
    free(cp[i].sB);
    free(cp[i].sAp);
    free(cp[i].sAm);
    free(cp[i].tA);
  }
  free(cp);
}

/* Omega = Sigma + Delta Delta^T, L = chol(Omega), log|Omega| = 2 sum log L_kk,
 * B = Omega^{-1} Delta, Lambda = I - Delta^T B, D = diag(Lambda)^{1/2},
 * R = D^{-1} Lambda D^{-1}, C = chol(R),
 * kappa = log pi + q log 2 + lgamma((nu+p)/2) - lgamma(nu/2) - (p/2) log(nu pi) - log|Omega|/2. */
static int make_comps(int p, int q, int g, const double* pi, const double* Sigma,
                      const double* Delta, const double* nu, const double* u, int n_qmc,
                      int tables, comp_t** out, int* bad) {
  comp_t* cp = (comp_t*)calloc(g, sizeof(comp_t));
  if (!cp) return ORC_ENOMEM;
  double* Om = (double*)malloc(sizeof(double) * p * p);
  double* Lam = (double*)malloc(sizeof(double) * q * q);
  double* Rm = (double*)malloc(sizeof(double) * q * q);
  double* col = (double*)malloc(sizeof(double) * p);
  double* tmp = (double*)malloc(sizeof(double) * p);
  int rc = ORC_OK;
  if (!Om || !Lam || !Rm || !col || !tmp) rc = ORC_ENOMEM;
  for (int i = 0; i < g && rc == ORC_OK; ++i) {
    const double* Sg = Sigma + (size_t)i * p * p;
    const double* Dl = Delta + (size_t)i * p * q;
    comp_t* c = &cp[i];
    c->L = (double*)malloc(sizeof(double) * p * p);
    c->B = (double*)malloc(sizeof(double) * p * q);
    c->D = (double*)malloc(sizeof(double) * q);
    c->C = (double*)malloc(sizeof(double) * q * q);
    c->R = (double*)malloc(sizeof(double) * q * q);
    if (tables) {
      c->sA = (double*)malloc(sizeof(double) * n_qmc);
      c->sB = (double*)malloc(sizeof(double) * n_qmc);
    }
    if (tables == 2) {
      c->sAp = (double*)malloc(sizeof(double) * n_qmc);
      c->sAm = (double*)malloc(sizeof(double) * n_qmc);
    }
    if (tables == 3) c->tA = (double*)malloc(sizeof(double) * n_qmc);
    if (!c->L || !c->B || !c->D || !c->C || !c->R || (tables && (!c->sA || !c->sB)) ||
        (tables == 2 && (!c->sAp || !c->sAm)) || (tables == 3 && !c->tA)) {
      rc = ORC_ENOMEM;
      break;
    }
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < p; ++b) {
        double t = Sg[a * p + b];
        for (int k = 0; k < q; ++k) t += Dl[a * q + k] * Dl[b * q + k];
        Om[a * p + b] = t;
      }
    if (cholesky(Om, p, c->L)) {
      rc = ORC_ENOTPD;
      *bad = i;
      break;
    }
    double logdet = 0.0;
    for (int a = 0; a < p; ++a) logdet += 2.0 * log(c->L[a * p + a]);
    for (int k = 0; k < q; ++k) {
      for (int a = 0; a < p; ++a) col[a] = Dl[a * q + k];
      fwd_solve(c->L, p, col, tmp);
      bwd_solve(c->L, p, tmp, col);
      for (int a = 0; a < p; ++a) c->B[a * q + k] = col[a];
    }
    for (int k = 0; k < q; ++k)
      for (int l = 0; l < q; ++l) {
        double t = (k == l) ? 1.0 : 0.0;
        for (int a = 0; a < p; ++a) t -= Dl[a * q + k] * c->B[a * q + l];
        Lam[k * q + l] = t;
      }
    for (int k = 0; k < q; ++k)
      for (int l = 0; l < k; ++l) {
        double t = 0.5 * (Lam[k * q + l] + Lam[l * q + k]);
        Lam[k * q + l] = t;
        Lam[l * q + k] = t;
      }
    for (int k = 0; k < q; ++k) {
      if (!(Lam[k * q + k] > 0.0)) {
        rc = ORC_ENOTPD;
        *bad = i;
        break;
      }
      c->D[k] = sqrt(Lam[k * q + k]);
    }
    if (rc) break;
    for (int k = 0; k < q; ++k)
      for (int l = 0; l < q; ++l) Rm[k * q + l] = Lam[k * q + l] / (c->D[k] * c->D[l]);
    memcpy(c->R, Rm, sizeof(double) * q * q);
    /* R has a unit diagonal, so its pivots are conditional variances; one at
     * or below ORC_R_PIVOT_MIN makes R numerically singular (the GHK bounds
     * divide by its square root) and counts as not positive definite */
    if (cholesky_min(Rm, q, c->C, ORC_R_PIVOT_MIN)) {
      rc = ORC_ENOTPD;
      *bad = i;
      break;
    }
    double v = nu[i];
    c->nu = v;
    c->kappa = log(pi[i]) + q * LN2_ + lgamma(0.5 * (v + p)) - lgamma(0.5 * v) -
               0.5 * p * (log(v) + LOG_PI_) - 0.5 * logdet;
    if (tables) {
      chi_scale_table(u, n_qmc, q, v + p, c->sA);
      chi_scale_table(u, n_qmc, q, v + p + 2.0, c->sB);
    }
    if (tables == 2) {
      chi_scale_table(u, n_qmc, q, (v + p) * (1.0 + ORC_FD_REL), c->sAp);
      chi_scale_table(u, n_qmc, q, (v + p) * (1.0 - ORC_FD_REL), c->sAm);
    }
    if (tables == 3) chi_tangent_table(u, n_qmc, q, 0.5 * (v + p), c->sA, c->tA);
  }
  free(Om);
  free(Lam);
  free(Rm);
  free(col);
  free(tmp);
  if (rc) {
    free_comps(cp, g);
    return rc;
  }
  *out = cp;
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* E-step (section 2 eq. (2)-(4); section 3.2 Algorithm 2)                   */
/* ------------------------------------------------------------------------- */

/* Per pair (j, i), with r = y_j - mu_i, a = (nu+p)/2, b = (nu+d)/2, c = B^T r:
 *   hidden model: W | y has density prop. to w^{a-1} e^{-b w} Phi_q(sqrt(w) c; Lambda),
 *   U | y, w ~ N_q(c, Lambda / w) truncated to U > 0.
 *   log pi_i f_i(y_j) = kappa - a log1p(d/nu) + log T_A,
 *       T_A = T_q(h_A; R, nu+p),   h_A = D^{-1} c sqrt((nu+p)/(nu+d));
 *   e2 = E[W | y]  = (a/b) T_B / T_A,
 *       T_B = T_q(h_B; R, nu+p+2), h_B = D^{-1} c sqrt((nu+p+2)/(nu+d));
 *   e3 = E[W U | y]     = e2 E[X],  e4 = E[W U U^T | y] = e2 E[X X^T],
 *       X ~ t_q(c, ((nu+d)/(nu+p+2)) Lambda, nu+p+2) truncated to X > 0,
 *       X = c - Ds V with Ds = sqrt((nu+d)/(nu+p+2)) D and V ~ t_q(0,R,nu+p+2), V <= h_B;
 *   e1 = E[log W | y]: with J(a') = T_q(D^{-1} c sqrt(a'/b); R, 2a') (J(a) = T_A),
 *       e1 = psi(a) - log b + d/da log J(a);
 *     nu_mode ORC_NU_OSL uses the one-step-late form d/da log J ~ e2 - a/b,
 *       e1 - e2 = psi(a) - log b - a/b   (exact when Delta = 0);
 *     nu_mode ORC_NU_EXACT takes the derivative of the estimate of J itself,
 *       on the same points (ghk_tangent with chi_tangent_table);
 *     nu_mode ORC_NU_EXACT_FD takes the central difference with step
 *       ORC_FD_REL a on the same points: integrals at dof (nu+p)(1 +- eps)
 *       and bounds h_A sqrt(1 +- eps).
 * Partial sums (Algorithm 2), centred at the current mu_i:
 *   s1 = sum tau, s2 = sum tau e2, s3 = sum tau e2 r, s4 = sum tau e3,
 *   s5 = sum tau e4, s6 = sum tau r e3^T, s7 = sum tau e2 r r^T,
 *   s8 = sum tau (e1 - e2). */
int orc_estep(const double* y, int64_t n, int p, int q, int g, const double* pi,
              const double* mu, const double* Sigma, const double* Delta, const double* nu,
              const double* u, int n_qmc, int nu_mode, int reorder, double* tau, double* logf,
              double* e1, double* e2, double* e3, double* e4, double* stats, double* loglik,
              int* bad_component) {
  int bad = -1;
  if (bad_component) *bad_component = -1;
  if (!y || !pi || !mu || !Sigma || !Delta || !nu || !u || !stats || !loglik) return ORC_EINVAL;
  if (n_qmc < 1) return ORC_EINVAL;
  int rc = validate_model(n, p, q, g, pi, mu, Sigma, Delta, nu, y);
  if (rc) return rc;
  const int exact = nu_mode == ORC_NU_EXACT_FD;
  const int tangent = nu_mode == ORC_NU_EXACT;
  offs_t o = stat_offsets(p, q);
  comp_t* cp = NULL;
  rc = make_comps(p, q, g, pi, Sigma, Delta, nu, u, n_qmc, exact ? 2 : tangent ? 3 : 1, &cp, &bad);
  if (rc) {
    if (bad_component) *bad_component = bad;
    return rc;
  }
  double* logw = (double*)malloc(sizeof(double) * n_qmc);
  double* ehat = (double*)malloc(sizeof(double) * (size_t)n_qmc * q);
  double* dlw = (double*)malloc(sizeof(double) * n_qmc);
  double* lf = (double*)malloc(sizeof(double) * g);
  double* E2 = (double*)malloc(sizeof(double) * g);
  double* E1m2 = (double*)malloc(sizeof(double) * g);
  double* E3 = (double*)malloc(sizeof(double) * g * q);
  double* E4 = (double*)malloc(sizeof(double) * g * q * q);
  double* R = (double*)malloc(sizeof(double) * g * p);
  double* z = (double*)malloc(sizeof(double) * p);
  if (!logw || !ehat || !dlw || !lf || !E2 || !E1m2 || !E3 || !E4 || !R || !z) {
    rc = ORC_ENOMEM;
    goto done;
  }
  memset(stats, 0, sizeof(double) * g * o.S);
  double ll = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    const double* yj = y + j * p;
    for (int i = 0; i < g; ++i) {
      const comp_t* c = &cp[i];
      double v = c->nu;
      double* r = R + i * p;
      for (int a = 0; a < p; ++a) r[a] = yj[a] - mu[i * p + a];
      fwd_solve(c->L, p, r, z);
      double d = 0.0;
      for (int a = 0; a < p; ++a) d += z[a] * z[a];
      double cv[64], hA[64], hB[64];
      for (int k = 0; k < q; ++k) {
        double t = 0.0;
        for (int a = 0; a < p; ++a) t += c->B[a * q + k] * r[a];
        cv[k] = t;
        hA[k] = t / c->D[k] * sqrt((v + p) / (v + d));
        hB[k] = t / c->D[k] * sqrt((v + p + 2.0) / (v + d));
      }
      /* optional variable ordering, found from h_A and used for every
       * integral of the pair */
      int perm[64];
      double Cp[64 * 64];
      const int* pm = NULL;
      const double* Cu = c->C;
      if (reorder) {
        if (genz_order(q, hA, c->R, perm, Cp)) {
          rc = ORC_ENOTPD;
          if (bad_component) *bad_component = i;
          goto done;
        }
        pm = perm;
        Cu = Cp;
      }
      double logTA, logTB, EV[64], EVV[64 * 64];
      ghk_in_order(q, hA, Cu, pm, c->sA, u, n_qmc, 0, logw, ehat, &logTA, NULL, NULL);
      ghk_in_order(q, hB, Cu, pm, c->sB, u, n_qmc, 1, logw, ehat, &logTB, EV, EVV);
      double aa = 0.5 * (v + p), bb = 0.5 * (v + d);
      lf[i] = c->kappa - aa * log1p(d / v) + logTA;
      E1m2[i] = orc_digamma(aa) - log(bb) - aa / bb;
      if (isfinite(logTA) && isfinite(logTB)) {
        double e2v = (aa / bb) * exp(logTB - logTA);
        if (exact) {
          double hP[64], hM[64], lP, lM;
          for (int k = 0; k < q; ++k) {
            hP[k] = hA[k] * sqrt(1.0 + ORC_FD_REL);
            hM[k] = hA[k] * sqrt(1.0 - ORC_FD_REL);
          }
          ghk_in_order(q, hP, Cu, pm, c->sAp, u, n_qmc, 0, logw, ehat, &lP, NULL, NULL);
          ghk_in_order(q, hM, Cu, pm, c->sAm, u, n_qmc, 0, logw, ehat, &lM, NULL, NULL);
          if (isfinite(lP) && isfinite(lM))
            E1m2[i] = orc_digamma(aa) - log(bb) + (lP - lM) / (2.0 * ORC_FD_REL * aa) - e2v;
        }
        if (tangent) {
          double hp[64], lT, dlT;
          for (int k = 0; k < q; ++k) hp[k] = pm ? hA[pm[k]] : hA[k];
          ghk_tangent(q, hp, Cu, c->sA, c->tA, u, n_qmc, logw, dlw, &lT, &dlT);
          E1m2[i] = orc_digamma(aa) - log(bb) + dlT - e2v;
        }
        double sc = sqrt((v + d) / (v + p + 2.0));
        double mx[64];
        for (int k = 0; k < q; ++k) mx[k] = sc * c->D[k] * EV[k];
        E2[i] = e2v;
        for (int k = 0; k < q; ++k) E3[i * q + k] = e2v * (cv[k] - mx[k]);
        for (int k = 0; k < q; ++k)
          for (int l = 0; l < q; ++l) {
            double exx = cv[k] * cv[l] - cv[k] * mx[l] - mx[k] * cv[l] +
                         sc * c->D[k] * EVV[k * q + l] * sc * c->D[l];
            E4[(i * q + k) * q + l] = e2v * exx;
          }
      } else {
        E2[i] = 0.0;
        for (int k = 0; k < q; ++k) E3[i * q + k] = 0.0;
        for (int k = 0; k < q * q; ++k) E4[i * q * q + k] = 0.0;
      }
    }
    /* eq. (3)-(4): log f(y_j) = log sum_i pi_i f_i(y_j); tau_ij = pi_i f_i / f */
    double M = -INFINITY;
    for (int i = 0; i < g; ++i)
      if (lf[i] > M) M = lf[i];
    double ssum = 0.0;
    for (int i = 0; i < g; ++i) ssum += exp(lf[i] - M);
    double lfj = M + log(ssum);
    ll += lfj;
    for (int i = 0; i < g; ++i) {
      double t = exp(lf[i] - lfj);
      double* st = stats + (size_t)i * o.S;
      const double* r = R + i * p;
      const double* e3v = E3 + i * q;
      const double* e4v = E4 + i * q * q;
      /* a pair whose responsibility underflows to zero adds nothing (the
       * limit of tau e as tau -> 0): its GHK ratio T_B/T_A may be beyond
       * the double range, and 0 * inf would poison the sums */
      if (t > 0.0) {
        st[o.s1] += t;
        st[o.s2] += t * E2[i];
        for (int a = 0; a < p; ++a) st[o.s3 + a] += t * E2[i] * r[a];
        for (int k = 0; k < q; ++k) st[o.s4 + k] += t * e3v[k];
        for (int k = 0; k < q; ++k)
          for (int l = k; l < q; ++l) st[o.s5 + tri_idx(k, l, q)] += t * e4v[k * q + l];
        for (int a = 0; a < p; ++a)
          for (int k = 0; k < q; ++k) st[o.s6 + a * q + k] += t * r[a] * e3v[k];
        for (int a = 0; a < p; ++a)
          for (int b = a; b < p; ++b) st[o.s7 + tri_idx(a, b, p)] += t * E2[i] * r[a] * r[b];
        st[o.s8] += t * E1m2[i];
      }
      size_t ji = (size_t)j * g + i;
      if (tau) tau[ji] = t;
      if (logf) logf[ji] = lf[i];
      if (e1) e1[ji] = E2[i] + E1m2[i];
      if (e2) e2[ji] = E2[i];
      if (e3)
        for (int k = 0; k < q; ++k) e3[ji * q + k] = e3v[k];
      if (e4)
        for (int k = 0; k < q * q; ++k) e4[ji * q * q + k] = e4v[k];
    }
  }
  *loglik = ll;
done:
  free(logw);
  free(ehat);
  free(dlw);
  free(lf);
  free(E2);
  free(E1m2);
  free(E3);
  free(E4);
  free(R);
  free(z);
  free_comps(cp, g);
  return rc;
}

/* eq. (3) with integral A only. */
int orc_loglik(const double* y, int64_t n, int p, int q, int g, const double* pi,
               const double* mu, const double* Sigma, const double* Delta, const double* nu,
               const double* u, int n_qmc, int reorder, double* loglik, double* logf) {
  if (!y || !pi || !mu || !Sigma || !Delta || !nu || !u || !loglik) return ORC_EINVAL;
  if (n_qmc < 1) return ORC_EINVAL;
  int rc = validate_model(n, p, q, g, pi, mu, Sigma, Delta, nu, y);
  if (rc) return rc;
  int bad = -1;
  comp_t* cp = NULL;
  rc = make_comps(p, q, g, pi, Sigma, Delta, nu, u, n_qmc, 1, &cp, &bad);
  if (rc) return rc;
  double* logw = (double*)malloc(sizeof(double) * n_qmc);
  double* lf = (double*)malloc(sizeof(double) * g);
  double* r = (double*)malloc(sizeof(double) * p);
  double* z = (double*)malloc(sizeof(double) * p);
  if (!logw || !lf || !r || !z) {
    rc = ORC_ENOMEM;
    goto done;
  }
  double ll = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    for (int i = 0; i < g; ++i) {
      const comp_t* c = &cp[i];
      double v = c->nu;
      for (int a = 0; a < p; ++a) r[a] = y[j * p + a] - mu[i * p + a];
      fwd_solve(c->L, p, r, z);
      double d = 0.0;
      for (int a = 0; a < p; ++a) d += z[a] * z[a];
      double hA[64];
      for (int k = 0; k < q; ++k) {
        double t = 0.0;
        for (int a = 0; a < p; ++a) t += c->B[a * q + k] * r[a];
        hA[k] = t / c->D[k] * sqrt((v + p) / (v + d));
      }
      int perm[64];
      double Cp[64 * 64];
      const int* pm = NULL;
      const double* Cu = c->C;
      if (reorder) {
        if (genz_order(q, hA, c->R, perm, Cp)) {
          rc = ORC_ENOTPD;
          goto done;
        }
        pm = perm;
        Cu = Cp;
      }
      double logTA;
      ghk_in_order(q, hA, Cu, pm, c->sA, u, n_qmc, 0, logw, NULL, &logTA, NULL, NULL);
      lf[i] = c->kappa - 0.5 * (v + p) * log1p(d / v) + logTA;
      if (logf) logf[(size_t)j * g + i] = lf[i];
    }
    double M = -INFINITY;
    for (int i = 0; i < g; ++i)
      if (lf[i] > M) M = lf[i];
    double ssum = 0.0;
    for (int i = 0; i < g; ++i) ssum += exp(lf[i] - M);
    ll += M + log(ssum);
  }
  *loglik = ll;
done:
  free(logw);
  free(lf);
  free(r);
  free(z);
  free_comps(cp, g);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* M-step (section 3.3, Algorithm 3), one component at a time                */
/* ------------------------------------------------------------------------- */

/* Conditional maximisation of the expected complete-data log-likelihood, in
 * the order mu (old Delta), Delta (new mu), Sigma, then nu and pi:
 *   pi    = s1 / n
 *   mu'   = mu + dmu,  dmu = (s3 - Delta s4) / s2
 *   re-centre at mu': s6' = s6 - dmu s4^T,
 *                     s7' = s7 - s3 dmu^T - dmu s3^T + s2 dmu dmu^T
 *   Delta' = s6' s5^{-1}
 *   Sigma' = (s7' - Delta' s6'^T - s6' Delta'^T + Delta' s5 Delta'^T) / s1
 *   nu'   = root of 1 + log(nu/2) - psi(nu/2) + s8/s1 = 0 on [nu_lo, nu_hi]
 *           (bisection; clipped to the bracket when there is no sign change). */
static double nu_equation(double v, double c) { return 1.0 + log(0.5 * v) - orc_digamma(0.5 * v) + c; }

int orc_mstep(const double* stats, int64_t n, int p, int q, int g, const double* mu_old,
              const double* Delta_old, const double* nu_old, int nu_mode, int fix_delta_zero,
              double nu_lo, double nu_hi, double* pi, double* mu, double* Sigma, double* Delta,
              double* nu, int* bad_component) {
  if (bad_component) *bad_component = -1;
  if (!stats || !mu_old || !Delta_old || !nu_old || !pi || !mu || !Sigma || !Delta || !nu)
    return ORC_EINVAL;
  if (n < 1 || p < 1 || q < 1 || g < 1 || p > 64 || q > 64) return ORC_EINVAL;
  if (!(nu_lo > 0.0) || !(nu_hi >= nu_lo)) return ORC_EINVAL;
  offs_t o = stat_offsets(p, q);
  for (int a = 0; a < g * o.S; ++a)
    if (!isfinite(stats[a])) return ORC_ENONFINITE;
  double s5[64 * 64], s6[64 * 64], s7[64 * 64], Ls5[64 * 64];
  double dmu[64], s3[64], s4[64], D[64 * 64], Sg[64 * 64], Ls[64 * 64];
  for (int i = 0; i < g; ++i) {
    const double* st = stats + (size_t)i * o.S;
    double s1 = st[o.s1], s2 = st[o.s2], s8 = st[o.s8];
    if (!(s1 > 0.0) || !(s2 > 0.0)) {
      if (bad_component) *bad_component = i;
      return ORC_ENOTPD;
    }
    for (int a = 0; a < p; ++a) s3[a] = st[o.s3 + a];
    for (int k = 0; k < q; ++k) s4[k] = st[o.s4 + k];
    for (int k = 0; k < q; ++k)
      for (int l = 0; l < q; ++l) s5[k * q + l] = st[o.s5 + tri_idx(k, l, q)];
    for (int a = 0; a < p; ++a)
      for (int k = 0; k < q; ++k) s6[a * q + k] = st[o.s6 + a * q + k];
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < p; ++b) s7[a * p + b] = st[o.s7 + tri_idx(a, b, p)];
    const double* Dold = Delta_old + (size_t)i * p * q;
    for (int a = 0; a < p; ++a) {
      double t = s3[a];
      for (int k = 0; k < q; ++k) t -= Dold[a * q + k] * s4[k];
      dmu[a] = t / s2;
    }
    double munew[64];
    for (int a = 0; a < p; ++a) munew[a] = mu_old[i * p + a] + dmu[a];
    for (int a = 0; a < p; ++a)
      for (int k = 0; k < q; ++k) s6[a * q + k] -= dmu[a] * s4[k];
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < p; ++b)
        s7[a * p + b] += -s3[a] * dmu[b] - dmu[a] * s3[b] + s2 * dmu[a] * dmu[b];
    if (fix_delta_zero) {
      for (int a = 0; a < p * q; ++a) D[a] = 0.0;
    } else {
      if (cholesky(s5, q, Ls5)) {
        if (bad_component) *bad_component = i;
        return ORC_ENOTPD;
      }
      /* Delta' = s6' s5^{-1}: row a of Delta' solves s5 x = (row a of s6')^T */
      double tmp[64], x[64];
      for (int a = 0; a < p; ++a) {
        fwd_solve(Ls5, q, s6 + a * q, tmp);
        bwd_solve(Ls5, q, tmp, x);
        for (int k = 0; k < q; ++k) D[a * q + k] = x[k];
      }
    }
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < p; ++b) {
        double t = s7[a * p + b];
        for (int k = 0; k < q; ++k) t -= D[a * q + k] * s6[b * q + k] + s6[a * q + k] * D[b * q + k];
        for (int k = 0; k < q; ++k)
          for (int l = 0; l < q; ++l) t += D[a * q + k] * s5[k * q + l] * D[b * q + l];
        Sg[a * p + b] = t / s1;
      }
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < a; ++b) {
        double t = 0.5 * (Sg[a * p + b] + Sg[b * p + a]);
        Sg[a * p + b] = t;
        Sg[b * p + a] = t;
      }
    /* a pivot of Sigma' at or below ORC_SIGMA_PIVOT_REL (sqrt(eps)) of its
     * diagonal entry: one coordinate is a linear function of the others
     * to about half the digits, Sigma' is numerically singular and the
     * component has degenerated (the likelihood is unbounded there) */
    if (cholesky_rel(Sg, p, Ls, ORC_SIGMA_PIVOT_REL)) {
      if (bad_component) *bad_component = i;
      return ORC_ENOTPD;
    }
    double vnew = nu_old[i];
    if (nu_mode != ORC_NU_FIXED) {
      double cst = s8 / s1;
      if (nu_equation(nu_hi, cst) >= 0.0) {
        vnew = nu_hi;
      } else if (nu_equation(nu_lo, cst) <= 0.0) {
        vnew = nu_lo;
      } else {
        double lo = nu_lo, hi = nu_hi;
        while (hi - lo > 1e-14 * lo) {
          double mid = 0.5 * (lo + hi);
          if (mid <= lo || mid >= hi) break;
          if (nu_equation(mid, cst) > 0.0)
            lo = mid;
          else
            hi = mid;
        }
        vnew = 0.5 * (lo + hi);
      }
    }
    pi[i] = s1 / (double)n;
    for (int a = 0; a < p; ++a) mu[i * p + a] = munew[a];
    for (int a = 0; a < p * q; ++a) Delta[(size_t)i * p * q + a] = D[a];
    for (int a = 0; a < p * p; ++a) Sigma[(size_t)i * p * p + a] = Sg[a];
    nu[i] = vnew;
  }
  /* pi sums to one up to rounding; renormalise so the next E-step's check holds */
  double ps = 0.0;
  for (int i = 0; i < g; ++i) ps += pi[i];
  for (int i = 0; i < g; ++i) pi[i] /= ps;
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* EM fit (Algorithms 2-4)                                                   */
/* ------------------------------------------------------------------------- */

/* Iteration t: E-step at Psi^(t) gives l^(t) (the log-likelihood of the
 * previous M-step's output); for t >= 2 Aitken's rule
 *   a = (l^(t) - l^(t-1)) / (l^(t-1) - l^(t-2)),
 *   l_inf = l^(t-1) + (l^(t) - l^(t-1)) / (1 - a)
 * stops when |l_inf - l^(t)| < tol, returning Psi^(t) and l^(t); otherwise
 * the M-step gives Psi^(t+1).  At most max_iter M-steps are taken;
 * loglik_trace holds l^(0..n_iter). */
double orc_aitken_linf(double l0, double l1, double l2) {
  double den = l1 - l0;
  double a = (den != 0.0) ? (l2 - l1) / den : 0.0;
  return l1 + (l2 - l1) / (1.0 - a);
}

int orc_em_fit(const double* y, int64_t n, int p, int q, int g, double* pi, double* mu,
               double* Sigma, double* Delta, double* nu, const double* u, int n_qmc, int nu_mode,
               int reorder, int fix_delta_zero, int max_iter, double tol, double nu_lo,
               double nu_hi, double* loglik_trace, int* n_iter, int* bad_component) {
  if (!loglik_trace || !n_iter || max_iter < 0) return ORC_EINVAL;
  if (n < 1) return ORC_EINVAL;
  offs_t o = stat_offsets(p, q);
  double* stats = (double*)malloc(sizeof(double) * g * o.S);
  if (!stats) return ORC_ENOMEM;
  int rc = ORC_OK;
  for (int t = 0;; ++t) {
    double ll;
    rc = orc_estep(y, n, p, q, g, pi, mu, Sigma, Delta, nu, u, n_qmc, nu_mode, reorder, NULL,
                   NULL, NULL, NULL, NULL, NULL, stats, &ll, bad_component);
    if (rc) break;
    loglik_trace[t] = ll;
    *n_iter = t;
    if (t >= 2) {
      double linf = orc_aitken_linf(loglik_trace[t - 2], loglik_trace[t - 1], loglik_trace[t]);
      if (fabs(linf - loglik_trace[t]) < tol) break;
    }
    if (t == max_iter) break;
    rc = orc_mstep(stats, n, p, q, g, mu, Delta, nu, nu_mode, fix_delta_zero, nu_lo, nu_hi, pi, mu,
                   Sigma, Delta, nu, bad_component);
    if (rc) break;
  }
  free(stats);
  return rc;
}
