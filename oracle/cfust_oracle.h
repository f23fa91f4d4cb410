/*
 * cfust_oracle.h -- plain FP64 CPU oracle for the CFUST mixture EM.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this library; the GPU product path never
 * does.  It shares no code with the GPU library.
 *
 * All arrays are host memory, C row-major, float64:
 *   y[n][p]; pi[g]; mu[g][p]; Sigma[g][p][p]; Delta[g][p][q]; nu[g];
 *   u[n_qmc][q+1] quasi-Monte Carlo points in (0,1).
 * Sufficient statistics stats[g][S], S = 3 + p + q + p*q + p(p+1)/2 + q(q+1)/2,
 * per component in the order
 *   s1 | s2 | s3[p] | s4[q] | s5[q(q+1)/2] | s6[p][q] | s7[p(p+1)/2] | s8
 * with symmetric matrices packed as their upper triangle, row by row.
 */
#ifndef CFUST_ORACLE_H
#define CFUST_ORACLE_H
#include <stdint.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOTPD 2
#define ORC_ENONFINITE 3
#define ORC_ENOMEM 5

#define ORC_NU_OSL 0
#define ORC_NU_EXACT_FD 1   /* e1 = E[log W | y] with a central difference in a */
#define ORC_FD_REL 1e-3     /* relative step of that difference */
#define ORC_NU_FIXED 2
#define ORC_R_PIVOT_MIN 1e-10 /* smallest accepted pivot of chol(R) (R: unit diagonal) */
#define ORC_SIGMA_PIVOT_REL 0x1p-26 /* smallest accepted pivot of chol(Sigma'), relative to
                                       its diagonal entry: sqrt of the FP64 epsilon */
#define ORC_NU_EXACT 3      /* e1 = E[log W | y] with the derivative of the estimate itself */

#ifdef __cplusplus
extern "C" {
#endif

/* special functions (exported for the pin tests) */
double orc_norm_cdf(double x);
double orc_log_norm_cdf(double x);
double orc_norm_quantile(double p);
double orc_norm_quantile_log(double log_p);
double orc_digamma(double x);
double orc_gamma_p(double a, double x);
double orc_gamma_q(double a, double x);
double orc_chi2_quantile(double u, double dof);
double orc_chi2_quantile_ddof(double u, double dof);

/* GHK estimate of P(V <= h) for V ~ t_q(0, R, dof), R = C C^T (C lower,
 * q*q row-major, positive diagonal).  s[k] = sqrt(chi2_quantile(u[k][0],dof)/dof).
 * moments != 0 also returns EV[q] = E[V | V <= h] and EVV[q*q] = E[V V^T | V <= h]. */
int orc_ghk(int q, const double* h, const double* C, double dof, const double* u,
            int n_qmc, int moments, double* logT, double* EV, double* EVV);

/* Genz-Bretz variable ordering of P(Z <= h), Z ~ N(0, R), R with unit
 * diagonal: perm[i] = variable placed at step i, Cp = chol(R[perm][perm]). */
int orc_genz_order(int q, const double* h, const double* R, int* perm, double* Cp);

/* log T = log P(V <= h), V ~ t_q(0, C C^T, 2a), by orc_ghk without moments,
 * and d/da' log of the same estimate with bound h sqrt(a'/a) and dof 2a', at
 * a' = a, on the same points (the derivative of the estimate itself). */
int orc_ghk_tangent(int q, const double* h, const double* C, double a, const double* u,
                    int n_qmc, double* logT, double* dlogT);

/* orc_ghk with the variables in the Genz-Bretz order found from h and R
 * (R a correlation matrix); moments in the original labelling; perm[q]
 * returns the order. */
int orc_ghk_ordered(int q, const double* h, const double* R, double dof, const double* u,
                    int n_qmc, int moments, double* logT, double* EV, double* EVV, int* perm);

/* reorder != 0: every pair's integrals take the variables in the Genz-Bretz
 * order found from that pair's bound h_A (orc_genz_order). */
int orc_estep(const double* y, int64_t n, int p, int q, int g, const double* pi,
              const double* mu, const double* Sigma, const double* Delta, const double* nu,
              const double* u, int n_qmc, int nu_mode, int reorder,
              double* tau, double* logf, double* e1, double* e2, double* e3, double* e4,
              double* stats, double* loglik, int* bad_component);

int orc_mstep(const double* stats, int64_t n, int p, int q, int g, const double* mu_old,
              const double* Delta_old, const double* nu_old, int nu_mode, int fix_delta_zero,
              double nu_lo, double nu_hi, double* pi, double* mu, double* Sigma, double* Delta,
              double* nu, int* bad_component);

int orc_loglik(const double* y, int64_t n, int p, int q, int g, const double* pi,
               const double* mu, const double* Sigma, const double* Delta, const double* nu,
               const double* u, int n_qmc, int reorder, double* loglik, double* logf);

int orc_em_fit(const double* y, int64_t n, int p, int q, int g, double* pi, double* mu,
               double* Sigma, double* Delta, double* nu, const double* u, int n_qmc,
               int nu_mode, int reorder, int fix_delta_zero, int max_iter, double tol, double nu_lo,
               double nu_hi, double* loglik_trace, int* n_iter, int* bad_component);

int orc_stats_size(int p, int q);

/* Aitken-accelerated limit l_inf from three successive log-likelihoods. */
double orc_aitken_linf(double l0, double l1, double l2);

#ifdef __cplusplus
}
#endif
#endif
