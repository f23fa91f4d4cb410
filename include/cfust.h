/*
 * cfust.h -- C ABI of the MI355X (gfx950) library for the EM algorithm of
 * finite mixtures of canonical fundamental skew-t (CFUST) distributions
 * (Lee, McLachlan & Leemaqz, "Multi-Node EM Algorithm for Finite Mixture
 * Models": section 2 eq. (1)-(4); section 3, Algorithms 2-4).
 *
 * Conventions
 *  - Every array argument is a DEVICE pointer (HIP global memory) unless the
 *    comment says "host".  All arrays are C row-major float64:
 *      y[n][p]           observations
 *      pi[g]             mixing proportions (each > 0, sum 1 within 1e-12)
 *      mu[g][p]          locations
 *      Sigma[g][p][p]    scale matrices (symmetric positive definite)
 *      Delta[g][p][q]    skewness matrices
 *      nu[g]             degrees of freedom (> 0)
 *      u[n_qmc][q+1]     quasi-Monte Carlo points in the open unit interval;
 *                        column 0 drives the chi-square scale, column m the
 *                        m-th truncated-normal draw of the GHK estimator
 *  - The caller owns every buffer.  The library allocates only its internal
 *    workspace, stream-ordered on opts->stream, unless the caller passes one
 *    (opts->workspace, at least cfust_workspace_size() bytes).
 *  - Work is stream-ordered on opts->stream (a hipStream_t; NULL = the null
 *    stream).  Every entry point waits for its own work before returning, so
 *    that it can report errors found on the device.
 *  - Functions return CFUST_OK (0) or an error code; they never throw.
 *  - Limits: 1 <= p <= 32, 1 <= q <= 12, 1 <= g <= 16, n_qmc >= 1, n >= 0.
 *    For 9 <= q <= 12 the natural-order E-step, log-likelihood, M-step and
 *    EM fit exist (FP64 and FP32, with every nu_mode); the variable
 *    ordering, the surrogate, the batched form, the multistart fit and the
 *    GHK label batch return CFUST_EINVAL there.
 *
 * Sufficient statistics ("partial sums" of Algorithm 2) are stats[g][S] with
 * S = cfust_stats_size(p, q) = 3 + p + q + p q + p(p+1)/2 + q(q+1)/2, per
 * component, centred at the component's current mu:
 *   s1 | s2 | s3[p] | s4[q] | s5[q(q+1)/2] | s6[p][q] | s7[p(p+1)/2] | s8
 *   s1 = sum_j tau_ij              s2 = sum_j tau_ij e2_ij
 *   s3 = sum_j tau_ij e2_ij r_ij   s4 = sum_j tau_ij e3_ij
 *   s5 = sum_j tau_ij e4_ij        s6 = sum_j tau_ij r_ij e3_ij^T
 *   s7 = sum_j tau_ij e2_ij r_ij r_ij^T   s8 = sum_j tau_ij (e1_ij - e2_ij)
 * with r_ij = y_j - mu_i; symmetric matrices are packed as their upper
 * triangle, row by row.
 */
#ifndef CFUST_H
#define CFUST_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CFUST_OK 0
#define CFUST_EINVAL 1      /* bad size, NULL pointer, nu <= 0, pi off the simplex */
#define CFUST_ENOTPD 2      /* a Cholesky factorisation failed (bad_component set) */
#define CFUST_ENONFINITE 3  /* NaN or Inf in an input or a statistic */
#define CFUST_EHIP 4        /* a HIP runtime call failed */
#define CFUST_ENOMEM 5      /* workspace too small or allocation failed */

#define CFUST_FP64 0        /* GHK integrand in float64 */
#define CFUST_FP32 1        /* GHK integrand in float32, its weight and moment
                               sums in float64; everything else stays float64 */

#define CFUST_NU_OSL 0      /* nu update with the one-step-late E[log W | y] */
#define CFUST_NU_EXACT 1    /* nu update with the exact E[log W | y] = psi(a) - log b
                               + d/da log T_q(h_A sqrt(a'/a); R, 2a') at a' = a, the
                               derivative that of the GHK estimate itself on the same
                               points (a tangent carried through integral A: its
                               bounds, draws and chi-square scale); not with a
                               surrogate */
#define CFUST_NU_FIXED 2    /* nu held fixed */

typedef struct cfust_opts {
  int precision;          /* CFUST_FP64 or CFUST_FP32 */
  int nu_mode;            /* CFUST_NU_OSL, CFUST_NU_EXACT or CFUST_NU_FIXED */
  int fix_delta_zero;     /* nonzero: Delta held at 0 (t-mixture special case) */
  int max_iter;           /* cfust_em_fit: maximum number of M-steps */
  double tol;             /* cfust_em_fit: Aitken tolerance on |l_inf - l| */
  double nu_lo, nu_hi;    /* bracket of the nu root (defaults 1 and 200) */
  void* stream;           /* hipStream_t */
  void* workspace;        /* optional device workspace */
  size_t workspace_bytes;
  double* prof_ms;        /* optional host [CFUST_PROF_SLOTS]: HIP-event times (ms) of
                             the library's kernels on `stream` are ADDED here:
                             [0] precompute + chi tables, [1] pair kernel (the two
                             GHK integrals), [2] responsibilities + partial sums,
                             [3] M-step */
  int graph;              /* cfust_em_fit_batched: nonzero = capture one iteration in a
                             hipGraph and replay it (default 1) */
  int tile;               /* cfust_em_fit_batched: launch shape of the pair kernels,
                             0 = autotune, else 1 + index into the candidate table
                             (cfust_batched_shape); a shape with more waves per pair
                             than the batch allows is CFUST_EINVAL */
  struct cfust_surrogate* surrogate; /* optional trained surrogate network: when set,
                             cfust_estep / cfust_loglik / cfust_em_fit evaluate the two
                             GHK integrals of every in-range pair with it and the
                             GHK kernel only for the others (q must match) */
  int adapt_samples;      /* cfust_em_fit with a surrogate: pairs sampled for
                             cfust_surrogate_adapt before every surrogate E-step
                             (0 = no adaptation) */
  int adapt_epochs;       /* epochs of each of those adaptations */
  int reorder;            /* 1: every pair's GHK integrals take the variables in the
                             Genz-Bretz order (Genz & Bretz 2009, section 4.1.3) found
                             from that pair's bound h_A: at each step the variable with
                             the smallest standardised conditional bound goes next.
                             Changes only the QMC error, not the quantity estimated.
                             cfust_estep, cfust_loglik, cfust_loglik_rqmc, cfust_em_fit,
                             and cfust_em_fit_multistart after its burn-in; EINVAL with a
                             surrogate, in cfust_em_fit_batched and cfust_ghk_batch.
                             0 (default): natural order */
  int surrogate_check;    /* with a surrogate: m > 0 samples the observations
                             j_i = floor((2i+1) n / (2m)), i < m (the same ones every call),
                             evaluates their pairs with the GHK kernel as well, and corrects
                             the partial sums and the log-likelihood by (n/m) times the
                             sample's GHK-minus-network totals (a difference estimator;
                             m >= n gives the GHK E-step).  Per-pair outputs (tau, logf,
                             e1..e4) stay the network's.  The workspace then needs
                             cfust_workspace_size_opts bytes.  0 (default): no check */
  double surrogate_switch; /* cfust_em_fit with a surrogate: the surrogate phase also
                             ends (and the GHK phase begins) after an iteration that
                             changed l by less than surrogate_switch * |l|, the network's
                             relative accuracy on l: further surrogate iterations cannot
                             be told apart from its error.  0 (default): only Aitken's
                             rule ends the surrogate phase */
} cfust_opts;

#define CFUST_PROF_SLOTS 4

/* Outputs of cfust_estep.  Optional per-pair arrays may be NULL. */
typedef struct cfust_estep_out {
  double* tau;    /* [n][g]  posterior membership, eq. (4) (optional) */
  double* logf;   /* [n][g]  log(pi_i f_i(y_j)), eq. (2) (optional) */
  double* e1;     /* [n][g]  E[log W | y_j, component i] (one-step-late form) (optional) */
  double* e2;     /* [n][g]  E[W | ...] (optional) */
  double* e3;     /* [n][g][q]    E[W U | ...] (optional) */
  double* e4;     /* [n][g][q][q] E[W U U^T | ...] (optional) */
  double* stats;  /* [g][S]  partial sums (required) */
  double* loglik; /* [1]     log-likelihood eq. (3) at the input parameters (required) */
  int bad_component; /* host: component that failed, or -1 */
} cfust_estep_out;

/* Fills *opts with the defaults (FP64, OSL, max_iter 100, tol 1e-6, nu in [1,200]). */
void cfust_default_opts(cfust_opts* opts);

/* Number of statistics per component, S above. */
int cfust_stats_size(int p, int q);

/* Bytes of workspace for this problem size under these options (precision
 * and the surrogate check's sample); opts may be NULL (the defaults). */
int cfust_workspace_size_opts(int64_t n, int p, int q, int g, int n_qmc, const cfust_opts* opts,
                              size_t* bytes);

/* sizeof(cfust_opts) as compiled into the library (bindings check it). */
size_t cfust_opts_size(void);

/* Bytes of device workspace the entry points need for this problem size. */
int cfust_workspace_size(int64_t n, int p, int q, int g, int n_qmc, int precision,
                         size_t* bytes);

/* One E-step at Psi = (pi, mu, Sigma, Delta, nu) (section 3.2, Algorithm 2):
 * for every (observation, component) pair the CFUST log density (eq. (2))
 * with the q-variate t CDF T_q estimated by GHK over the points u, the
 * conditional expectations e1..e4 of the latent gamma and truncated-normal
 * variables (section 2), the posterior membership tau (eq. (4)), the
 * log-likelihood (eq. (3)) and the partial sums s1..s8. */
int cfust_estep(const double* y, int64_t n, int p, int q, int g, const double* pi,
                const double* mu, const double* Sigma, const double* Delta, const double* nu,
                const double* u, int n_qmc, const cfust_opts* opts, cfust_estep_out* out);

/* The E-step of cfust_estep for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, outputs and results as cfust_estep (the same
 * kernels in the same order, so the outputs are identical), but the
 * workspace is the library's static device scratch array of
 * CFUST_NOALLOC_SCRATCH_BYTES bytes: one copy per GPU, allocated when the
 * library's code is loaded on that GPU and held until the process ends.
 * The call allocates nothing.  Returns CFUST_ENOMEM when the problem needs
 * more workspace than that (cfust_workspace_size_opts gives the bytes), and
 * CFUST_EINVAL if opts sets a surrogate (its buffers grow on demand),
 * prof_ms (timing events) or a workspace of its own.  Every call on one GPU
 * uses that GPU's one scratch array: calls that overlap on one GPU (several
 * host threads, or streams that run concurrently) race and must be
 * serialised by the caller. */
#define CFUST_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int cfust_estep_noalloc(const double* y, int64_t n, int p, int q, int g, const double* pi,
                        const double* mu, const double* Sigma, const double* Delta,
                        const double* nu, const double* u, int n_qmc, const cfust_opts* opts,
                        cfust_estep_out* out);

/* One M-step from the partial sums (section 3.3, Algorithm 3): conditional
 * maximisation in the order mu (with the old Delta), Delta, Sigma, then nu
 * (root of 1 + log(nu/2) - psi(nu/2) + s8/s1 = 0 in [nu_lo, nu_hi], clipped)
 * and pi = s1 / n.  Outputs may alias the old parameters.
 * CFUST_ENOTPD (bad_component set) when a pivot of the new Sigma's Cholesky
 * factor is at or below 2^-26 (the square root of the FP64 epsilon) times
 * its diagonal entry: the component has degenerated.  CFUST_ENONFINITE when
 * a component's partial sums are not finite.
 * bad_component: host pointer or NULL. */
int cfust_mstep(const double* stats, int64_t n, int p, int q, int g, const double* mu_old,
                const double* Delta_old, const double* nu_old, const cfust_opts* opts,
                double* pi, double* mu, double* Sigma, double* Delta, double* nu,
                int* bad_component);

/* Log-likelihood eq. (3) at Psi (integral T_q of eq. (2) only).
 * loglik: device [1]; logf: device [n][g] or NULL. */
int cfust_loglik(const double* y, int64_t n, int p, int q, int g, const double* pi,
                 const double* mu, const double* Sigma, const double* Delta, const double* nu,
                 const double* u, int n_qmc, const cfust_opts* opts, double* loglik,
                 double* logf);

/* EM fit (Algorithms 2-4).  pi, mu, Sigma, Delta, nu hold Psi^(0) on entry
 * and the estimate on return.  Iteration t evaluates l^(t) at Psi^(t); for
 * t >= 2 it stops when the Aitken limit l_inf = l^(t-1) +
 * (l^(t) - l^(t-1)) / (1 - a), a = (l^(t) - l^(t-1)) / (l^(t-1) - l^(t-2)),
 * is within opts->tol of l^(t); otherwise the M-step gives Psi^(t+1).  At
 * most opts->max_iter M-steps.  loglik_trace: host [max_iter + 1], receives
 * l^(0..*n_iter).  n_iter, bad_component: host.
 * With opts->surrogate the fit runs in two phases: surrogate E-steps until
 * the rule above stops, then one GHK E-step at the same parameters (the GHK
 * log-likelihood at the surrogate's estimate; no M-step in between) and GHK
 * EM from there until the rule stops again, the Aitken test using only
 * values of the current phase (cfust_surrogate_em_switch gives the index of
 * the first GHK E-step).  With opts->adapt_samples > 0, every surrogate
 * E-step is preceded by cfust_surrogate_adapt at the current parameters
 * (opts->adapt_samples pairs, opts->adapt_epochs epochs, seed = iteration). */
int cfust_em_fit(const double* y, int64_t n, int p, int q, int g, double* pi, double* mu,
                 double* Sigma, double* Delta, double* nu, const double* u, int n_qmc,
                 const cfust_opts* opts, double* loglik_trace, int* n_iter,
                 int* bad_component);

/* Batched EM fit (section 3.1, Algorithm 1: many starts; sections 3.2-3.4
 * for each): n_problems independent problems with shared p, q and QMC points.
 * Problem k owns rows [off_k, off_k + n_obs[k]) of y (off_k = sum of the
 * previous n_obs) and components [c_k, c_k + g[k]) of pi, mu, Sigma, Delta
 * and nu (c_k = sum of the previous g); the parameter arrays hold Psi^(0) on
 * entry and each problem's estimate on return.  Each problem stops on its own
 * Aitken test, at opts->max_iter, or on an error (its status), while the
 * others continue.  The integrand runs in opts->precision; partial sums, the
 * M-step and the stopping rule in float64.  All iterations run on the device;
 * with opts->graph one iteration is captured as a hipGraph and replayed.
 * Host outputs: loglik_trace [n_problems][max_iter + 1] (NaN past n_iter),
 * n_iter [n_problems], status [n_problems] (CFUST_* codes).
 * Requires n_obs[k] >= 1, 1 <= g[k] <= 16, n_problems >= 1. */
int cfust_em_fit_batched(const double* y, int p, int q, int n_problems, const int64_t* n_obs,
                         const int* g, double* pi, double* mu, double* Sigma, double* Delta,
                         double* nu, const double* u, int n_qmc, const cfust_opts* opts,
                         double* loglik_trace, int* n_iter, int* status);

/* Randomised-QMC error bar of the log-likelihood eq. (3): l evaluated with
 * each of K point sets (u: device [K][n_qmc][q+1], e.g. one base sequence
 * under K independent random shifts); ll (host [K]) receives every value,
 * *mean and *std_err (host) their mean and standard error sd / sqrt(K)
 * (0 when K = 1). */
int cfust_loglik_rqmc(const double* y, int64_t n, int p, int q, int g, const double* pi,
                      const double* mu, const double* Sigma, const double* Delta, const double* nu,
                      const double* u, int n_qmc, int K, const cfust_opts* opts, double* ll,
                      double* mean, double* std_err);

/* Parallel initialisation (section 3.1, Algorithm 1, read with the largest
 * l selected) followed by the EM fit: m starting values Psi^(0)_k (device,
 * concatenated: pi0[m][g], mu0[m][g][p], Sigma0[m][g][p][p],
 * Delta0[m][g][p][q], nu0[m][g], e.g. from m initial partitions) are
 * evaluated together on the same data y[n][p] (through the batched kernels:
 * l^(0) and `burn_in` EM iterations per start, exactly that many unless a
 * start fails); the start with the largest l after its burn-in continues
 * with cfust_em_fit (opts->max_iter, opts->tol) into pi, mu, Sigma, Delta, nu
 * (device outputs [g]...).  The burn-in uses opts->nu_mode as the
 * continuation does, in the natural variable order.  start_loglik (host [m], may be NULL):
 * l of each start after its burn-in (NaN if the start failed); best (host):
 * the selected start; loglik_trace, n_iter, bad_component as cfust_em_fit.
 * Needs m copies of y in device memory. */
int cfust_em_fit_multistart(const double* y, int64_t n, int p, int q, int g, int m,
                            const double* pi0, const double* mu0, const double* Sigma0,
                            const double* Delta0, const double* nu0, const double* u, int n_qmc,
                            int burn_in, const cfust_opts* opts, double* pi, double* mu,
                            double* Sigma, double* Delta, double* nu, double* start_loglik,
                            int* best, double* loglik_trace, int* n_iter, int* bad_component);

/* Bytes of device workspace cfust_em_fit_batched needs. */
int cfust_batched_workspace_size(int p, int q, int n_problems, const int64_t* n_obs, const int* g,
                                 int n_qmc, int precision, int max_iter, size_t* bytes);

/* Launch shape chosen for the last cfust_em_fit_batched call (host outputs,
 * each may be NULL): waves per block, work items per work-queue fetch,
 * persistent waves per SIMD, waves per pair K (each of a pair's K waves
 * integrates N / K of its QMC points; the K partial sums are combined in a
 * fixed order), the QMC points per wave N / K, and the autotuner's timing of
 * that shape in ms (0 if not tuned).  Returns the number of candidate shapes.
 * The autotuner offers K > 1 only to batches of fewer than 65536 pairs, with
 * K a power of two, K <= 8 and K <= N / 256; the choice is cached per (q, N,
 * precision, largest K offered) for the life of the process.  Results depend
 * on K only through the order of the QMC sums (FP64: about 1e-13 relative);
 * pin the shape with opts.tile for results that are bitwise repeatable
 * across processes. */
int cfust_batched_config(int* waves_per_block, int* chunk, int* waves_per_simd,
                         int* waves_per_pair, int* points_per_wave, double* tuned_ms);

/* Candidate launch shape `index` (0-based; opts.tile = index + 1 selects it):
 * host outputs as in cfust_batched_config, each may be NULL.  Returns
 * CFUST_EINVAL for an index outside [0, number of candidates). */
int cfust_batched_shape(int index, int* waves_per_block, int* chunk, int* waves_per_simd,
                        int* waves_per_pair);

/* GHK estimates for M standardised problems (the integrals behind eq. (2) and
 * the truncated moments of section 2): for sample s, V ~ t_q(0, R_s, dof_s)
 * with R: device [M][q][q] correlation matrices (symmetric positive definite,
 * unit diagonal; only the lower triangle is read), bound h: device [M][q],
 * dof: device [M] (at most 4096 distinct values).  out: device
 * [M][1 + q + q(q+1)/2] = log P(V <= h) | E[V | V <= h] | E[V V^T | V <= h]
 * (upper triangle, row by row).  opts->precision selects the integrand type.
 * CFUST_ENOTPD if some R_s is not positive definite.  These are the labels
 * the surrogate network learns. */
int cfust_ghk_batch(int q, int64_t M, const double* h, const double* R, const double* dof,
                    const double* u, int n_qmc, const cfust_opts* opts, double* out);

/* ---------------------------------------------------------------------------
 * Surrogate network for the two GHK integrals of a pair.
 *
 * For pair (j, i) the integrals of eq. (2) and the truncated moments of
 * section 2 reduce to standardised problems P(V <= h), V ~ t_q(0, R_i, dof)
 * with R_i the correlation matrix of Lambda_i = I - Delta_i^T Omega_i^-1
 * Delta_i: integral A at dof nu_i + p, integral B at dof nu_i + p + 2.  A
 * feature row is  h[q] | r[q(q-1)/2] | dof  (r: entries of R above the
 * diagonal, row by row), F = q + q(q-1)/2 + 1 doubles; a target row is the
 * cfust_ghk_batch output, T = 1 + q + q(q+1)/2 doubles.  The network is a
 * perceptron F -> 256 -> 256 -> 256 -> T with SiLU activations, bf16 weights
 * and activations on the matrix cores, fp32 accumulation, fp32 master
 * weights, trained with Adam on a mean squared error of standardised outputs.
 * Internally it predicts log P | E[V] | U with Cov(V | V <= h) = U^T U (U
 * upper triangular, log diagonal), so every predicted covariance is
 * positive definite; inputs and outputs of the entry points are label rows.
 * A handle owns its device memory; calls that share a handle must not
 * overlap.  Limits: 1 <= q <= 8.
 * ------------------------------------------------------------------------- */
typedef struct cfust_surrogate cfust_surrogate;

#define CFUST_SURR_PARAMS 164672  /* fp32 parameters incl. zero padding */
#define CFUST_SURR_STD 256        /* standardisation: mean_x[64] | sd_x[64] | mean_y[64] | sd_y[64] */

/* Creates an untrained network for q with the training range
 * range[6] (host) = h_lo, h_hi (box for every h_m), dof_lo, dof_hi,
 * r_max (bound on |r|), eig_min (bound on the smallest eigenvalue of R):
 * the E-step uses the network only for pairs inside it, after lowering
 * every h_m above h_hi to h_hi (a coordinate bounded that high is nearly
 * untruncated: the t tail above 6 is below 1e-3 for dof >= 5).  Weights are drawn
 * from a seeded normal of variance 2 / fan_in, biases zero. */
int cfust_surrogate_create(int q, const double* range, unsigned long long seed,
                           cfust_surrogate** out);
void cfust_surrogate_destroy(cfust_surrogate* s);

/* Trains for `epochs` passes over M samples (feat: device [M][F], targ:
 * device [M][T]) in shuffled minibatches of `batch` rows (a multiple of 64,
 * at most 65536), learning rate cosine-annealed from lr0 to lr1, per-output
 * loss weights wo (host [T] or NULL for ones).  The first call sets the
 * standardisation from this data.  loss_trace: host [epochs] mean training
 * loss per epoch (or NULL). */
int cfust_surrogate_train(cfust_surrogate* s, const double* feat, const double* targ, int64_t M,
                          int epochs, int batch, double lr0, double lr1, unsigned long long seed,
                          const float* wo, const cfust_opts* opts, double* loss_trace);

/* One forward and backward pass over M <= 65536 samples without an update:
 * grad (host [CFUST_SURR_PARAMS]) = gradient of the loss, *loss (host).
 * Needs the standardisation (set by cfust_surrogate_train or _set_state). */
int cfust_surrogate_grad(cfust_surrogate* s, const double* feat, const double* targ, int64_t M,
                         const float* wo, const cfust_opts* opts, float* grad, double* loss);

/* Network outputs for M feature rows: out device [M][T] (de-standardised). */
int cfust_surrogate_eval(cfust_surrogate* s, const double* feat, int64_t M,
                         const cfust_opts* opts, double* out);

/* Host copies of the parameters ([CFUST_SURR_PARAMS] fp32) and of the
 * standardisation ([CFUST_SURR_STD] fp32); either pointer may be NULL. */
int cfust_surrogate_get_state(const cfust_surrogate* s, float* params, float* stdv);
int cfust_surrogate_set_state(cfust_surrogate* s, const float* params, const float* stdv);

/* File I/O of a handle (range, standardisation, parameters). */
int cfust_surrogate_save(const cfust_surrogate* s, const char* path);
int cfust_surrogate_load(const char* path, cfust_surrogate** out);

/* Fine-tunes the network for the E-step at Psi = (pi, mu, Sigma, Delta, nu):
 * `samples` pairs drawn uniformly (seeded) from the n*g pairs give their
 * two feature rows; rows inside the training range get GHK labels over the
 * points u (FP64, as cfust_ghk_batch) and the network trains `epochs`
 * passes over them (minibatches of 1024, learning rate 5e-4 cosine-annealed
 * to 1e-6, standardisation kept).  *loss (host, may be NULL) receives the
 * last epoch's mean loss, *rows (host, may be NULL) the rows trained on. */
int cfust_surrogate_adapt(cfust_surrogate* s, const double* y, int64_t n, int p, int q, int g,
                          const double* pi, const double* mu, const double* Sigma,
                          const double* Delta, const double* nu, const double* u, int n_qmc,
                          int64_t samples, int epochs, unsigned long long seed,
                          const cfust_opts* opts, double* loss, int64_t* rows);

/* Pairs the last E-step with this handle sent to the GHK kernel (outside the
 * training range). */
int64_t cfust_surrogate_fallback_count(const cfust_surrogate* s);

/* Index of the first GHK E-step in the trace of the last cfust_em_fit with
 * this handle (the switch from surrogate to GHK E-steps), -1 if the fit
 * stopped before switching. */
int cfust_surrogate_em_switch(const cfust_surrogate* s);

/* Raw feature rows of every pair at Psi: out device [n*g*2][F], row 2(j g + i)
 * for integral A and 2(j g + i) + 1 for integral B. */
int cfust_pair_features(const double* y, int64_t n, int p, int q, int g, const double* pi,
                        const double* mu, const double* Sigma, const double* Delta,
                        const double* nu, const cfust_opts* opts, double* out);

/* Test hook of the network's matrix-core product: C[M][N] (device fp32) =
 * op(A) op(B) with bf16 operands A, B (device, raw 16-bit patterns),
 * op(A)[m][k] = ta ? A[k][m] : A[m][k], op(B)[k][n] = tb ? B[n][k] : B[k][n]
 * (leading dimensions M or K and K or N).  M, N multiples of 64, K of 32. */
int cfust_mlp_gemm(int ta, int tb, int M, int N, int K, const unsigned short* A,
                   const unsigned short* B, float* C, void* stream);

/* Aitken-accelerated limit l_inf from l^(t-2), l^(t-1), l^(t) (Algorithm 4,
 * read with the denominator 1 - a). Host scalars. */
double cfust_aitken_linf(double l0, double l1, double l2);

/* Diagnostic: evaluates a device special function elementwise on x[n]
 * (device), writing out[n] (device).  fn: 0 Phi, 1 log Phi, 2 Phi^-1,
 * 3 Phi^-1 from log p, 4 chi-square quantile at (x, x2 = dof), 5 digamma,
 * 6 trigamma, 7 Phi in float32, 8 Phi^-1 in float32, 9 log, 10 sqrt,
 * 11 d/d(dof) of the chi-square quantile at (x, x2 = dof), 12 phi(x)/Phi(x),
 * 13 phi(x)/Phi(x) in float32; the per-call cost probes of the GHK point
 * loop (section 2): 14 one coordinate step Phi^-1(u Phi(x)) with u = x2,
 * 15 the same in float32, 16 the accumulation of the weight x 2^x2 into a
 * running sum and reference exponent taken from element i ^ 1 (out[i] =
 * the new sum), 17 the same with a float32 weight.  x2 may be NULL unless
 * fn is 4, 11 or 14..17. */
int cfust_eval_special(int fn, const double* x, const double* x2, double* out, int64_t n,
                       void* stream);

const char* cfust_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
