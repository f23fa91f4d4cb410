// C ABI of the CFUST mixture EM library (see include/cfust.h).
//
// Host side only: argument checks, workspace planning, kernel launches on the
// caller's stream, and the EM driver loop with Aitken's stopping rule
// (section 3.4, Algorithm 4).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include "../../include/cfust.h"
#include "cfust_kernels.hpp"

using namespace cfust;

namespace {

struct Plan {
  int64_t n;
  int p, q, g, N, prec;
  int W, S, GS, stride;
  int tile, nb, ny;
  int64_t per_block;
  size_t lds_bytes;
  // byte offsets inside the workspace
  size_t o_status, o_comp, o_uT, o_ubT, o_sA, o_sB, o_rsB, o_pair, o_part, o_pll, o_pitmp,
      o_ll, o_stats, total;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

Plan make_plan(int64_t n, int p, int q, int g, int N, int prec) {
  Plan pl;
  pl.n = n;
  pl.p = p;
  pl.q = q;
  pl.g = g;
  pl.N = N;
  pl.prec = prec;
  pl.W = pair_width(q);
  StatLayout sl(p, q);
  pl.S = sl.S;
  pl.GS = g * sl.S;
  pl.stride = CompLayout(p, q).stride;
  size_t per_obs = (size_t)(g * pl.W + g + p + 1) * sizeof(double);
  int tile = (int)((48 * 1024) / per_obs);
  pl.tile = tile < 1 ? 1 : (tile > 16 ? 16 : tile);
  int64_t per = (n + 1023) / 1024;
  if (per < pl.tile) per = pl.tile;
  per = ((per + pl.tile - 1) / pl.tile) * pl.tile;
  pl.per_block = per;
  pl.nb = (int)((n + per - 1) / per);
  if (pl.nb < 1) pl.nb = 1;
  pl.ny = (pl.GS + kStatsPerBlock - 1) / kStatsPerBlock;
  pl.lds_bytes = per_obs * pl.tile;
  size_t es = prec == CFUST_FP32 ? sizeof(float) : sizeof(double);
  size_t off = 0;
  pl.o_status = off;
  off = align_up(off + 4 * sizeof(int));
  pl.o_comp = off;
  off = align_up(off + (size_t)g * pl.stride * sizeof(double));
  pl.o_uT = off;
  off = align_up(off + (size_t)(q + 1) * N * es);
  pl.o_ubT = off;
  off = align_up(off + (size_t)(q + 1) * N * es);
  pl.o_sA = off;
  off = align_up(off + (size_t)g * N * es);
  pl.o_sB = off;
  off = align_up(off + (size_t)g * N * es);
  pl.o_rsB = off;
  off = align_up(off + (size_t)g * N * es);
  pl.o_pair = off;
  off = align_up(off + (size_t)(n > 0 ? n : 1) * g * pl.W * sizeof(double));
  pl.o_part = off;
  off = align_up(off + (size_t)pl.nb * pl.GS * sizeof(double));
  pl.o_pll = off;
  off = align_up(off + (size_t)pl.nb * sizeof(double));
  pl.o_pitmp = off;
  off = align_up(off + (size_t)g * sizeof(double));
  pl.o_ll = off;
  off = align_up(off + sizeof(double));
  pl.o_stats = off;
  off = align_up(off + (size_t)pl.GS * sizeof(double));
  pl.total = off;
  return pl;
}

struct Ws {
  char* base = nullptr;
  bool owned = false;
  hipStream_t st = nullptr;
  double* prof = nullptr;             // host accumulator, CFUST_PROF_SLOTS entries
  hipEvent_t ev[2 * CFUST_PROF_SLOTS] = {};
  bool ev_pending[CFUST_PROF_SLOTS] = {};
  template <typename X>
  X* at(size_t off) const {
    return reinterpret_cast<X*>(base + off);
  }
};

int check_dims(int64_t n, int p, int q, int g, int N) {
  if (n < 0 || p < 1 || p > kMaxP || q < 1 || q > kMaxQ || g < 1 || g > kMaxG || N < 1)
    return CFUST_EINVAL;
  return CFUST_OK;
}

// HIP-event brackets around one kernel group (only when the caller asked for
// timings); elapsed times are collected after the call's final synchronise.
void prof_begin(Ws& ws, int slot) {
  if (!ws.prof) return;
  hipEventRecord(ws.ev[2 * slot], ws.st);
}
void prof_end(Ws& ws, int slot) {
  if (!ws.prof) return;
  hipEventRecord(ws.ev[2 * slot + 1], ws.st);
  ws.ev_pending[slot] = true;
}
// called after a stream synchronise
void prof_collect(Ws& ws) {
  if (!ws.prof) return;
  for (int s = 0; s < CFUST_PROF_SLOTS; ++s) {
    if (!ws.ev_pending[s]) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ws.ev[2 * s], ws.ev[2 * s + 1]) == hipSuccess) ws.prof[s] += ms;
    ws.ev_pending[s] = false;
  }
}

int acquire(const Plan& pl, const cfust_opts* o, Ws* ws) {
  ws->st = o ? (hipStream_t)o->stream : nullptr;
  ws->prof = o ? o->prof_ms : nullptr;
  if (ws->prof)
    for (int e = 0; e < 2 * CFUST_PROF_SLOTS; ++e)
      if (hipEventCreate(&ws->ev[e]) != hipSuccess) return CFUST_EHIP;
  if (o && o->workspace) {
    if (o->workspace_bytes < pl.total) return CFUST_ENOMEM;
    ws->base = (char*)o->workspace;
    ws->owned = false;
    return CFUST_OK;
  }
  void* ptr = nullptr;
  if (hipMallocAsync(&ptr, pl.total, ws->st) != hipSuccess) return CFUST_ENOMEM;
  ws->base = (char*)ptr;
  ws->owned = true;
  return CFUST_OK;
}

void release(Ws* ws) {
  if (ws->owned && ws->base) (void)hipFreeAsync(ws->base, ws->st);
  ws->base = nullptr;
  if (ws->prof)
    for (int e = 0; e < 2 * CFUST_PROF_SLOTS; ++e)
      if (ws->ev[e]) (void)hipEventDestroy(ws->ev[e]);
  ws->prof = nullptr;
}

int hip_ok(hipError_t e) { return e == hipSuccess ? CFUST_OK : CFUST_EHIP; }

int launch_check() { return hip_ok(hipGetLastError()); }

void clear_status(const Ws& ws, const Plan& pl) {
  fill_int_kernel<<<1, 64, 0, ws.st>>>(ws.at<int>(pl.o_status), 4, 0);
}

int fetch_status(Ws& ws, const Plan& pl, int* bad) {
  int h[4] = {0, -1, 0, 0};
  if (hipMemcpyAsync(h, ws.at<int>(pl.o_status), 2 * sizeof(int), hipMemcpyDeviceToHost, ws.st) !=
      hipSuccess)
    return CFUST_EHIP;
  if (hipStreamSynchronize(ws.st) != hipSuccess) return CFUST_EHIP;
  prof_collect(ws);
  if (bad) *bad = h[0] ? h[1] : -1;
  switch (h[0]) {
    case kOk: return CFUST_OK;
    case kEInval: return CFUST_EINVAL;
    case kENotPD: return CFUST_ENOTPD;
    case kENonFinite: return CFUST_ENONFINITE;
    default: return CFUST_EHIP;
  }
}

// per-call parameter preparation: component blocks and chi scale tables
template <typename T>
void launch_prepare(const Ws& ws, const Plan& pl, const double* pi, const double* mu,
                    const double* Sigma, const double* Delta, const double* nu, const double* u,
                    bool points) {
  precompute_kernel<<<1, 64, 0, ws.st>>>(pl.p, pl.q, pl.g, pi, Sigma, Delta, mu, nu,
                                         ws.at<double>(pl.o_comp), ws.at<int>(pl.o_status));
  const int q1 = pl.q + 1;
  if (points) {
    int64_t tot = (int64_t)pl.N * q1;
    points_kernel<T><<<(unsigned)((tot + 255) / 256), 256, 0, ws.st>>>(
        u, pl.N, q1, ws.at<T>(pl.o_uT), ws.at<T>(pl.o_ubT), ws.at<int>(pl.o_status));
  }
  int64_t tot = (int64_t)2 * pl.g * pl.N;
  chi_kernel<T><<<(unsigned)((tot + 127) / 128), 128, 0, ws.st>>>(
      ws.at<double>(pl.o_comp), pl.stride, CompLayout(pl.p, pl.q).nu, pl.p, pl.g, u, pl.N, q1,
      ws.at<T>(pl.o_sA), ws.at<T>(pl.o_sB), ws.at<T>(pl.o_rsB), ws.at<int>(pl.o_status));
}

template <typename T, int Q, bool MOM>
void launch_pairs_q(const Ws& ws, const Plan& pl, const double* y, const double* mu) {
  int64_t pairs = pl.n * pl.g;
  if (pairs == 0) return;
  unsigned blocks = (unsigned)((pairs + 3) / 4);
  pair_kernel<T, Q, MOM><<<blocks, 256, 0, ws.st>>>(
      y, pl.n, pl.p, pl.g, mu, ws.at<double>(pl.o_comp), ws.at<T>(pl.o_sA), ws.at<T>(pl.o_sB),
      ws.at<T>(pl.o_rsB), ws.at<T>(pl.o_uT), ws.at<T>(pl.o_ubT), pl.N, ws.at<double>(pl.o_pair),
      pl.W, ws.at<int>(pl.o_status));
}

template <typename T, bool MOM>
void launch_pairs(const Ws& ws, const Plan& pl, const double* y, const double* mu) {
  switch (pl.q) {
    case 1: launch_pairs_q<T, 1, MOM>(ws, pl, y, mu); break;
    case 2: launch_pairs_q<T, 2, MOM>(ws, pl, y, mu); break;
    case 3: launch_pairs_q<T, 3, MOM>(ws, pl, y, mu); break;
    case 4: launch_pairs_q<T, 4, MOM>(ws, pl, y, mu); break;
    case 5: launch_pairs_q<T, 5, MOM>(ws, pl, y, mu); break;
    case 6: launch_pairs_q<T, 6, MOM>(ws, pl, y, mu); break;
    case 7: launch_pairs_q<T, 7, MOM>(ws, pl, y, mu); break;
    case 8: launch_pairs_q<T, 8, MOM>(ws, pl, y, mu); break;
  }
}

void launch_stats(const Ws& ws, const Plan& pl, const double* y, const double* mu, bool with_stats,
                  double* stats, double* loglik, const cfust_estep_out* out, double* logf_only) {
  dim3 grid(pl.nb, with_stats ? pl.ny : 1);
  stats_kernel<<<grid, 256, pl.lds_bytes, ws.st>>>(
      y, pl.n, pl.p, pl.q, pl.g, mu, ws.at<double>(pl.o_pair), pl.W, pl.per_block, pl.tile,
      with_stats ? 1 : 0, ws.at<double>(pl.o_part), ws.at<double>(pl.o_pll),
      out ? out->tau : nullptr, out ? out->logf : logf_only, out ? out->e1 : nullptr,
      out ? out->e2 : nullptr, out ? out->e3 : nullptr, out ? out->e4 : nullptr,
      ws.at<int>(pl.o_status));
  reduce_kernel<<<pl.GS + 1, 64, 0, ws.st>>>(
      ws.at<double>(pl.o_part), ws.at<double>(pl.o_pll), pl.nb, pl.GS,
      with_stats ? stats : nullptr, loglik, ws.at<int>(pl.o_status));
}

template <typename T>
void run_estep(Ws& ws, const Plan& pl, const double* y, const double* pi, const double* mu,
               const double* Sigma, const double* Delta, const double* nu, const double* u,
               bool points, bool moments, double* stats, double* loglik,
               const cfust_estep_out* out, double* logf_only) {
  prof_begin(ws, 0);
  launch_prepare<T>(ws, pl, pi, mu, Sigma, Delta, nu, u, points);
  prof_end(ws, 0);
  prof_begin(ws, 1);
  if (moments)
    launch_pairs<T, true>(ws, pl, y, mu);
  else
    launch_pairs<T, false>(ws, pl, y, mu);
  prof_end(ws, 1);
  prof_begin(ws, 2);
  launch_stats(ws, pl, y, mu, moments, stats, loglik, out, logf_only);
  prof_end(ws, 2);
}

void run_mstep(Ws& ws, const Plan& pl, int64_t n, const double* stats, const double* mu_old,
               const double* Delta_old, const double* nu_old, const cfust_opts* o, double* pi,
               double* mu, double* Sigma, double* Delta, double* nu) {
  double lo = 1.0, hi = 200.0;
  int fixed = 0, fixd = 0;
  if (o) {
    lo = o->nu_lo;
    hi = o->nu_hi;
    fixed = o->nu_mode == CFUST_NU_FIXED;
    fixd = o->fix_delta_zero != 0;
  }
  prof_begin(ws, 3);
  mstep_kernel<<<1, 64, 0, ws.st>>>(stats, n, pl.p, pl.q, pl.g, mu_old, Delta_old, nu_old,
                                    fixed, fixd, lo, hi, pi, mu, Sigma, Delta, nu,
                                    ws.at<double>(pl.o_pitmp), ws.at<int>(pl.o_status));
  prof_end(ws, 3);
}

int check_opts(const cfust_opts* o) {
  if (!o) return CFUST_OK;
  if (o->precision != CFUST_FP64 && o->precision != CFUST_FP32) return CFUST_EINVAL;
  if (o->nu_mode != CFUST_NU_OSL && o->nu_mode != CFUST_NU_FIXED) return CFUST_EINVAL;
  if (!(o->nu_lo > 0.0) || !(o->nu_hi >= o->nu_lo)) return CFUST_EINVAL;
  return CFUST_OK;
}

}  // namespace

extern "C" {

void cfust_default_opts(cfust_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->precision = CFUST_FP64;
  o->nu_mode = CFUST_NU_OSL;
  o->max_iter = 100;
  o->tol = 1e-6;
  o->nu_lo = 1.0;
  o->nu_hi = 200.0;
}

int cfust_stats_size(int p, int q) { return StatLayout(p, q).S; }

int cfust_workspace_size(int64_t n, int p, int q, int g, int n_qmc, int precision, size_t* bytes) {
  if (!bytes) return CFUST_EINVAL;
  int rc = check_dims(n, p, q, g, n_qmc);
  if (rc) return rc;
  if (precision != CFUST_FP64 && precision != CFUST_FP32) return CFUST_EINVAL;
  *bytes = make_plan(n, p, q, g, n_qmc, precision).total;
  return CFUST_OK;
}

double cfust_aitken_linf(double l0, double l1, double l2) {
  double den = l1 - l0;
  double a = den != 0.0 ? (l2 - l1) / den : 0.0;
  return l1 + (l2 - l1) / (1.0 - a);
}

int cfust_estep(const double* y, int64_t n, int p, int q, int g, const double* pi,
                const double* mu, const double* Sigma, const double* Delta, const double* nu,
                const double* u, int n_qmc, const cfust_opts* o, cfust_estep_out* out) {
  if (!out) return CFUST_EINVAL;
  out->bad_component = -1;
  int rc = check_dims(n, p, q, g, n_qmc);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  if ((n > 0 && !y) || !pi || !mu || !Sigma || !Delta || !nu || !u || !out->stats || !out->loglik)
    return CFUST_EINVAL;
  const int prec = o ? o->precision : CFUST_FP64;
  Plan pl = make_plan(n, p, q, g, n_qmc, prec);
  Ws ws;
  if ((rc = acquire(pl, o, &ws))) return rc;
  clear_status(ws, pl);
  if (prec == CFUST_FP32)
    run_estep<float>(ws, pl, y, pi, mu, Sigma, Delta, nu, u, true, true, out->stats, out->loglik,
                     out, nullptr);
  else
    run_estep<double>(ws, pl, y, pi, mu, Sigma, Delta, nu, u, true, true, out->stats, out->loglik,
                      out, nullptr);
  rc = launch_check();
  int st = fetch_status(ws, pl, &out->bad_component);
  release(&ws);
  return rc ? rc : st;
}

int cfust_loglik(const double* y, int64_t n, int p, int q, int g, const double* pi,
                 const double* mu, const double* Sigma, const double* Delta, const double* nu,
                 const double* u, int n_qmc, const cfust_opts* o, double* loglik, double* logf) {
  int rc = check_dims(n, p, q, g, n_qmc);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  if ((n > 0 && !y) || !pi || !mu || !Sigma || !Delta || !nu || !u || !loglik) return CFUST_EINVAL;
  const int prec = o ? o->precision : CFUST_FP64;
  Plan pl = make_plan(n, p, q, g, n_qmc, prec);
  Ws ws;
  if ((rc = acquire(pl, o, &ws))) return rc;
  clear_status(ws, pl);
  if (prec == CFUST_FP32)
    run_estep<float>(ws, pl, y, pi, mu, Sigma, Delta, nu, u, true, false, nullptr, loglik,
                     nullptr, logf);
  else
    run_estep<double>(ws, pl, y, pi, mu, Sigma, Delta, nu, u, true, false, nullptr, loglik,
                      nullptr, logf);
  rc = launch_check();
  int st = fetch_status(ws, pl, nullptr);
  release(&ws);
  return rc ? rc : st;
}

int cfust_mstep(const double* stats, int64_t n, int p, int q, int g, const double* mu_old,
                const double* Delta_old, const double* nu_old, const cfust_opts* o, double* pi,
                double* mu, double* Sigma, double* Delta, double* nu, int* bad_component) {
  if (bad_component) *bad_component = -1;
  int rc = check_dims(n, p, q, g, 1);
  if (rc) return rc;
  if (n < 1) return CFUST_EINVAL;
  if ((rc = check_opts(o))) return rc;
  if (!stats || !mu_old || !Delta_old || !nu_old || !pi || !mu || !Sigma || !Delta || !nu)
    return CFUST_EINVAL;
  // the M-step needs only the status word and g scratch doubles
  Plan pl = make_plan(0, p, q, g, 1, CFUST_FP64);
  Ws ws;
  if ((rc = acquire(pl, o, &ws))) return rc;
  clear_status(ws, pl);
  run_mstep(ws, pl, n, stats, mu_old, Delta_old, nu_old, o, pi, mu, Sigma, Delta, nu);
  rc = launch_check();
  int st = fetch_status(ws, pl, bad_component);
  release(&ws);
  return rc ? rc : st;
}

int cfust_em_fit(const double* y, int64_t n, int p, int q, int g, double* pi, double* mu,
                 double* Sigma, double* Delta, double* nu, const double* u, int n_qmc,
                 const cfust_opts* o, double* loglik_trace, int* n_iter, int* bad_component) {
  if (bad_component) *bad_component = -1;
  int rc = check_dims(n, p, q, g, n_qmc);
  if (rc) return rc;
  if (n < 1) return CFUST_EINVAL;
  if ((rc = check_opts(o))) return rc;
  if (!y || !pi || !mu || !Sigma || !Delta || !nu || !u || !loglik_trace || !n_iter)
    return CFUST_EINVAL;
  cfust_opts def;
  cfust_default_opts(&def);
  if (!o) o = &def;
  if (o->max_iter < 0) return CFUST_EINVAL;
  Plan pl = make_plan(n, p, q, g, n_qmc, o->precision);
  Ws ws;
  if ((rc = acquire(pl, o, &ws))) return rc;
  double* stats = ws.at<double>(pl.o_stats);
  double* ll_dev = ws.at<double>(pl.o_ll);
  clear_status(ws, pl);
  *n_iter = 0;
  int result = CFUST_OK;
  for (int t = 0;; ++t) {
    const bool last = t == o->max_iter;
    if (o->precision == CFUST_FP32)
      run_estep<float>(ws, pl, y, pi, mu, Sigma, Delta, nu, u, t == 0, !last, stats, ll_dev,
                       nullptr, nullptr);
    else
      run_estep<double>(ws, pl, y, pi, mu, Sigma, Delta, nu, u, t == 0, !last, stats, ll_dev,
                        nullptr, nullptr);
    if ((result = launch_check())) break;
    double ll = 0.0;
    if (hipMemcpyAsync(&ll, ll_dev, sizeof(double), hipMemcpyDeviceToHost, ws.st) != hipSuccess) {
      result = CFUST_EHIP;
      break;
    }
    if ((result = fetch_status(ws, pl, bad_component))) break;
    loglik_trace[t] = ll;
    *n_iter = t;
    if (t >= 2) {
      double linf = cfust_aitken_linf(loglik_trace[t - 2], loglik_trace[t - 1], ll);
      if (fabs(linf - ll) < o->tol) break;
    }
    if (last) break;
    run_mstep(ws, pl, n, stats, mu, Delta, nu, o, pi, mu, Sigma, Delta, nu);
  }
  if (result == CFUST_OK) {
    int st = fetch_status(ws, pl, bad_component);
    result = st;
  }
  release(&ws);
  return result;
}

int cfust_eval_special(int fn, const double* x, const double* x2, double* out, int64_t n,
                       void* stream) {
  if (!x || !out || n < 0 || fn < 0 || fn > 10 || (fn == 4 && !x2)) return CFUST_EINVAL;
  if (n == 0) return CFUST_OK;
  hipStream_t st = (hipStream_t)stream;
  special_kernel<<<(unsigned)((n + 127) / 128), 128, 0, st>>>(fn, x, x2, out, n);
  if (hipGetLastError() != hipSuccess) return CFUST_EHIP;
  return hipStreamSynchronize(st) == hipSuccess ? CFUST_OK : CFUST_EHIP;
}

const char* cfust_strerror(int code) {
  switch (code) {
    case CFUST_OK: return "ok";
    case CFUST_EINVAL: return "invalid argument";
    case CFUST_ENOTPD: return "matrix not positive definite";
    case CFUST_ENONFINITE: return "non-finite value";
    case CFUST_EHIP: return "HIP runtime error";
    case CFUST_ENOMEM: return "out of memory or workspace too small";
    default: return "unknown error";
  }
}

}  // extern "C"
