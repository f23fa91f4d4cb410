// C ABI of the CFUST mixture EM library (see include/cfust.h): the
// single-problem E-step, log-likelihood and M-step, and the EM driver loop
// with Aitken's stopping rule (section 3.4, Algorithm 4), plus the host
// helpers the other translation units share (cfust_host.hpp).
//
// Host side only: argument checks, workspace planning and kernel launches on
// the caller's stream.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "../../include/cfust.h"
#include "cfust_host.hpp"
#include "cfust_kernels.hpp"
#include "cfust_surrogate.hpp"

using namespace cfust;
using namespace cfust::host;

namespace {

// observations per statistics block for n observations (a multiple of tile)
int64_t stats_per_block(int64_t n, int tile) {
  int64_t per = (n + 1023) / 1024;
  if (per < tile) per = tile;
  return ((per + tile - 1) / tile) * tile;
}

// A launch of fewer than kSplitWaves pairs spreads each pair's points over
// up to kSplitMax waves (each wave keeps at least 4 points per lane).  The
// batched form keeps one wave per pair (its problems fill the chip
// together), so a single-problem call sums in the batched form's order only
// where it does not split: N < 512 or at least kSplitWaves pairs.
constexpr int64_t kSplitWaves = 4096;
constexpr int kSplitMax = 16;

int split_of(int64_t pairs, int N) {
  if (pairs < 1 || pairs >= kSplitWaves) return 1;
  int64_t K = (kSplitWaves + pairs - 1) / pairs;
  K = std::min<int64_t>(K, kSplitMax);
  K = std::min<int64_t>(K, N / 256);
  return K >= 2 ? (int)K : 1;
}

int hip_ok(hipError_t e) { return e == hipSuccess ? CFUST_OK : CFUST_EHIP; }

// HIP-event brackets around one kernel group (only when the caller asked for
// timings); elapsed times are collected after the call's final synchronise.
void prof_begin(Ws& ws, int slot) {
  if (!ws.prof) return;
  (void)hipEventRecord(ws.ev[2 * slot], ws.st);
}
void prof_end(Ws& ws, int slot) {
  if (!ws.prof) return;
  (void)hipEventRecord(ws.ev[2 * slot + 1], ws.st);
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

}  // namespace

namespace cfust {
namespace host {

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

Plan make_plan(int64_t n, int p, int q, int g, int N, int prec, int64_t check_m) {
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
  size_t per_obs = (size_t)stats_lds_per_obs(p, g, pl.W) * sizeof(double);
  int tile = (int)((48 * 1024) / per_obs);
  pl.tile = tile < 1 ? 1 : (tile > 16 ? 16 : tile);
  const int64_t per = stats_per_block(n, pl.tile);
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
  pl.o_tA = off;
  off = align_up(off + (size_t)g * N * es);
  pl.o_pair = off;
  off = align_up(off + (size_t)(n > 0 ? n : 1) * g * pl.W * sizeof(double));
  pl.split = split_of(n * g, N);
  if (pl.split > 1) {
    // widest record: A with its tangent, B with moments
    const size_t pw = 3 + 2 + q + (size_t)q * (q + 1) / 2;
    pl.o_parts = off;
    off = align_up(off + (size_t)n * g * pl.split * pw * sizeof(double));
  }
  pl.o_part = off;
  off = align_up(off + (size_t)pl.nb * pl.GS * sizeof(double));
  pl.o_pll = off;
  off = align_up(off + (size_t)pl.nb * sizeof(double));
  pl.o_pitmp = off;
  off = align_up(off + (size_t)g * sizeof(double));
  pl.o_mwork = off;
  off = align_up(off + (size_t)g * mstep_work_doubles(p, q) * sizeof(double));
  pl.o_ll = off;
  off = align_up(off + sizeof(double));
  pl.o_stats = off;
  off = align_up(off + (size_t)pl.GS * sizeof(double));
  if (check_m > 0) {
    const int64_t m = check_m < n ? check_m : n;
    pl.check_m = m;
    pl.chk_per_block = stats_per_block(m, pl.tile);
    pl.chk_nb = (int)((m + pl.chk_per_block - 1) / pl.chk_per_block);
    if (pl.chk_nb < 1) pl.chk_nb = 1;
    const size_t rec = (size_t)(m > 0 ? m : 1) * g * pl.W * sizeof(double);
    pl.o_chk_y = off;
    off = align_up(off + (size_t)(m > 0 ? m : 1) * p * sizeof(double));
    pl.o_chk_rnet = off;
    off = align_up(off + rec);
    pl.o_chk_rghk = off;
    off = align_up(off + rec);
    pl.o_chk_part = off;
    off = align_up(off + (size_t)pl.chk_nb * pl.GS * sizeof(double));
    pl.o_chk_pll = off;
    off = align_up(off + (size_t)pl.chk_nb * sizeof(double));
    pl.o_chk_stats = off;  // network then GHK: GS statistics + log-likelihood each
    off = align_up(off + (size_t)2 * (pl.GS + 1) * sizeof(double));
  }
  pl.total = off;
  return pl;
}


int check_dims(int64_t n, int p, int q, int g, int N) {
  if (n < 0 || p < 1 || p > kMaxP || q < 1 || q > kMaxQ || g < 1 || g > kMaxG || N < 1)
    return CFUST_EINVAL;
  return CFUST_OK;
}

int acquire(const Plan& pl, const cfust_opts* o, Ws* ws) {
  ws->st = o ? (hipStream_t)o->stream : nullptr;
  ws->prof = o ? o->prof_ms : nullptr;
  ws->surr = o ? o->surrogate : nullptr;
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


int check_opts(const cfust_opts* o) {
  if (!o) return CFUST_OK;
  if (o->precision != CFUST_FP64 && o->precision != CFUST_FP32) return CFUST_EINVAL;
  if (o->nu_mode != CFUST_NU_OSL && o->nu_mode != CFUST_NU_EXACT &&
      o->nu_mode != CFUST_NU_FIXED)
    return CFUST_EINVAL;
  if (!(o->nu_lo > 0.0) || !(o->nu_hi >= o->nu_lo)) return CFUST_EINVAL;
  if (o->reorder != 0 && o->reorder != 1) return CFUST_EINVAL;
  if (o->surrogate_check < 0) return CFUST_EINVAL;
  if (!(o->surrogate_switch >= 0.0)) return CFUST_EINVAL;
  return CFUST_OK;
}

// per-component blocks (eq. (2)) of all g components on one block
void launch_precompute(const Ws& ws, const Plan& pl, const double* pi, const double* mu,
                       const double* Sigma, const double* Delta, const double* nu) {
  precompute_kernel<<<1, kPrecompThreads, precompute_lds_bytes(pl.p, pl.q, pl.g), ws.st>>>(
      pl.p, pl.q, pl.g, pi, Sigma, Delta, mu, nu, ws.at<double>(pl.o_comp),
      ws.at<int>(pl.o_status));
}

}  // namespace host
}  // namespace cfust

namespace {

// the plan of the m sampled observations of the surrogate check: shares the
// per-component blocks, chi tables and points; records in `rec`
Plan check_plan(const Plan& pl, size_t rec) {
  Plan ps = pl;
  ps.n = pl.check_m;
  ps.per_block = pl.chk_per_block;
  ps.nb = pl.chk_nb;
  ps.o_pair = rec;
  ps.o_part = pl.o_chk_part;
  ps.o_pll = pl.o_chk_pll;
  ps.exact = false;
  ps.reorder = false;
  ps.split = 1;
  return ps;
}

// per-call parameter preparation: component blocks and chi scale tables
template <typename T>
void launch_prepare(const Ws& ws, const Plan& pl, const double* pi, const double* mu,
                    const double* Sigma, const double* Delta, const double* nu, const double* u,
                    bool points) {
  launch_precompute(ws, pl, pi, mu, Sigma, Delta, nu);
  const int q1 = pl.q + 1;
  if (points) {
    int64_t tot = (int64_t)pl.N * q1;
    points_kernel<T><<<(unsigned)((tot + 255) / 256), 256, 0, ws.st>>>(
        u, pl.N, q1, ws.at<T>(pl.o_uT), ws.at<T>(pl.o_ubT), ws.at<int>(pl.o_status));
  }
  int64_t tot = (int64_t)2 * pl.g * pl.N;
  chi_kernel<T><<<(unsigned)((tot + 127) / 128), 128, 0, ws.st>>>(
      ws.at<double>(pl.o_comp), pl.stride, CompLayout(pl.p, pl.q).nu, pl.p, pl.g, u, pl.N, q1,
      ws.at<T>(pl.o_sA), ws.at<T>(pl.o_sB), ws.at<T>(pl.o_rsB),
      pl.exact ? ws.at<T>(pl.o_tA) : nullptr, ws.at<int>(pl.o_status));
}


template <typename T, bool MOM>
void launch_pairs(const Ws& ws, const Plan& pl, const double* y, const double* mu) {
  switch (pl.q) {
    case 1: host::launch_pairs_q<T, 1, MOM>(ws, pl, y, mu); break;
    case 2: host::launch_pairs_q<T, 2, MOM>(ws, pl, y, mu); break;
    case 3: host::launch_pairs_q<T, 3, MOM>(ws, pl, y, mu); break;
    case 4: host::launch_pairs_q<T, 4, MOM>(ws, pl, y, mu); break;
    case 5: host::launch_pairs_q<T, 5, MOM>(ws, pl, y, mu); break;
    case 6: host::launch_pairs_q<T, 6, MOM>(ws, pl, y, mu); break;
    case 7: host::launch_pairs_q<T, 7, MOM>(ws, pl, y, mu); break;
    case 8: host::launch_pairs_q<T, 8, MOM>(ws, pl, y, mu); break;
    case 9: host::launch_pairs_q<T, 9, MOM>(ws, pl, y, mu); break;
    case 10: host::launch_pairs_q<T, 10, MOM>(ws, pl, y, mu); break;
    case 11: host::launch_pairs_q<T, 11, MOM>(ws, pl, y, mu); break;
    case 12: host::launch_pairs_q<T, 12, MOM>(ws, pl, y, mu); break;
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
int run_estep(Ws& ws, const Plan& pl, const double* y, const double* pi, const double* mu,
              const double* Sigma, const double* Delta, const double* nu, const double* u,
              bool points, bool moments, double* stats, double* loglik,
              const cfust_estep_out* out, double* logf_only) {
  prof_begin(ws, 0);
  launch_prepare<T>(ws, pl, pi, mu, Sigma, Delta, nu, u, points);
  prof_end(ws, 0);
  prof_begin(ws, 1);
  if (ws.surr) {
    int rc = host::launch_surrogate_pairs<T>(ws, pl, y, mu);
    if (rc) return rc;
  } else if (moments) {
    launch_pairs<T, true>(ws, pl, y, mu);
  } else {
    launch_pairs<T, false>(ws, pl, y, mu);
  }
  prof_end(ws, 1);
  prof_begin(ws, 2);
  launch_stats(ws, pl, y, mu, moments, stats, loglik, out, logf_only);
  prof_end(ws, 2);
  if (ws.surr && pl.check_m > 0) {
    // difference estimator: totals += (n/m) (GHK - network) over the m
    // sampled observations, whose network records are copied out first
    const int64_t m = pl.check_m;
    double* ysub = ws.at<double>(pl.o_chk_y);
    double* cst = ws.at<double>(pl.o_chk_stats);
    const int64_t cells = m * (int64_t)(pl.p > pl.g * pl.W ? pl.p : pl.g * pl.W);
    check_gather_kernel<<<(unsigned)((cells + 255) / 256), 256, 0, ws.st>>>(
        y, pl.n, pl.p, ws.at<double>(pl.o_pair), pl.g * pl.W, m, ysub,
        ws.at<double>(pl.o_chk_rnet));
    const Plan pg = check_plan(pl, pl.o_chk_rghk);
    if (moments)
      launch_pairs<T, true>(ws, pg, ysub, mu);
    else
      launch_pairs<T, false>(ws, pg, ysub, mu);
    launch_stats(ws, pg, ysub, mu, moments, moments ? cst + pl.GS + 1 : nullptr,
                 cst + 2 * pl.GS + 1, nullptr, nullptr);
    const Plan pn = check_plan(pl, pl.o_chk_rnet);
    launch_stats(ws, pn, ysub, mu, moments, moments ? cst : nullptr, cst + pl.GS, nullptr,
                 nullptr);
    check_combine_kernel<<<(pl.GS + 256) / 256, 256, 0, ws.st>>>(
        cst, pl.GS, moments ? 1 : 0, (double)pl.n / (double)m, moments ? stats : nullptr, loglik,
        ws.at<int>(pl.o_status));
  }
  return CFUST_OK;
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
  mstep_kernel<<<1, 256, mstep_lds_bytes(pl.p, pl.q, pl.g), ws.st>>>(
      stats, n, pl.p, pl.q, pl.g, mu_old, Delta_old, nu_old,
                                    fixed, fixd, lo, hi, pi, mu, Sigma, Delta, nu,
                                    ws.at<double>(pl.o_pitmp), ws.at<double>(pl.o_mwork),
                                    ws.at<int>(pl.o_status));
  prof_end(ws, 3);
}

int check_surrogate(const cfust_opts* o, int q) {
  if (!o || !o->surrogate) return CFUST_OK;
  const cfust_surrogate* s = o->surrogate;
  // the network has no derivative output for the exact E[log W | y], and it
  // was trained on natural-order GHK labels
  if (o->nu_mode == CFUST_NU_EXACT || o->reorder) return CFUST_EINVAL;
  return surrogate_ready(s, q) ? CFUST_OK : CFUST_EINVAL;
}

// sampled observations of the surrogate check (0: none)
int64_t check_of(const cfust_opts* o) {
  return (o && o->surrogate && o->surrogate_check > 0) ? (int64_t)o->surrogate_check : 0;
}

// forms that exist only up to kMaxQFull
int check_q_forms(const cfust_opts* o, int q) {
  if (!o || q <= kMaxQFull) return CFUST_OK;
  return (o->reorder || o->surrogate) ? CFUST_EINVAL : CFUST_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free E-step (cfust_estep_noalloc): one
// copy per GPU, allocated when this code object is loaded on the GPU.  Host
// code must never pass `scratch` itself to a kernel or a copy (on the host
// it is only a stand-in for the symbol): scratch_ptr() gives the device
// address of the current GPU's copy.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = CFUST_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// device address of the current GPU's scratch array, looked up once per GPU
int scratch_ptr(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return CFUST_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return CFUST_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
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
  o->graph = 1;
  o->tile = 0;
}

int cfust_stats_size(int p, int q) { return StatLayout(p, q).S; }

size_t cfust_opts_size(void) { return sizeof(cfust_opts); }

int cfust_workspace_size(int64_t n, int p, int q, int g, int n_qmc, int precision, size_t* bytes) {
  if (!bytes) return CFUST_EINVAL;
  int rc = check_dims(n, p, q, g, n_qmc);
  if (rc) return rc;
  if (precision != CFUST_FP64 && precision != CFUST_FP32) return CFUST_EINVAL;
  *bytes = make_plan(n, p, q, g, n_qmc, precision).total;
  return CFUST_OK;
}

int cfust_workspace_size_opts(int64_t n, int p, int q, int g, int n_qmc, const cfust_opts* o,
                              size_t* bytes) {
  if (!bytes) return CFUST_EINVAL;
  int rc = check_dims(n, p, q, g, n_qmc);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  *bytes = make_plan(n, p, q, g, n_qmc, o ? o->precision : CFUST_FP64, check_of(o)).total;
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
  if ((rc = check_surrogate(o, q))) return rc;
  if ((rc = check_q_forms(o, q))) return rc;
  if ((n > 0 && !y) || !pi || !mu || !Sigma || !Delta || !nu || !u || !out->stats || !out->loglik)
    return CFUST_EINVAL;
  const int prec = o ? o->precision : CFUST_FP64;
  Plan pl = make_plan(n, p, q, g, n_qmc, prec, check_of(o));
  pl.exact = o && o->nu_mode == CFUST_NU_EXACT;
  pl.reorder = o && o->reorder;
  Ws ws;
  if ((rc = acquire(pl, o, &ws))) return rc;
  clear_status(ws, pl);
  if (prec == CFUST_FP32)
    rc = run_estep<float>(ws, pl, y, pi, mu, Sigma, Delta, nu, u, true, true, out->stats,
                          out->loglik, out, nullptr);
  else
    rc = run_estep<double>(ws, pl, y, pi, mu, Sigma, Delta, nu, u, true, true, out->stats,
                           out->loglik, out, nullptr);
  if (!rc) rc = launch_check();
  int st = fetch_status(ws, pl, &out->bad_component);
  release(&ws);
  return rc ? rc : st;
}

int cfust_estep_noalloc(const double* y, int64_t n, int p, int q, int g, const double* pi,
                        const double* mu, const double* Sigma, const double* Delta,
                        const double* nu, const double* u, int n_qmc, const cfust_opts* o,
                        cfust_estep_out* out) {
  if (!out) return CFUST_EINVAL;
  out->bad_component = -1;
  int rc = check_dims(n, p, q, g, n_qmc);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  if (o && (o->surrogate || o->prof_ms || o->workspace)) return CFUST_EINVAL;
  if ((rc = check_q_forms(o, q))) return rc;
  const Plan pl = make_plan(n, p, q, g, n_qmc, o ? o->precision : CFUST_FP64);
  if (pl.total > kScratchBytes) return CFUST_ENOMEM;
  void* base = nullptr;
  if ((rc = scratch_ptr(&base))) return rc;
  cfust_opts oo;
  if (o)
    oo = *o;
  else
    cfust_default_opts(&oo);
  oo.workspace = base;
  oo.workspace_bytes = kScratchBytes;
  return cfust_estep(y, n, p, q, g, pi, mu, Sigma, Delta, nu, u, n_qmc, &oo, out);
}

int cfust_loglik(const double* y, int64_t n, int p, int q, int g, const double* pi,
                 const double* mu, const double* Sigma, const double* Delta, const double* nu,
                 const double* u, int n_qmc, const cfust_opts* o, double* loglik, double* logf) {
  int rc = check_dims(n, p, q, g, n_qmc);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  if ((rc = check_surrogate(o, q))) return rc;
  if ((rc = check_q_forms(o, q))) return rc;
  if ((n > 0 && !y) || !pi || !mu || !Sigma || !Delta || !nu || !u || !loglik) return CFUST_EINVAL;
  const int prec = o ? o->precision : CFUST_FP64;
  Plan pl = make_plan(n, p, q, g, n_qmc, prec, check_of(o));
  pl.reorder = o && o->reorder;
  Ws ws;
  if ((rc = acquire(pl, o, &ws))) return rc;
  clear_status(ws, pl);
  if (prec == CFUST_FP32)
    rc = run_estep<float>(ws, pl, y, pi, mu, Sigma, Delta, nu, u, true, false, nullptr, loglik,
                          nullptr, logf);
  else
    rc = run_estep<double>(ws, pl, y, pi, mu, Sigma, Delta, nu, u, true, false, nullptr, loglik,
                           nullptr, logf);
  if (!rc) rc = launch_check();
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
  if ((rc = check_surrogate(o, q))) return rc;
  if ((rc = check_q_forms(o, q))) return rc;
  if (!y || !pi || !mu || !Sigma || !Delta || !nu || !u || !loglik_trace || !n_iter)
    return CFUST_EINVAL;
  cfust_opts def;
  cfust_default_opts(&def);
  if (!o) o = &def;
  if (o->max_iter < 0) return CFUST_EINVAL;
  Plan pl = make_plan(n, p, q, g, n_qmc, o->precision, check_of(o));
  pl.exact = o && o->nu_mode == CFUST_NU_EXACT;
  pl.reorder = o->reorder != 0;
  Ws ws;
  if ((rc = acquire(pl, o, &ws))) return rc;
  double* stats = ws.at<double>(pl.o_stats);
  double* ll_dev = ws.at<double>(pl.o_ll);
  clear_status(ws, pl);
  *n_iter = 0;
  int result = CFUST_OK;
  // With a surrogate: phase 1 runs surrogate E-steps until Aitken's rule
  // stops; the next E-step re-evaluates the same parameters with the GHK
  // kernel and phase 2 continues with GHK E-steps until the rule stops again.
  cfust_surrogate* surr = ws.surr;
  if (surr) surrogate_set_switch(surr, -1);
  int phase_start = 0;
  for (int t = 0;; ++t) {
    const bool last = t == o->max_iter;
    if (ws.surr && o->adapt_samples > 0) {
      result = cfust_surrogate_adapt(ws.surr, y, n, p, q, g, pi, mu, Sigma, Delta, nu, u, n_qmc,
                                     o->adapt_samples, o->adapt_epochs,
                                     (unsigned long long)t + 1, o, nullptr, nullptr);
      if (result) break;
    }
    if (o->precision == CFUST_FP32)
      result = run_estep<float>(ws, pl, y, pi, mu, Sigma, Delta, nu, u, t == 0, !last, stats,
                                ll_dev, nullptr, nullptr);
    else
      result = run_estep<double>(ws, pl, y, pi, mu, Sigma, Delta, nu, u, t == 0, !last, stats,
                                 ll_dev, nullptr, nullptr);
    if (result || (result = launch_check())) break;
    double ll = 0.0;
    if (hipMemcpyAsync(&ll, ll_dev, sizeof(double), hipMemcpyDeviceToHost, ws.st) != hipSuccess) {
      result = CFUST_EHIP;
      break;
    }
    if ((result = fetch_status(ws, pl, bad_component))) break;
    loglik_trace[t] = ll;
    *n_iter = t;
    bool conv = false;
    if (t - phase_start >= 2) {
      double linf = cfust_aitken_linf(loglik_trace[t - 2], loglik_trace[t - 1], ll);
      conv = fabs(linf - ll) < o->tol;
    }
    // with a surrogate, an iteration that moved l by less than the network's
    // accuracy also ends the surrogate phase
    if (ws.surr && o->surrogate_switch > 0.0 && t > phase_start &&
        fabs(ll - loglik_trace[t - 1]) < o->surrogate_switch * fabs(ll))
      conv = true;
    if (conv && ws.surr && !last) {
      ws.surr = nullptr;
      surrogate_set_switch(surr, t + 1);
      phase_start = t + 1;
      continue;
    }
    if (conv || last) break;
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
  if (!x || !out || n < 0 || fn < 0 || fn > 17 || ((fn == 4 || fn == 11 || fn >= 14) && !x2))
    return CFUST_EINVAL;
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
