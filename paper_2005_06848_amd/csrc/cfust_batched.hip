// C ABI of the batched form (section 3.1, Algorithm 1: many EM starts
// advanced together in one persistent launch per iteration, replayed as a
// hipGraph, with the launch shape from an autotuner), of the multistart fit
// built on it (Algorithm 1 in full) and of the randomised-QMC error bar of the
// log-likelihood.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "../../include/cfust.h"
#include "cfust_batched.hpp"
#include "cfust_host.hpp"

using namespace cfust;
using namespace cfust::host;

namespace {

// Launch shape of the pair kernels: waves per block, work items per fetch,
// persistent waves per SIMD, and waves per pair (K: each wave integrates
// N / K of the pair's QMC points; K > 1 runs bpart_kernel + bfinish_kernel).
struct Shape {
  int wpb, chunk, wps, split;
};
const Shape kShapes[] = {{1, 1, 4, 1}, {1, 4, 4, 1}, {2, 2, 4, 1}, {4, 1, 4, 1},
                         {4, 4, 4, 1}, {1, 1, 8, 1}, {2, 4, 8, 1}, {4, 2, 8, 1},
                         {1, 16, 4, 1}, {4, 16, 8, 1}, {1, 1, 4, 2}, {4, 1, 4, 2},
                         {1, 2, 8, 2}, {1, 1, 4, 4}, {4, 1, 4, 4}, {1, 1, 4, 8}};
constexpr int kNumShapes = (int)(sizeof(kShapes) / sizeof(kShapes[0]));

// Splitting a pair is offered only to batches of fewer than kSplitPairs
// pairs (above that the persistent waves are busy for at least 16 pairs
// each and the tail is a small fraction), with at least four points per
// lane in every slice (K <= N / 256), K a power of two up to kSplitMax.
constexpr int64_t kSplitPairs = 65536;
constexpr int kSplitMax = 8;

int max_split(int64_t total_pairs, int N) {
  if (total_pairs >= kSplitPairs) return 1;
  int K = 1;
  while (2 * K <= kSplitMax && 2 * K <= N / 256) K *= 2;
  return K;
}

// doubles of one slice record of the split kernels (the exact-nu width, so
// the workspace size does not depend on the nu mode): integral A's R, S0
// and tangent, integral B's R, S0, S1[q] and S2[q(q+1)/2]
int split_part_width(int q) { return 5 + q + q * (q + 1) / 2; }

struct LastCfg {
  Shape s{4, 4, 4, 1};
  double ms = 0.0;
  int N = 0;
};
LastCfg g_last;
std::mutex g_mu;
struct TuneKey {
  int q, N, prec, kmax;
  bool operator==(const TuneKey& o) const {
    return q == o.q && N == o.N && prec == o.prec && kmax == o.kmax;
  }
};
std::vector<std::pair<TuneKey, LastCfg>> g_tuned;

struct BPlan {
  int P, p, q, N, prec, W, S, G, stride, tile, ny, total_blocks, red_total, max_iter, kmax;
  int64_t total_obs, total_pairs, total_part;
  std::vector<int64_t> n_off, pair_off, per_blk, part_off;
  std::vector<int> g_off, blk_off, red_off;
  size_t lds_bytes;
  // workspace offsets
  size_t o_noff, o_goff, o_poff, o_boff, o_perb, o_partoff, o_roff, o_active, o_status, o_iter,
      o_niter, o_llcur, o_trace, o_comp, o_uT, o_ubT, o_sA, o_sB, o_rsB, o_pair, o_part, o_pll,
      o_stats, o_pitmp, o_mwork, o_counter, o_pstat, o_tA, o_split, total;
  bool exact = false;  // exact E[log W | y] (tangent table o_tA)
};

int make_bplan(int P, int p, int q, const int64_t* n_obs, const int* g, int N, int prec,
               int max_iter, bool exact, BPlan* pl) {
  pl->P = P;
  pl->exact = exact;
  pl->p = p;
  pl->q = q;
  pl->N = N;
  pl->prec = prec;
  pl->max_iter = max_iter;
  pl->W = pair_width(q);
  pl->S = StatLayout(p, q).S;
  pl->stride = CompLayout(p, q).stride;
  pl->n_off.assign(P + 1, 0);
  pl->g_off.assign(P + 1, 0);
  pl->pair_off.assign(P + 1, 0);
  pl->blk_off.assign(P + 1, 0);
  pl->per_blk.assign(P, 1);
  pl->part_off.assign(P + 1, 0);
  pl->red_off.assign(P + 1, 0);
  int gmax = 1;
  for (int k = 0; k < P; ++k) {
    if (n_obs[k] < 1 || g[k] < 1 || g[k] > kMaxG) return CFUST_EINVAL;
    gmax = std::max(gmax, g[k]);
  }
  size_t per_obs = (size_t)stats_lds_per_obs(p, gmax, pl->W) * sizeof(double);
  int tile = (int)((48 * 1024) / per_obs);
  pl->tile = tile < 1 ? 1 : (tile > 16 ? 16 : tile);
  pl->lds_bytes = per_obs * pl->tile;
  int gs_max = 0;
  for (int k = 0; k < P; ++k) {
    pl->n_off[k + 1] = pl->n_off[k] + n_obs[k];
    pl->g_off[k + 1] = pl->g_off[k] + g[k];
    pl->pair_off[k + 1] = pl->pair_off[k] + n_obs[k] * g[k];
    int64_t per = (n_obs[k] + 127) / 128;
    if (per < pl->tile) per = pl->tile;
    per = ((per + pl->tile - 1) / pl->tile) * pl->tile;
    pl->per_blk[k] = per;
    int nb = (int)((n_obs[k] + per - 1) / per);
    int GS = g[k] * pl->S;
    gs_max = std::max(gs_max, GS);
    pl->blk_off[k + 1] = pl->blk_off[k] + nb;
    pl->part_off[k + 1] = pl->part_off[k] + (int64_t)nb * GS;
    pl->red_off[k + 1] = pl->red_off[k] + GS + 1;
  }
  pl->G = pl->g_off[P];
  pl->total_obs = pl->n_off[P];
  pl->total_pairs = pl->pair_off[P];
  if (pl->total_pairs >= ((int64_t)1 << 31)) return CFUST_EINVAL;  // 32-bit work counter with headroom
  pl->total_blocks = pl->blk_off[P];
  pl->total_part = pl->part_off[P];
  pl->red_total = pl->red_off[P];
  pl->ny = (gs_max + kStatsPerBlock - 1) / kStatsPerBlock;
  size_t es = prec == CFUST_FP32 ? sizeof(float) : sizeof(double);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  pl->o_noff = take((P + 1) * sizeof(int64_t));
  pl->o_goff = take((P + 1) * sizeof(int));
  pl->o_poff = take((P + 1) * sizeof(int64_t));
  pl->o_boff = take((P + 1) * sizeof(int));
  pl->o_perb = take(P * sizeof(int64_t));
  pl->o_partoff = take((P + 1) * sizeof(int64_t));
  pl->o_roff = take((P + 1) * sizeof(int));
  pl->o_active = take(P * sizeof(int));
  pl->o_status = take(2 * P * sizeof(int));
  pl->o_iter = take(P * sizeof(int));
  pl->o_niter = take(P * sizeof(int));
  pl->o_llcur = take(P * sizeof(double));
  pl->o_trace = take((size_t)P * (max_iter + 1) * sizeof(double));
  pl->o_comp = take((size_t)pl->G * pl->stride * sizeof(double));
  pl->o_uT = take((size_t)(q + 1) * N * es);
  pl->o_ubT = take((size_t)(q + 1) * N * es);
  pl->o_sA = take((size_t)pl->G * N * es);
  pl->o_sB = take((size_t)pl->G * N * es);
  pl->o_rsB = take((size_t)pl->G * N * es);
  pl->o_pair = take((size_t)pl->total_pairs * pl->W * sizeof(double));
  pl->o_part = take((size_t)pl->total_part * sizeof(double));
  pl->o_pll = take((size_t)pl->total_blocks * sizeof(double));
  pl->o_stats = take((size_t)pl->G * pl->S * sizeof(double));
  pl->o_pitmp = take((size_t)pl->G * sizeof(double));
  pl->o_mwork = take((size_t)pl->G * mstep_work_doubles(p, q) * sizeof(double));
  pl->o_counter = take(64);
  pl->o_pstat = take(4 * sizeof(int));
  pl->o_tA = take((size_t)pl->G * N * es);  // used with the exact nu step only
  pl->kmax = max_split(pl->total_pairs, N);
  pl->o_split = take(pl->kmax > 1 ? (size_t)pl->total_pairs * pl->kmax * split_part_width(q) *
                                        sizeof(double)
                                  : 0);
  pl->total = off;
  return CFUST_OK;
}

BatchDev batch_view(const BPlan& pl, char* base) {
  BatchDev b;
  b.P = pl.P;
  b.p = pl.p;
  b.q = pl.q;
  b.W = pl.W;
  b.S = pl.S;
  b.n_off = (const int64_t*)(base + pl.o_noff);
  b.g_off = (const int*)(base + pl.o_goff);
  b.pair_off = (const int64_t*)(base + pl.o_poff);
  b.blk_off = (const int*)(base + pl.o_boff);
  b.per_blk = (const int64_t*)(base + pl.o_perb);
  b.part_off = (const int64_t*)(base + pl.o_partoff);
  b.red_off = (const int*)(base + pl.o_roff);
  b.active = (int*)(base + pl.o_active);
  b.status = (int*)(base + pl.o_status);
  b.iter = (int*)(base + pl.o_iter);
  b.n_iter = (int*)(base + pl.o_niter);
  b.ll_cur = (double*)(base + pl.o_llcur);
  b.trace = (double*)(base + pl.o_trace);
  return b;
}

struct BArgs {
  const double* y;
  double *pi, *mu, *Sigma, *Delta, *nu;
  const double* u;
  int nu_fixed, fix_delta_zero;
  double nu_lo, nu_hi, tol;
};

template <typename T, int Q, bool EXACT>
void launch_bpair_e(const BPlan& pl, const BatchDev& b, char* base, const BArgs& a,
                    hipStream_t st, const Shape& sh, unsigned int total, int n_cu) {
  int waves = sh.wps * 4 * n_cu;
  int blocks = std::max(1, waves / sh.wpb);
  if (sh.split > 1) {
    const int K = sh.split;
    double* parts = (double*)(base + pl.o_split);
    bpart_kernel<T, Q, EXACT><<<blocks, 64 * sh.wpb, 0, st>>>(
        b, a.y, a.mu, (const double*)(base + pl.o_comp), (const T*)(base + pl.o_sA),
        (const T*)(base + pl.o_sB), (const T*)(base + pl.o_rsB), (const T*)(base + pl.o_uT),
        (const T*)(base + pl.o_ubT), pl.N, K, parts, (unsigned int*)(base + pl.o_counter),
        total * (unsigned int)K, sh.chunk, EXACT ? (const T*)(base + pl.o_tA) : nullptr);
    bfinish_kernel<T, Q, EXACT><<<(total + 3) / 4, 256, 0, st>>>(
        b, a.y, a.mu, (const double*)(base + pl.o_comp), pl.N, K, parts,
        (double*)(base + pl.o_pair), total);
    return;
  }
  bpair_kernel<T, Q, EXACT><<<blocks, 64 * sh.wpb, 0, st>>>(
      b, a.y, a.mu, (const double*)(base + pl.o_comp), (const T*)(base + pl.o_sA),
      (const T*)(base + pl.o_sB), (const T*)(base + pl.o_rsB), (const T*)(base + pl.o_uT),
      (const T*)(base + pl.o_ubT), pl.N, (double*)(base + pl.o_pair),
      (unsigned int*)(base + pl.o_counter), total, sh.chunk,
      EXACT ? (const T*)(base + pl.o_tA) : nullptr);
}

template <typename T, int Q>
void launch_bpair(const BPlan& pl, const BatchDev& b, char* base, const BArgs& a, hipStream_t st,
                  const Shape& sh, unsigned int total, int n_cu) {
  if (pl.exact)
    launch_bpair_e<T, Q, true>(pl, b, base, a, st, sh, total, n_cu);
  else
    launch_bpair_e<T, Q, false>(pl, b, base, a, st, sh, total, n_cu);
}

template <typename T>
void launch_bpair_q(const BPlan& pl, const BatchDev& b, char* base, const BArgs& a,
                    hipStream_t st, const Shape& sh, unsigned int total, int n_cu) {
  fill_uint_kernel<<<1, 64, 0, st>>>((unsigned int*)(base + pl.o_counter), 0u);
  switch (pl.q) {
    case 1: launch_bpair<T, 1>(pl, b, base, a, st, sh, total, n_cu); break;
    case 2: launch_bpair<T, 2>(pl, b, base, a, st, sh, total, n_cu); break;
    case 3: launch_bpair<T, 3>(pl, b, base, a, st, sh, total, n_cu); break;
    case 4: launch_bpair<T, 4>(pl, b, base, a, st, sh, total, n_cu); break;
    case 5: launch_bpair<T, 5>(pl, b, base, a, st, sh, total, n_cu); break;
    case 6: launch_bpair<T, 6>(pl, b, base, a, st, sh, total, n_cu); break;
    case 7: launch_bpair<T, 7>(pl, b, base, a, st, sh, total, n_cu); break;
    case 8: launch_bpair<T, 8>(pl, b, base, a, st, sh, total, n_cu); break;
  }
}

template <typename T>
void launch_bprepare(const BPlan& pl, const BatchDev& b, char* base, const BArgs& a,
                     hipStream_t st) {
  bprecompute_kernel<<<pl.P, kPrecompThreads, precompute_lds_bytes(pl.p, pl.q, kMaxG), st>>>(
      b, a.pi, a.Sigma, a.Delta, a.mu, a.nu,
                                          (double*)(base + pl.o_comp));
  int64_t tot = (int64_t)2 * pl.G * pl.N;
  bchi_kernel<T><<<(unsigned)((tot + 127) / 128), 128, 0, st>>>(
      b, (const double*)(base + pl.o_comp), pl.stride, CompLayout(pl.p, pl.q).nu, pl.G, a.u, pl.N,
      (T*)(base + pl.o_sA), (T*)(base + pl.o_sB), (T*)(base + pl.o_rsB),
      pl.exact ? (T*)(base + pl.o_tA) : nullptr);
}

// one EM iteration of every active problem; no host synchronisation
template <typename T>
void batched_iteration(const BPlan& pl, const BatchDev& b, char* base, const BArgs& a,
                       hipStream_t st, const Shape& sh, int n_cu) {
  launch_bprepare<T>(pl, b, base, a, st);
  launch_bpair_q<T>(pl, b, base, a, st, sh, (unsigned int)pl.total_pairs, n_cu);
  dim3 grid(pl.total_blocks, pl.ny);
  bstats_kernel<<<grid, 256, pl.lds_bytes, st>>>(b, a.y, a.mu, (const double*)(base + pl.o_pair),
                                                 pl.tile, (double*)(base + pl.o_part),
                                                 (double*)(base + pl.o_pll));
  breduce_kernel<<<pl.red_total, 64, 0, st>>>(b, (const double*)(base + pl.o_part),
                                              (const double*)(base + pl.o_pll),
                                              (double*)(base + pl.o_stats));
  baitken_kernel<<<(pl.P + 63) / 64, 64, 0, st>>>(b, pl.max_iter, a.tol);
  bmstep_kernel<<<pl.P, 64, mstep_lds_bytes(pl.p, pl.q, kMaxG), st>>>(
      b, (const double*)(base + pl.o_stats), a.nu_fixed,
                                     a.fix_delta_zero, a.nu_lo, a.nu_hi, a.pi, a.mu, a.Sigma,
                                     a.Delta, a.nu, (double*)(base + pl.o_pitmp),
                                     (double*)(base + pl.o_mwork));
}

// Autotuner: times the pair kernels of every candidate shape that the batch
// allows (waves per pair up to pl.kmax) after one warm-up launch, and keeps
// the fastest.  Large batches are timed on their first pairs (about 1/8 of
// the work, at least 8192 pairs); a batch small enough to be offered split
// shapes is timed whole, since the point of splitting is how the last
// pairs of a launch share the chip.
template <typename T>
LastCfg autotune(const BPlan& pl, const BatchDev& b, char* base, const BArgs& a, hipStream_t st,
                 int n_cu) {
  LastCfg best;
  best.ms = 1e300;
  best.N = pl.N;
  unsigned int sub =
      pl.kmax > 1 ? (unsigned int)pl.total_pairs
                  : (unsigned int)std::min<int64_t>(pl.total_pairs,
                                                    std::max<int64_t>(pl.total_pairs / 8, 8192));
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  launch_bprepare<T>(pl, b, base, a, st);
  launch_bpair_q<T>(pl, b, base, a, st, kShapes[0], sub, n_cu);
  for (int s = 0; s < kNumShapes; ++s) {
    if (kShapes[s].split > pl.kmax) continue;
    (void)hipEventRecord(e0, st);
    launch_bpair_q<T>(pl, b, base, a, st, kShapes[s], sub, n_cu);
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best.ms) {
      best.ms = ms;
      best.s = kShapes[s];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

template <typename T>
int run_batched(const BPlan& pl, char* base, const BArgs& a, hipStream_t st, const cfust_opts* o,
                double* loglik_trace, int* n_iter, int* status) {
  BatchDev b = batch_view(pl, base);
  int dev = 0, n_cu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) n_cu = prop.multiProcessorCount;
  }
  // offsets and state
  (void)hipMemcpyAsync(base + pl.o_noff, pl.n_off.data(), (pl.P + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(base + pl.o_goff, pl.g_off.data(), (pl.P + 1) * sizeof(int), hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(base + pl.o_poff, pl.pair_off.data(), (pl.P + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(base + pl.o_boff, pl.blk_off.data(), (pl.P + 1) * sizeof(int), hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(base + pl.o_perb, pl.per_blk.data(), pl.P * sizeof(int64_t), hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(base + pl.o_partoff, pl.part_off.data(), (pl.P + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(base + pl.o_roff, pl.red_off.data(), (pl.P + 1) * sizeof(int), hipMemcpyHostToDevice, st);
  binit_state_kernel<<<(pl.P + 63) / 64, 64, 0, st>>>(b, pl.max_iter);
  fill_int_kernel<<<1, 64, 0, st>>>((int*)(base + pl.o_pstat), 4, 0);
  int64_t tot = (int64_t)pl.N * (pl.q + 1);
  points_kernel<T><<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(
      a.u, pl.N, pl.q + 1, (T*)(base + pl.o_uT), (T*)(base + pl.o_ubT), (int*)(base + pl.o_pstat));
  if (hipGetLastError() != hipSuccess) return CFUST_EHIP;
  int pst[2] = {0, 0};
  (void)hipMemcpyAsync(pst, base + pl.o_pstat, 2 * sizeof(int), hipMemcpyDeviceToHost, st);
  if (hipStreamSynchronize(st) != hipSuccess) return CFUST_EHIP;
  if (pst[0] != kOk) return CFUST_EINVAL;
  // launch shape
  LastCfg cfg;
  const int tile = o ? o->tile : 0;
  cfg.N = pl.N;
  if (tile > 0) {
    if (tile > kNumShapes || kShapes[tile - 1].split > pl.kmax) return CFUST_EINVAL;
    cfg.s = kShapes[tile - 1];
  } else {
    TuneKey key{pl.q, pl.N, pl.prec, pl.kmax};
    bool found = false;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      for (auto& kv : g_tuned)
        if (kv.first == key) {
          cfg = kv.second;
          found = true;
        }
    }
    if (!found) {
      cfg = autotune<T>(pl, b, base, a, st, n_cu);
      std::lock_guard<std::mutex> lk(g_mu);
      g_tuned.push_back({key, cfg});
    }
    // the tuning launches touched the pair buffer and the chi tables only;
    // the iteration below recomputes both
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_last = cfg;
  }
  const bool use_graph = o ? o->graph != 0 : true;
  const int replays = pl.max_iter + 1;
  std::vector<int> act(pl.P);
  auto any_active = [&]() -> int {
    if (hipMemcpyAsync(act.data(), base + pl.o_active, pl.P * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
      return -1;
    if (hipStreamSynchronize(st) != hipSuccess) return -1;
    for (int v : act)
      if (v) return 1;
    return 0;
  };
  const int kCheck = 8;  // iterations between host checks of the active mask
  if (use_graph) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return CFUST_EHIP;
    batched_iteration<T>(pl, b, base, a, st, cfg.s, n_cu);
    if (hipStreamEndCapture(st, &graph) != hipSuccess) return CFUST_EHIP;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return CFUST_EHIP;
    }
    int rc = CFUST_OK;
    for (int r = 0; r < replays; ++r) {
      if (hipGraphLaunch(exec, st) != hipSuccess) {
        rc = CFUST_EHIP;
        break;
      }
      if ((r + 1) % kCheck == 0 || r + 1 == replays) {
        int aa = any_active();
        if (aa < 0) {
          rc = CFUST_EHIP;
          break;
        }
        if (aa == 0) break;
      }
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (rc) return rc;
  } else {
    for (int r = 0; r < replays; ++r) {
      batched_iteration<T>(pl, b, base, a, st, cfg.s, n_cu);
      if (hipGetLastError() != hipSuccess) return CFUST_EHIP;
      if ((r + 1) % kCheck == 0 || r + 1 == replays) {
        int aa = any_active();
        if (aa < 0) return CFUST_EHIP;
        if (aa == 0) break;
      }
    }
  }
  // results
  std::vector<int> stat(2 * pl.P);
  (void)hipMemcpyAsync(loglik_trace, base + pl.o_trace, (size_t)pl.P * (pl.max_iter + 1) * sizeof(double), hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(n_iter, base + pl.o_niter, pl.P * sizeof(int), hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(stat.data(), base + pl.o_status, 2 * pl.P * sizeof(int), hipMemcpyDeviceToHost, st);
  if (hipStreamSynchronize(st) != hipSuccess) return CFUST_EHIP;
  for (int k = 0; k < pl.P; ++k) {
    int c = stat[2 * k];
    status[k] = c == kOk ? CFUST_OK : c == kEInval ? CFUST_EINVAL : c == kENotPD ? CFUST_ENOTPD
                                                                 : CFUST_ENONFINITE;
  }
  return CFUST_OK;
}

}  // namespace

extern "C" int cfust_em_fit_batched(const double* y, int p, int q, int n_problems,
                                    const int64_t* n_obs, const int* g, double* pi, double* mu,
                                    double* Sigma, double* Delta, double* nu, const double* u,
                                    int n_qmc, const cfust_opts* o, double* loglik_trace,
                                    int* n_iter, int* status) {
  if (n_problems < 1 || !n_obs || !g || !y || !pi || !mu || !Sigma || !Delta || !nu || !u ||
      !loglik_trace || !n_iter || !status)
    return CFUST_EINVAL;
  if (p < 1 || p > kMaxP || q < 1 || q > kMaxQFull || n_qmc < 1) return CFUST_EINVAL;
  int rc = check_opts(o);
  if (rc) return rc;
  cfust_opts def;
  cfust_default_opts(&def);
  if (!o) o = &def;
  if (o->max_iter < 0 || o->reorder) return CFUST_EINVAL;
  BPlan pl;
  if ((rc = make_bplan(n_problems, p, q, n_obs, g, n_qmc, o->precision, o->max_iter,
                       o->nu_mode == CFUST_NU_EXACT, &pl)))
    return rc;
  hipStream_t caller = (hipStream_t)o->stream;
  // a library-owned stream (default priority): graph capture is not allowed
  // on the null stream; the caller's earlier work is awaited first
  if (hipStreamSynchronize(caller) != hipSuccess) return CFUST_EHIP;
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return CFUST_EHIP;
  char* base = nullptr;
  bool owned = false;
  if (o->workspace) {
    if (o->workspace_bytes < pl.total) {
      (void)hipStreamDestroy(st);
      return CFUST_ENOMEM;
    }
    base = (char*)o->workspace;
  } else {
    if (hipMalloc((void**)&base, pl.total) != hipSuccess) {
      (void)hipStreamDestroy(st);
      return CFUST_ENOMEM;
    }
    owned = true;
  }
  BArgs a;
  a.y = y;
  a.pi = pi;
  a.mu = mu;
  a.Sigma = Sigma;
  a.Delta = Delta;
  a.nu = nu;
  a.u = u;
  a.nu_fixed = o->nu_mode == CFUST_NU_FIXED;
  a.fix_delta_zero = o->fix_delta_zero != 0;
  a.nu_lo = o->nu_lo;
  a.nu_hi = o->nu_hi;
  a.tol = o->tol;
  if (o->precision == CFUST_FP32)
    rc = run_batched<float>(pl, base, a, st, o, loglik_trace, n_iter, status);
  else
    rc = run_batched<double>(pl, base, a, st, o, loglik_trace, n_iter, status);
  (void)hipStreamSynchronize(st);
  if (owned) (void)hipFree(base);
  (void)hipStreamDestroy(st);
  return rc;
}

extern "C" int cfust_loglik_rqmc(const double* y, int64_t n, int p, int q, int g,
                                 const double* pi, const double* mu, const double* Sigma,
                                 const double* Delta, const double* nu, const double* u,
                                 int n_qmc, int K, const cfust_opts* o, double* ll, double* mean,
                                 double* std_err) {
  if (K < 1 || !ll || !mean || !std_err || !u || n_qmc < 1) return CFUST_EINVAL;
  hipStream_t st = o ? (hipStream_t)o->stream : nullptr;
  double* dev_ll = nullptr;
  if (hipMallocAsync((void**)&dev_ll, sizeof(double), st) != hipSuccess) return CFUST_ENOMEM;
  int rc = CFUST_OK;
  for (int k = 0; k < K && !rc; ++k) {
    rc = cfust_loglik(y, n, p, q, g, pi, mu, Sigma, Delta, nu,
                      u + (size_t)k * n_qmc * (q + 1), n_qmc, o, dev_ll, nullptr);
    if (!rc && (hipMemcpyAsync(&ll[k], dev_ll, sizeof(double), hipMemcpyDeviceToHost, st) !=
                    hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess))
      rc = CFUST_EHIP;
  }
  (void)hipFreeAsync(dev_ll, st);
  (void)hipStreamSynchronize(st);
  if (rc) return rc;
  double m = 0.0;
  for (int k = 0; k < K; ++k) m += ll[k];
  m /= K;
  double v = 0.0;
  for (int k = 0; k < K; ++k) v += (ll[k] - m) * (ll[k] - m);
  *mean = m;
  *std_err = K > 1 ? sqrt(v / (K - 1) / K) : 0.0;
  return CFUST_OK;
}

extern "C" int cfust_em_fit_multistart(const double* y, int64_t n, int p, int q, int g, int m,
                                       const double* pi0, const double* mu0, const double* Sigma0,
                                       const double* Delta0, const double* nu0, const double* u,
                                       int n_qmc, int burn_in, const cfust_opts* o, double* pi,
                                       double* mu, double* Sigma, double* Delta, double* nu,
                                       double* start_loglik, int* best, double* loglik_trace,
                                       int* n_iter, int* bad_component) {
  if (bad_component) *bad_component = -1;
  int rc = check_dims(n, p, q, g, n_qmc);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  if (q > kMaxQFull) return CFUST_EINVAL;  // the burn-in runs in the batched form
  if (n < 1 || m < 1 || burn_in < 0 || !y || !pi0 || !mu0 || !Sigma0 || !Delta0 || !nu0 || !u ||
      !pi || !mu || !Sigma || !Delta || !nu || !best || !loglik_trace || !n_iter)
    return CFUST_EINVAL;
  cfust_opts def;
  cfust_default_opts(&def);
  if (!o) o = &def;
  hipStream_t st = (hipStream_t)o->stream;
  const size_t ny = (size_t)n * p, sp = (size_t)g, smu = (size_t)g * p,
               sS = (size_t)g * p * p, sD = (size_t)g * p * q;
  // m copies of y and of the starting values (the batched fit updates in place)
  double *yr = nullptr, *pr = nullptr, *mr = nullptr, *Sr = nullptr, *Dr = nullptr, *nr = nullptr;
  bool ok = hipMallocAsync((void**)&yr, m * ny * sizeof(double), st) == hipSuccess &&
            hipMallocAsync((void**)&pr, m * sp * sizeof(double), st) == hipSuccess &&
            hipMallocAsync((void**)&mr, m * smu * sizeof(double), st) == hipSuccess &&
            hipMallocAsync((void**)&Sr, m * sS * sizeof(double), st) == hipSuccess &&
            hipMallocAsync((void**)&Dr, m * sD * sizeof(double), st) == hipSuccess &&
            hipMallocAsync((void**)&nr, m * sp * sizeof(double), st) == hipSuccess;
  std::vector<double> trace((size_t)m * (burn_in + 1));
  std::vector<int> nit((size_t)m), stat((size_t)2 * m);
  std::vector<int64_t> nobs((size_t)m, n);
  std::vector<int> gs((size_t)m, g);
  if (ok) {
    for (int k = 0; k < m; ++k)
      ok = ok && hipMemcpyAsync(yr + k * ny, y, ny * sizeof(double), hipMemcpyDeviceToDevice, st) ==
                     hipSuccess;
    ok = ok &&
         hipMemcpyAsync(pr, pi0, m * sp * sizeof(double), hipMemcpyDeviceToDevice, st) == hipSuccess &&
         hipMemcpyAsync(mr, mu0, m * smu * sizeof(double), hipMemcpyDeviceToDevice, st) == hipSuccess &&
         hipMemcpyAsync(Sr, Sigma0, m * sS * sizeof(double), hipMemcpyDeviceToDevice, st) == hipSuccess &&
         hipMemcpyAsync(Dr, Delta0, m * sD * sizeof(double), hipMemcpyDeviceToDevice, st) == hipSuccess &&
         hipMemcpyAsync(nr, nu0, m * sp * sizeof(double), hipMemcpyDeviceToDevice, st) == hipSuccess;
  }
  if (!ok) rc = CFUST_ENOMEM;
  // the batched fit runs on a stream of its own: the copies must be done
  if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = CFUST_EHIP;
  if (!rc) {
    cfust_opts ob = *o;
    ob.max_iter = burn_in;
    ob.tol = 0.0;  // exactly burn_in iterations
    ob.reorder = 0;  // the batched kernels integrate in the natural order
    ob.surrogate = nullptr;
    ob.workspace = nullptr;
    ob.workspace_bytes = 0;
    rc = cfust_em_fit_batched(yr, p, q, m, nobs.data(), gs.data(), pr, mr, Sr, Dr, nr, u, n_qmc,
                              &ob, trace.data(), nit.data(), stat.data());
  }
  int sel = -1;
  if (!rc) {
    double bestl = -INFINITY;
    for (int k = 0; k < m; ++k) {
      const double l = stat[2 * k] == 0 ? trace[(size_t)k * (burn_in + 1) + nit[k]] : NAN;
      if (start_loglik) start_loglik[k] = l;
      if (std::isfinite(l) && (sel < 0 || l > bestl)) {
        sel = k;
        bestl = l;
      }
    }
    if (sel < 0) rc = CFUST_ENONFINITE;
  }
  if (!rc) {
    *best = sel;
    ok = hipMemcpyAsync(pi, pr + sel * sp, sp * sizeof(double), hipMemcpyDeviceToDevice, st) ==
             hipSuccess &&
         hipMemcpyAsync(mu, mr + sel * smu, smu * sizeof(double), hipMemcpyDeviceToDevice, st) ==
             hipSuccess &&
         hipMemcpyAsync(Sigma, Sr + sel * sS, sS * sizeof(double), hipMemcpyDeviceToDevice, st) ==
             hipSuccess &&
         hipMemcpyAsync(Delta, Dr + sel * sD, sD * sizeof(double), hipMemcpyDeviceToDevice, st) ==
             hipSuccess &&
         hipMemcpyAsync(nu, nr + sel * sp, sp * sizeof(double), hipMemcpyDeviceToDevice, st) ==
             hipSuccess;
    if (!ok) rc = CFUST_EHIP;
  }
  for (double* ptr : {yr, pr, mr, Sr, Dr, nr})
    if (ptr) (void)hipFreeAsync(ptr, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = CFUST_EHIP;
  if (rc) return rc;
  return cfust_em_fit(y, n, p, q, g, pi, mu, Sigma, Delta, nu, u, n_qmc, o, loglik_trace, n_iter,
                      bad_component);
}

extern "C" int cfust_batched_workspace_size(int p, int q, int n_problems, const int64_t* n_obs,
                                            const int* g, int n_qmc, int precision, int max_iter,
                                            size_t* bytes) {
  if (!bytes || n_problems < 1 || !n_obs || !g || p < 1 || p > kMaxP || q < 1 || q > kMaxQFull ||
      n_qmc < 1 || max_iter < 0)
    return CFUST_EINVAL;
  BPlan pl;
  int rc = make_bplan(n_problems, p, q, n_obs, g, n_qmc, precision, max_iter, false, &pl);
  if (rc) return rc;
  *bytes = pl.total;
  return CFUST_OK;
}

extern "C" int cfust_batched_config(int* waves_per_block, int* chunk, int* waves_per_simd,
                                    int* waves_per_pair, int* points_per_wave, double* tuned_ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (waves_per_block) *waves_per_block = g_last.s.wpb;
  if (chunk) *chunk = g_last.s.chunk;
  if (waves_per_simd) *waves_per_simd = g_last.s.wps;
  if (waves_per_pair) *waves_per_pair = g_last.s.split;
  if (points_per_wave) *points_per_wave = g_last.N / g_last.s.split;
  if (tuned_ms) *tuned_ms = g_last.ms;
  return kNumShapes;
}

extern "C" int cfust_batched_shape(int index, int* waves_per_block, int* chunk,
                                   int* waves_per_simd, int* waves_per_pair) {
  if (index < 0 || index >= kNumShapes) return CFUST_EINVAL;
  const Shape& s = kShapes[index];
  if (waves_per_block) *waves_per_block = s.wpb;
  if (chunk) *chunk = s.chunk;
  if (waves_per_simd) *waves_per_simd = s.wps;
  if (waves_per_pair) *waves_per_pair = s.split;
  return CFUST_OK;
}
