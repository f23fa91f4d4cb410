// C ABI of the CFUST mixture EM library (see include/cfust.h).
//
// Host side only: argument checks, workspace planning, kernel launches on the
// caller's stream, and the EM driver loop with Aitken's stopping rule
// (section 3.4, Algorithm 4).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include "../../include/cfust.h"
#include "cfust_batched.hpp"
#include "cfust_surrogate.hpp"

#include <stdio.h>

#include <algorithm>
#include <mutex>
#include <vector>

using namespace cfust;

// Surrogate network handle: parameters, optimiser state and standardisation
// on the device, plus the inference and training buffers it grows on demand.
struct cfust_surrogate {
  int q = 0, F = 0, T = 0;
  SurrRange rg{};
  float* params = nullptr;  // [kMlpParams] fp32 master weights
  float* grad = nullptr;    // [kMlpParams]
  float* adm = nullptr;     // Adam first moments
  float* adv = nullptr;     // Adam second moments
  bf16* wb = nullptr;       // [kMlpWeightsBf] bf16 weights
  float* stdv = nullptr;    // [CFUST_SURR_STD] device standardisation
  float* wo = nullptr;      // [64] loss weights per output
  float h_std[CFUST_SURR_STD];
  bool have_std = false;
  int64_t adam_t = 0;
  int em_switch = -1;                      // first GHK E-step of the last cfust_em_fit
  hipStream_t own = nullptr;               // training stream (capturable)
  int64_t* dstep = nullptr;                // device step counter of a training run
  unsigned long long* fb_total = nullptr;  // device: fallback pairs of the last E-step
  // inference buffers (pairs per chunk)
  int64_t cap_pairs = 0;
  bf16* X = nullptr;
  float* P = nullptr;
  unsigned char* inr = nullptr;
  int64_t* list = nullptr;
  unsigned int* count = nullptr;
  float* cf = nullptr;
  int* cok = nullptr;
  // training buffers (rows per minibatch)
  int64_t cap_rows = 0;
  bf16 *tX = nullptr, *tH[3] = {}, *tdPb = nullptr, *tdPlo = nullptr, *tdZb[2] = {},
       *tdZlo[2] = {};
  float *tT = nullptr, *tZ[3] = {}, *tP = nullptr, *tdP = nullptr, *tdZ[2] = {}, *tpart = nullptr,
        *tbpart = nullptr, *tloss = nullptr;
};

namespace {

struct Plan {
  int64_t n;
  int p, q, g, N, prec;
  int W, S, GS, stride;
  int tile, nb, ny;
  int64_t per_block;
  size_t lds_bytes;
  // byte offsets inside the workspace
  bool exact = false;  // exact E[log W | y] (nu_mode EXACT_FD)
  bool reorder = false;  // Genz-Bretz variable order per pair (opts.reorder)
  size_t o_sAp, o_sAm;
  size_t o_status, o_comp, o_uT, o_ubT, o_sA, o_sB, o_rsB, o_pair, o_part, o_pll, o_pitmp, o_mwork,
      o_ll, o_stats, total;
  // waves per pair (pair_part_kernel + pair_finish_kernel when > 1)
  int split = 1;
  size_t o_parts = 0;
  // surrogate check (difference estimator over m sampled observations)
  int64_t check_m = 0;
  int64_t chk_per_block = 0;
  int chk_nb = 0;
  size_t o_chk_y = 0, o_chk_rnet = 0, o_chk_rghk = 0, o_chk_part = 0, o_chk_pll = 0,
         o_chk_stats = 0;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

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

Plan make_plan(int64_t n, int p, int q, int g, int N, int prec, int64_t check_m = 0) {
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
  pl.o_sAp = off;
  off = align_up(off + (size_t)g * N * es);
  pl.o_sAm = off;
  off = align_up(off + (size_t)g * N * es);
  pl.o_pair = off;
  off = align_up(off + (size_t)(n > 0 ? n : 1) * g * pl.W * sizeof(double));
  pl.split = split_of(n * g, N);
  if (pl.split > 1) {
    // widest record: B with moments plus the two exact-nu integrals
    const size_t pw = 2 + 2 + q + (size_t)q * (q + 1) / 2 + 4;
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

struct Ws {
  char* base = nullptr;
  bool owned = false;
  hipStream_t st = nullptr;
  double* prof = nullptr;             // host accumulator, CFUST_PROF_SLOTS entries
  cfust_surrogate* surr = nullptr;    // surrogate network for the pair integrals
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
  precompute_kernel<<<1, kPrecompThreads, precompute_lds_bytes(pl.p, pl.q, pl.g), ws.st>>>(
      pl.p, pl.q, pl.g, pi, Sigma, Delta, mu, nu,
                                         ws.at<double>(pl.o_comp), ws.at<int>(pl.o_status));
  const int q1 = pl.q + 1;
  if (points) {
    int64_t tot = (int64_t)pl.N * q1;
    points_kernel<T><<<(unsigned)((tot + 255) / 256), 256, 0, ws.st>>>(
        u, pl.N, q1, ws.at<T>(pl.o_uT), ws.at<T>(pl.o_ubT), ws.at<int>(pl.o_status));
  }
  const int tables = pl.exact ? 4 : 2;
  int64_t tot = (int64_t)tables * pl.g * pl.N;
  chi_kernel<T><<<(unsigned)((tot + 127) / 128), 128, 0, ws.st>>>(
      ws.at<double>(pl.o_comp), pl.stride, CompLayout(pl.p, pl.q).nu, pl.p, pl.g, u, pl.N, q1,
      ws.at<T>(pl.o_sA), ws.at<T>(pl.o_sB), ws.at<T>(pl.o_rsB), ws.at<T>(pl.o_sAp),
      ws.at<T>(pl.o_sAm), tables, ws.at<int>(pl.o_status));
}

template <typename T, int Q, bool MOM>
void launch_pairs_q(const Ws& ws, const Plan& pl, const double* y, const double* mu) {
  int64_t pairs = pl.n * pl.g;
  if (pairs == 0) return;
  unsigned blocks = (unsigned)((pairs + 3) / 4);
  // Resident waves per SIMD asked of the compiler.  FP64 q <= 4: four (2.5%
  // faster at p=q=4, 48 B/lane of spill outside the point loop).  FP64
  // q = 5, 6: three (3.8% faster at p=q=6 than the compiler's two, despite
  // 192 B/lane of spill).  FP32 q = 5: four (7.6% faster than the
  // compiler's choice at p=q=5).  FP32 q = 6 and larger q keep the
  // compiler's choice (at p=q=6 four waves spill 176 B/lane and are 8%
  // slower).
  constexpr int OCC = (sizeof(T) == 8 && Q <= 4)        ? 4
                      : (sizeof(T) == 8 && (Q == 5 || Q == 6)) ? 3
                      : (sizeof(T) == 4 && Q == 5)             ? 4
                                                               : 0;
  const double* comp = ws.at<double>(pl.o_comp);
  double* pairs_out = ws.at<double>(pl.o_pair);
  int* status = ws.at<int>(pl.o_status);
  const T *sA = ws.at<T>(pl.o_sA), *sB = ws.at<T>(pl.o_sB), *rsB = ws.at<T>(pl.o_rsB);
  const T *uT = ws.at<T>(pl.o_uT), *ubT = ws.at<T>(pl.o_ubT);
  // the exact-nu variants exist for the E-step only (MOM); the ordered ones
  // keep the default occupancy (the ordering adds registers).  Above
  // kMaxQFull only the natural-order kernel exists (the entry points reject
  // the other forms there).
  if (pl.split > 1 && !pl.reorder) {
    const int K = pl.split;
    double* parts = ws.at<double>(pl.o_parts);
    const unsigned pblocks = (unsigned)((pairs * K + 3) / 4);
    if constexpr (MOM && Q <= kMaxQFull) {
      if (pl.exact) {
        pair_part_kernel<T, Q, MOM, OCC, true><<<pblocks, 256, 0, ws.st>>>(
            y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, K, parts, status,
            ws.at<T>(pl.o_sAp), ws.at<T>(pl.o_sAm));
        pair_finish_kernel<T, Q, MOM, true><<<blocks, 256, 0, ws.st>>>(
            y, pl.n, pl.p, pl.g, mu, comp, pl.N, K, parts, pairs_out, pl.W, status);
        return;
      }
    }
    pair_part_kernel<T, Q, MOM, OCC><<<pblocks, 256, 0, ws.st>>>(
        y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, K, parts, status);
    pair_finish_kernel<T, Q, MOM><<<blocks, 256, 0, ws.st>>>(
        y, pl.n, pl.p, pl.g, mu, comp, pl.N, K, parts, pairs_out, pl.W, status);
    return;
  }
  if constexpr (Q > kMaxQFull) {
    pair_kernel<T, Q, MOM><<<blocks, 256, 0, ws.st>>>(
        y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, pairs_out, pl.W, status);
  } else if constexpr (MOM) {
    if (pl.exact && pl.reorder)
      pair_kernel<T, Q, MOM, 0, true, true><<<blocks, 256, 0, ws.st>>>(
          y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, pairs_out, pl.W, status,
          ws.at<T>(pl.o_sAp), ws.at<T>(pl.o_sAm));
    else if (pl.exact)
      pair_kernel<T, Q, MOM, 0, true><<<blocks, 256, 0, ws.st>>>(
          y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, pairs_out, pl.W, status,
          ws.at<T>(pl.o_sAp), ws.at<T>(pl.o_sAm));
    else if (pl.reorder)
      pair_kernel<T, Q, MOM, 0, false, true><<<blocks, 256, 0, ws.st>>>(
          y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, pairs_out, pl.W, status);
    else
      pair_kernel<T, Q, MOM, OCC><<<blocks, 256, 0, ws.st>>>(
          y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, pairs_out, pl.W, status);
  } else {
    if (pl.reorder)
      pair_kernel<T, Q, MOM, 0, false, true><<<blocks, 256, 0, ws.st>>>(
          y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, pairs_out, pl.W, status);
    else
      pair_kernel<T, Q, MOM, OCC><<<blocks, 256, 0, ws.st>>>(
          y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, pairs_out, pl.W, status);
  }
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
    case 9: launch_pairs_q<T, 9, MOM>(ws, pl, y, mu); break;
    case 10: launch_pairs_q<T, 10, MOM>(ws, pl, y, mu); break;
    case 11: launch_pairs_q<T, 11, MOM>(ws, pl, y, mu); break;
    case 12: launch_pairs_q<T, 12, MOM>(ws, pl, y, mu); break;
  }
}

// ---------------------------------------------------------------------------
// surrogate network: matrix-core products and the forward pass
// ---------------------------------------------------------------------------
int64_t round64(int64_t x) { return (x + 63) / 64 * 64; }

// M (rows) on grid x, N / 64 column tiles on grid y, K split over grid z
template <bool TA, bool TB, int MODE, bool SPLIT = false>
void gemm(const bf16* A, const bf16* A2, int lda, const bf16* B, int ldb, int64_t M, int N, int K,
          int splits, Epi ep, hipStream_t st) {
  int kps = K;
  if (splits > 1) {
    kps = ((K + splits - 1) / splits + 31) / 32 * 32;
    splits = (K + kps - 1) / kps;
  } else {
    splits = 1;
  }
  dim3 grid((unsigned)(M / 64), (unsigned)(N / 64), (unsigned)splits);
  gemm_bf16_kernel<TA, TB, MODE, SPLIT><<<grid, 256, 0, st>>>(A, A2, lda, B, ldb, (int)M, N, K,
                                                               kps, ep);
}

// rows (multiple of 64) through the four layers: X -> H[0] -> H[1] -> H[2] ->
// P (fp32, 64 wide); pre-activations kept in Z when given (training)
void mlp_forward(const cfust_surrogate* s, const bf16* X, int64_t rows, bf16* const H[3],
                 float* const* Z, float* P, hipStream_t st) {
  const bf16* in = X;
  for (int l = 0; l < kMlpLayers; ++l) {
    const int K = mlp_k(l), N = mlp_n(l);
    Epi ep{};
    ep.b = s->params + mlp_b_off(l);
    if (l < kMlpLayers - 1) {
      ep.H = H[l];
      ep.Zs = Z ? Z[l] : nullptr;
      ep.ldc = N;
      gemm<false, true, kEpiBiasSilu>(in, nullptr, K, s->wb + mlp_wb_off(l), K, rows, N, K, 1, ep,
                                      st);
      in = H[l];
    } else {
      ep.C = P;
      ep.ldc = N;
      gemm<false, true, kEpiBias>(in, nullptr, K, s->wb + mlp_wb_off(l), K, rows, N, K, 1, ep, st);
    }
  }
}

// inference: all four layers in one kernel per 16 kInferRT rows (the last
// block ragged)
void mlp_infer(const cfust_surrogate* s, const bf16* X, int64_t rows, float* P, hipStream_t st) {
  constexpr int R = 16 * kInferRT;
  if (rows > 0)
    mlp_infer_kernel<kInferRT><<<(unsigned)((rows + R - 1) / R), 256, 0, st>>>(X, rows, s->wb,
                                                                              s->params, P);
}

template <typename X>
bool dev_alloc(X** p, size_t count) {
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  return hipMalloc((void**)p, count * sizeof(X) + 256) == hipSuccess;
}

// inference buffers for `pairs` pairs per chunk (two feature rows each)
int ensure_infer(cfust_surrogate* s, int64_t pairs) {
  if (pairs <= s->cap_pairs) return CFUST_OK;
  const int64_t rows = round64(2 * pairs);
  bool ok = dev_alloc(&s->X, rows * kMlpPad) && dev_alloc(&s->P, rows * kMlpPad) &&
            dev_alloc(&s->inr, pairs) && dev_alloc(&s->list, pairs);
  if (!ok) {
    s->cap_pairs = 0;
    return CFUST_ENOMEM;
  }
  s->cap_pairs = pairs;
  return CFUST_OK;
}

constexpr int64_t kSurrChunkPairs = int64_t(1) << 19;

// E-step pairs through the network; pairs outside the training range through
// the GHK kernel (on a compacted list per chunk)
template <typename T, int Q, int PM>
int launch_surrogate_pairs_q(const Ws& ws, const Plan& pl, const double* y, const double* mu) {
  cfust_surrogate* s = ws.surr;
  const int64_t pairs = pl.n * pl.g;
  if (pairs == 0) return CFUST_OK;
  const int64_t chunk = std::min(pairs, kSurrChunkPairs);
  int rc = ensure_infer(s, chunk);
  if (rc) return rc;
  const double* comp = ws.at<double>(pl.o_comp);
  int* status = ws.at<int>(pl.o_status);
  surr_comp_kernel<<<1, 64, 0, ws.st>>>(pl.p, pl.q, pl.g, comp, s->rg, s->stdv, s->cf, s->cok);
  fill_u64_kernel<<<1, 64, 0, ws.st>>>(s->fb_total, 0ull);
  for (int64_t c0 = 0; c0 < pairs; c0 += chunk) {
    const int64_t cn = std::min(chunk, pairs - c0);
    const unsigned nb = (unsigned)((cn + 255) / 256);
    fill_uint_kernel<<<1, 64, 0, ws.st>>>(s->count, 0u);
    surr_feat_kernel<Q, PM><<<nb, 256, 0, ws.st>>>(y, pl.p, pl.g, mu, comp, c0, cn, s->rg, s->stdv,
                                               s->cf, s->cok, s->X, s->inr, s->list, s->count,
                                               status);
    mlp_infer(s, s->X, round64(2 * cn), s->P, ws.st);
    surr_assemble_kernel<Q, PM><<<nb, 256, 0, ws.st>>>(y, pl.p, pl.g, mu, comp, c0, cn, s->P,
                                                   s->stdv, s->inr, ws.at<double>(pl.o_pair),
                                                   pl.W);
    const unsigned lb = (unsigned)std::min<int64_t>((cn + 3) / 4, 8192);
    pair_list_kernel<T, Q><<<lb, 256, 0, ws.st>>>(
        y, pl.p, pl.g, mu, comp, ws.at<T>(pl.o_sA), ws.at<T>(pl.o_sB), ws.at<T>(pl.o_rsB),
        ws.at<T>(pl.o_uT), ws.at<T>(pl.o_ubT), pl.N, s->list, s->count, ws.at<double>(pl.o_pair),
        pl.W, status);
    add_count_kernel<<<1, 64, 0, ws.st>>>(s->count, s->fb_total);
  }
  return CFUST_OK;
}

template <typename T, int PM>
int launch_surrogate_pairs_p(const Ws& ws, const Plan& pl, const double* y, const double* mu) {
  switch (pl.q) {
    case 1: return launch_surrogate_pairs_q<T, 1, PM>(ws, pl, y, mu);
    case 2: return launch_surrogate_pairs_q<T, 2, PM>(ws, pl, y, mu);
    case 3: return launch_surrogate_pairs_q<T, 3, PM>(ws, pl, y, mu);
    case 4: return launch_surrogate_pairs_q<T, 4, PM>(ws, pl, y, mu);
    case 5: return launch_surrogate_pairs_q<T, 5, PM>(ws, pl, y, mu);
    case 6: return launch_surrogate_pairs_q<T, 6, PM>(ws, pl, y, mu);
    case 7: return launch_surrogate_pairs_q<T, 7, PM>(ws, pl, y, mu);
    case 8: return launch_surrogate_pairs_q<T, 8, PM>(ws, pl, y, mu);
  }
  return CFUST_EINVAL;
}

// thread-per-pair kernels keep p-vectors in registers for p <= 8
template <typename T>
int launch_surrogate_pairs(const Ws& ws, const Plan& pl, const double* y, const double* mu) {
  if (pl.p <= 8) return launch_surrogate_pairs_p<T, 8>(ws, pl, y, mu);
  return launch_surrogate_pairs_p<T, kMaxP>(ws, pl, y, mu);
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
    int rc = launch_surrogate_pairs<T>(ws, pl, y, mu);
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
  if (o->nu_mode == CFUST_NU_EXACT_FD || o->reorder) return CFUST_EINVAL;
  return (s->q == q && s->have_std) ? CFUST_OK : CFUST_EINVAL;
}

// sampled observations of the surrogate check (0: none)
int64_t check_of(const cfust_opts* o) {
  return (o && o->surrogate && o->surrogate_check > 0) ? (int64_t)o->surrogate_check : 0;
}

// forms that exist only up to kMaxQFull
int check_q_forms(const cfust_opts* o, int q) {
  if (!o || q <= kMaxQFull) return CFUST_OK;
  return (o->nu_mode == CFUST_NU_EXACT_FD || o->reorder || o->surrogate) ? CFUST_EINVAL
                                                                          : CFUST_OK;
}

int check_opts(const cfust_opts* o) {
  if (!o) return CFUST_OK;
  if (o->precision != CFUST_FP64 && o->precision != CFUST_FP32) return CFUST_EINVAL;
  if (o->nu_mode != CFUST_NU_OSL && o->nu_mode != CFUST_NU_EXACT_FD &&
      o->nu_mode != CFUST_NU_FIXED)
    return CFUST_EINVAL;
  if (!(o->nu_lo > 0.0) || !(o->nu_hi >= o->nu_lo)) return CFUST_EINVAL;
  if (o->reorder != 0 && o->reorder != 1) return CFUST_EINVAL;
  if (o->surrogate_check < 0) return CFUST_EINVAL;
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
  pl.exact = o && o->nu_mode == CFUST_NU_EXACT_FD;
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
  pl.exact = o && o->nu_mode == CFUST_NU_EXACT_FD;
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
  if (surr) surr->em_switch = -1;
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
    if (conv && ws.surr && !last) {
      ws.surr = nullptr;
      surr->em_switch = t + 1;
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

// ===========================================================================
// batched EM
// ===========================================================================
namespace {

struct Shape {
  int wpb, chunk, wps;  // waves per block, pairs per fetch, waves per SIMD
};
const Shape kShapes[] = {{1, 1, 4}, {1, 4, 4}, {2, 2, 4}, {4, 1, 4}, {4, 4, 4},
                         {1, 1, 8}, {2, 4, 8}, {4, 2, 8}, {1, 16, 4}, {4, 16, 8}};
constexpr int kNumShapes = (int)(sizeof(kShapes) / sizeof(kShapes[0]));

struct LastCfg {
  Shape s{4, 4, 4};
  double ms = 0.0;
};
LastCfg g_last;
std::mutex g_mu;
struct TuneKey {
  int q, N, prec;
  bool operator==(const TuneKey& o) const { return q == o.q && N == o.N && prec == o.prec; }
};
std::vector<std::pair<TuneKey, LastCfg>> g_tuned;

struct BPlan {
  int P, p, q, N, prec, W, S, G, stride, tile, ny, total_blocks, red_total, max_iter;
  int64_t total_obs, total_pairs, total_part;
  std::vector<int64_t> n_off, pair_off, per_blk, part_off;
  std::vector<int> g_off, blk_off, red_off;
  size_t lds_bytes;
  // workspace offsets
  size_t o_noff, o_goff, o_poff, o_boff, o_perb, o_partoff, o_roff, o_active, o_status, o_iter,
      o_niter, o_llcur, o_trace, o_comp, o_uT, o_ubT, o_sA, o_sB, o_rsB, o_pair, o_part, o_pll,
      o_stats, o_pitmp, o_mwork, o_counter, o_pstat, total;
};

int make_bplan(int P, int p, int q, const int64_t* n_obs, const int* g, int N, int prec,
               int max_iter, BPlan* pl) {
  pl->P = P;
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
  size_t per_obs = (size_t)(gmax * pl->W + gmax + p + 1) * sizeof(double);
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

template <typename T, int Q>
void launch_bpair(const BPlan& pl, const BatchDev& b, char* base, const BArgs& a, hipStream_t st,
                  const Shape& sh, unsigned int total, int n_cu) {
  int waves = sh.wps * 4 * n_cu;
  int blocks = std::max(1, waves / sh.wpb);
  bpair_kernel<T, Q><<<blocks, 64 * sh.wpb, 0, st>>>(
      b, a.y, a.mu, (const double*)(base + pl.o_comp), (const T*)(base + pl.o_sA),
      (const T*)(base + pl.o_sB), (const T*)(base + pl.o_rsB), (const T*)(base + pl.o_uT),
      (const T*)(base + pl.o_ubT), pl.N, (double*)(base + pl.o_pair),
      (unsigned int*)(base + pl.o_counter), total, sh.chunk);
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
      (T*)(base + pl.o_sA), (T*)(base + pl.o_sB), (T*)(base + pl.o_rsB));
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

// Autotuner: times the persistent pair kernel of every candidate shape on the
// first pairs of the batch (about 1/8 of the work, at least one full wave of
// fetches) after one warm-up launch, and keeps the fastest.
template <typename T>
LastCfg autotune(const BPlan& pl, const BatchDev& b, char* base, const BArgs& a, hipStream_t st,
                 int n_cu) {
  LastCfg best;
  best.ms = 1e300;
  unsigned int sub = (unsigned int)std::min<int64_t>(pl.total_pairs,
                                                     std::max<int64_t>(pl.total_pairs / 8, 8192));
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  launch_bprepare<T>(pl, b, base, a, st);
  launch_bpair_q<T>(pl, b, base, a, st, kShapes[0], sub, n_cu);
  for (int s = 0; s < kNumShapes; ++s) {
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
  if (tile > 0) {
    if (tile > kNumShapes) return CFUST_EINVAL;
    cfg.s = kShapes[tile - 1];
  } else {
    TuneKey key{pl.q, pl.N, pl.prec};
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
  if (o->max_iter < 0 || o->nu_mode == CFUST_NU_EXACT_FD || o->reorder) return CFUST_EINVAL;
  BPlan pl;
  if ((rc = make_bplan(n_problems, p, q, n_obs, g, n_qmc, o->precision, o->max_iter, &pl))) return rc;
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
    if (ob.nu_mode == CFUST_NU_EXACT_FD) ob.nu_mode = CFUST_NU_OSL;
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
  int rc = make_bplan(n_problems, p, q, n_obs, g, n_qmc, precision, max_iter, &pl);
  if (rc) return rc;
  *bytes = pl.total;
  return CFUST_OK;
}

extern "C" int cfust_batched_config(int* waves_per_block, int* chunk, int* waves_per_simd,
                                    double* tuned_ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (waves_per_block) *waves_per_block = g_last.s.wpb;
  if (chunk) *chunk = g_last.s.chunk;
  if (waves_per_simd) *waves_per_simd = g_last.s.wps;
  if (tuned_ms) *tuned_ms = g_last.ms;
  return kNumShapes;
}

// ===========================================================================
// GHK integrals for a batch of standardised problems
// ===========================================================================
namespace {

template <typename T, int Q>
void launch_ghk_batch_q(int64_t M, const double* h, const double* R, const int* tab, char* base,
                        size_t o_s, size_t o_rs, size_t o_uT, size_t o_ubT, int N, double* out,
                        int* status, hipStream_t st) {
  ghk_batch_kernel<T, Q><<<(unsigned)((M + 3) / 4), 256, 0, st>>>(
      M, h, R, tab, (const T*)(base + o_s), (const T*)(base + o_rs), (const T*)(base + o_uT),
      (const T*)(base + o_ubT), N, out, status);
}

template <typename T>
int run_ghk_batch(int q, int64_t M, const double* h, const double* R, const double* dof,
                  const double* u, int N, double* out, hipStream_t st) {
  // distinct degrees of freedom (host) -> one table pair each
  std::vector<double> hd((size_t)M);
  if (hipMemcpyAsync(hd.data(), dof, M * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return CFUST_EHIP;
  std::vector<double> uniq(hd);
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  if (uniq.size() > 4096) return CFUST_EINVAL;
  std::vector<int> tab((size_t)M);
  for (int64_t s = 0; s < M; ++s)
    tab[s] = (int)(std::lower_bound(uniq.begin(), uniq.end(), hd[s]) - uniq.begin());
  const int nd = (int)uniq.size();
  const size_t es = sizeof(T);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  size_t o_status = take(4 * sizeof(int));
  size_t o_d = take(nd * sizeof(double));
  size_t o_tab = take(M * sizeof(int));
  size_t o_s = take((size_t)nd * N * es);
  size_t o_rs = take((size_t)nd * N * es);
  size_t o_uT = take((size_t)(q + 1) * N * es);
  size_t o_ubT = take((size_t)(q + 1) * N * es);
  char* base = nullptr;
  if (hipMallocAsync((void**)&base, off, st) != hipSuccess) return CFUST_ENOMEM;
  int* status = (int*)(base + o_status);
  fill_int_kernel<<<1, 64, 0, st>>>(status, 4, 0);
  (void)hipMemcpyAsync(base + o_d, uniq.data(), nd * sizeof(double), hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(base + o_tab, tab.data(), M * sizeof(int), hipMemcpyHostToDevice, st);
  int64_t tot = (int64_t)N * (q + 1);
  points_kernel<T><<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(u, N, q + 1, (T*)(base + o_uT),
                                                                  (T*)(base + o_ubT), status);
  int64_t tq = (int64_t)nd * N;
  chi_list_kernel<T><<<(unsigned)((tq + 127) / 128), 128, 0, st>>>(
      (const double*)(base + o_d), nd, u, N, q + 1, (T*)(base + o_s), (T*)(base + o_rs), status);
  const int* tb = (const int*)(base + o_tab);
  switch (q) {
    case 1: launch_ghk_batch_q<T, 1>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
    case 2: launch_ghk_batch_q<T, 2>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
    case 3: launch_ghk_batch_q<T, 3>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
    case 4: launch_ghk_batch_q<T, 4>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
    case 5: launch_ghk_batch_q<T, 5>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
    case 6: launch_ghk_batch_q<T, 6>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
    case 7: launch_ghk_batch_q<T, 7>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
    case 8: launch_ghk_batch_q<T, 8>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
  }
  int rc = launch_check();
  int hs[2] = {0, 0};
  (void)hipMemcpyAsync(hs, status, 2 * sizeof(int), hipMemcpyDeviceToHost, st);
  if (hipStreamSynchronize(st) != hipSuccess) rc = CFUST_EHIP;
  (void)hipFreeAsync(base, st);
  (void)hipStreamSynchronize(st);
  if (rc) return rc;
  if (hs[0] == kOk) return CFUST_OK;
  return hs[0] == kENotPD ? CFUST_ENOTPD : CFUST_EINVAL;
}

}  // namespace

extern "C" int cfust_ghk_batch(int q, int64_t M, const double* h, const double* R,
                               const double* dof, const double* u, int n_qmc, const cfust_opts* o,
                               double* out) {
  if (q < 1 || q > kMaxQFull || M < 0 || n_qmc < 1 || (M > 0 && (!h || !R || !dof || !out)) || !u)
    return CFUST_EINVAL;
  int rc = check_opts(o);
  if (rc) return rc;
  if (o && o->reorder) return CFUST_EINVAL;
  if (M == 0) return CFUST_OK;
  hipStream_t st = o ? (hipStream_t)o->stream : nullptr;
  if (o && o->precision == CFUST_FP32) return run_ghk_batch<float>(q, M, h, R, dof, u, n_qmc, out, st);
  return run_ghk_batch<double>(q, M, h, R, dof, u, n_qmc, out, st);
}

// ===========================================================================
// surrogate network: handle, training, inference
// ===========================================================================
namespace {

// splitmix64 (Steele, Lea & Flood 2014) and Box-Muller normals for the
// weight initialisation and the minibatch shuffles
struct Rng {
  unsigned long long x;
  unsigned long long next() {
    unsigned long long z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u1 = uniform(), u2 = uniform();
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
};

int surr_feat_width(int q) { return q + q * (q - 1) / 2 + 1; }
int surr_targ_width(int q) { return 1 + q + q * (q + 1) / 2; }

void free_surrogate(cfust_surrogate* s) {
  void* ptrs[] = {s->params, s->grad, s->adm,   s->adv,  s->wb,    s->stdv,  s->wo,
                  s->fb_total, s->X,  s->P,     s->inr,   s->list,
                  s->count,  s->cf,   s->cok,   s->tX,   s->tH[0], s->tH[1], s->tH[2],
                  s->tdPb,   s->tdZb[0], s->tdZb[1], s->tT, s->tZ[0], s->tZ[1], s->tZ[2],
                  s->tdPlo,  s->tdZlo[0], s->tdZlo[1],
                  s->tP,     s->tdP,  s->tdZ[0], s->tdZ[1], s->tpart, s->tbpart, s->tloss};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (s->dstep) (void)hipFree(s->dstep);
  if (s->own) (void)hipStreamDestroy(s->own);
  delete s;
}

int refresh_bf16(cfust_surrogate* s, hipStream_t st) {
  weights_to_bf16_kernel<<<(unsigned)((kMlpWeightsBf + 255) / 256), 256, 0, st>>>(s->params, s->wb);
  return launch_check();
}

// buffers of one training minibatch of `rows` rows (multiple of 64)
int ensure_train(cfust_surrogate* s, int64_t rows) {
  if (rows <= s->cap_rows) return CFUST_OK;
  bool ok = dev_alloc(&s->tX, rows * kMlpPad) && dev_alloc(&s->tT, rows * kMlpPad) &&
            dev_alloc(&s->tP, rows * kMlpPad) && dev_alloc(&s->tdP, rows * kMlpPad) &&
            dev_alloc(&s->tdPb, rows * kMlpPad) && dev_alloc(&s->tdPlo, rows * kMlpPad) &&
            dev_alloc(&s->tpart, (size_t)256 * 4096) &&
            dev_alloc(&s->tbpart, (size_t)(rows / 256 + 1) * kMlpHid) &&
            dev_alloc(&s->tloss, rows * kMlpPad / 256 + 1);
  for (int l = 0; l < 3 && ok; ++l)
    ok = dev_alloc(&s->tH[l], rows * kMlpHid) && dev_alloc(&s->tZ[l], rows * kMlpHid);
  for (int l = 0; l < 2 && ok; ++l)
    ok = dev_alloc(&s->tdZ[l], rows * kMlpHid) && dev_alloc(&s->tdZb[l], rows * kMlpHid) &&
         dev_alloc(&s->tdZlo[l], rows * kMlpHid);
  if (!ok) {
    s->cap_rows = 0;
    return CFUST_ENOMEM;
  }
  s->cap_rows = rows;
  return CFUST_OK;
}

// column sums of X[rows][N] into out[N]
void colsum(cfust_surrogate* s, const float* X, int64_t rows, int N, float* out, hipStream_t st) {
  const unsigned chunks = (unsigned)((rows + 255) / 256);
  colsum_part_kernel<<<dim3(N / 64, chunks), 256, 0, st>>>(X, rows, N, s->tbpart);
  sum_slices_kernel<<<(N + 255) / 256, 256, 0, st>>>(s->tbpart, (int)chunks, N, out);
}

// dW (fp32, [N_out][K_in]) = dZ^T H over `rows` rows (dZ as high and low
// bf16 parts), split over the rows
void weight_grad(cfust_surrogate* s, const bf16* dZb, const bf16* dZlo, int n_out,
                 const bf16* Hin, int k_in, int64_t rows, float* out, hipStream_t st) {
  const int tiles = (n_out / 64) * (k_in / 64);
  int splits = (int)std::max<int64_t>(1, std::min<int64_t>(256 / tiles, rows / 128));
  int kps = (int)((rows + splits - 1) / splits + 31) / 32 * 32;
  splits = (int)((rows + kps - 1) / kps);
  Epi ep{};
  ep.C = s->tpart;
  ep.ldc = k_in;
  dim3 grid((unsigned)(n_out / 64), (unsigned)(k_in / 64), (unsigned)splits);
  gemm_bf16_kernel<true, false, kEpiStore, true><<<grid, 256, 0, st>>>(
      dZb, dZlo, n_out, Hin, k_in, n_out, k_in, (int)rows, kps, ep);
  const int64_t n = (int64_t)n_out * k_in;
  sum_slices_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(s->tpart, splits, n, out);
}

// one minibatch already gathered into tX / tT (Bp rows, B valid): forward,
// loss (added to lacc[slot], or lacc[*dstep / per_epoch] when dstep is given)
// and gradient into s->grad
void forward_backward(cfust_surrogate* s, int64_t B, int64_t Bp, float wsum, double* lacc,
                      int slot, hipStream_t st, const int64_t* dstep = nullptr,
                      int64_t per_epoch = 1) {
  mlp_forward(s, s->tX, Bp, s->tH, s->tZ, s->tP, st);
  const unsigned nlb = (unsigned)(Bp * kMlpPad / 256);
  mse_grad_kernel<<<nlb, 256, 0, st>>>(s->tP, s->tT, Bp, B, s->T, s->wo, wsum, s->tdP, s->tdPb,
                                       s->tdPlo, s->tloss);
  if (dstep)
    accumulate_step_kernel<<<1, 256, 0, st>>>(s->tloss, (int)nlb, lacc, dstep, per_epoch);
  else
    accumulate_kernel<<<1, 256, 0, st>>>(s->tloss, (int)nlb, lacc, slot);
  // layer 3 (linear output)
  weight_grad(s, s->tdPb, s->tdPlo, kMlpPad, s->tH[2], kMlpHid, Bp, s->grad + mlp_w_off(3), st);
  colsum(s, s->tdP, Bp, kMlpPad, s->grad + mlp_b_off(3), st);
  const bf16* dzb = s->tdPb;
  const bf16* dzlo = s->tdPlo;
  int nout = kMlpPad;
  int cur = 0;
  for (int l = 2; l >= 0; --l) {
    // dZ_l = (dZ_{l+1} W_{l+1}) * SiLU'(Z_l)
    Epi ep{};
    ep.C = s->tdZ[cur];
    ep.Zs = s->tZ[l];
    ep.H = s->tdZb[cur];
    ep.H2 = s->tdZlo[cur];
    ep.ldc = kMlpHid;
    gemm<false, false, kEpiSiluBwd, true>(dzb, dzlo, nout, s->wb + mlp_wb_off(l + 1), kMlpHid, Bp,
                                          kMlpHid, nout, 1, ep, st);
    const bf16* hin = l > 0 ? s->tH[l - 1] : s->tX;
    const int kin = mlp_k(l);
    weight_grad(s, s->tdZb[cur], s->tdZlo[cur], kMlpHid, hin, kin, Bp, s->grad + mlp_w_off(l), st);
    colsum(s, s->tdZ[cur], Bp, kMlpHid, s->grad + mlp_b_off(l), st);
    dzb = s->tdZb[cur];
    dzlo = s->tdZlo[cur];
    nout = kMlpHid;
    cur ^= 1;
  }
}

float set_loss_weights(cfust_surrogate* s, const float* wo, hipStream_t st) {
  float h[kMlpPad];
  float sum = 0.f;
  for (int o = 0; o < kMlpPad; ++o) {
    h[o] = o < s->T ? (wo ? wo[o] : 1.0f) : 0.0f;
    sum += h[o];
  }
  (void)hipMemcpyAsync(s->wo, h, sizeof(h), hipMemcpyHostToDevice, st);
  (void)hipStreamSynchronize(st);
  return sum;
}

// label rows -> network rows in a stream-ordered temporary (caller frees)
int network_rows(cfust_surrogate* s, const double* targ, int64_t M, hipStream_t st, double** nt) {
  *nt = nullptr;
  if (hipMallocAsync((void**)nt, (size_t)M * s->T * sizeof(double), st) != hipSuccess)
    return CFUST_ENOMEM;
  net_targets_kernel<<<(unsigned)((M + 255) / 256), 256, 0, st>>>(targ, M, s->q, s->T, *nt);
  return launch_check();
}

// standardisation from features and network rows
int set_std_from_data(cfust_surrogate* s, const double* feat, const double* nt, int64_t M,
                      hipStream_t st) {
  col_moments_kernel<<<s->F, 256, 0, st>>>(feat, M, s->F, s->stdv, s->stdv + kMlpPad);
  col_moments_kernel<<<s->T, 256, 0, st>>>(nt, M, s->T, s->stdv + 2 * kMlpPad,
                                           s->stdv + 3 * kMlpPad);
  if (hipMemcpyAsync(s->h_std, s->stdv, sizeof(s->h_std), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return CFUST_EHIP;
  s->have_std = true;
  return CFUST_OK;
}

template <int PM>
void launch_pair_features(int q, unsigned nb, hipStream_t st, const double* y, int64_t n, int p,
                          int g, const double* mu, const double* comp, double* out, int* status) {
  switch (q) {
    case 1: pair_features_kernel<1, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
    case 2: pair_features_kernel<2, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
    case 3: pair_features_kernel<3, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
    case 4: pair_features_kernel<4, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
    case 5: pair_features_kernel<5, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
    case 6: pair_features_kernel<6, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
    case 7: pair_features_kernel<7, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
    case 8: pair_features_kernel<8, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
  }
}

template <int PM>
void launch_features_list(int q, unsigned nb, hipStream_t st, const double* y, int p, int g,
                          const double* mu, const double* comp, const int64_t* pick, int64_t m,
                          double* out, int* status) {
  switch (q) {
    case 1: pair_features_list_kernel<1, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
    case 2: pair_features_list_kernel<2, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
    case 3: pair_features_list_kernel<3, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
    case 4: pair_features_list_kernel<4, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
    case 5: pair_features_list_kernel<5, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
    case 6: pair_features_list_kernel<6, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
    case 7: pair_features_list_kernel<7, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
    case 8: pair_features_list_kernel<8, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
  }
}

struct SurrFileHeader {
  char magic[8];
  int32_t version, q, F, T, hidden, layers;
  int64_t nparams;
  double range[6];
};

}  // namespace

extern "C" {

int cfust_surrogate_create(int q, const double* range, unsigned long long seed,
                           cfust_surrogate** out) {
  if (!out || !range || q < 1 || q > kMaxQFull) return CFUST_EINVAL;
  *out = nullptr;
  if (!(range[0] < range[1]) || !(range[2] > 0.0) || !(range[2] <= range[3]) ||
      !(range[4] > 0.0) || !(range[5] >= 0.0))
    return CFUST_EINVAL;
  static_assert(kMlpParams == CFUST_SURR_PARAMS, "parameter count");
  cfust_surrogate* s = new cfust_surrogate;
  s->q = q;
  s->F = surr_feat_width(q);
  s->T = surr_targ_width(q);
  s->rg = SurrRange{range[0], range[1], range[2], range[3], range[4], range[5]};
  bool ok = dev_alloc(&s->params, kMlpParams) && dev_alloc(&s->grad, kMlpParams) &&
            dev_alloc(&s->adm, kMlpParams) && dev_alloc(&s->adv, kMlpParams) &&
            dev_alloc(&s->wb, kMlpWeightsBf) && dev_alloc(&s->stdv, CFUST_SURR_STD) &&
            dev_alloc(&s->wo, kMlpPad) && dev_alloc(&s->fb_total, 1) &&
            dev_alloc(&s->count, 1) && dev_alloc(&s->cf, kMaxG * 32) && dev_alloc(&s->cok, kMaxG) &&
            dev_alloc(&s->dstep, 1) &&
            hipStreamCreateWithFlags(&s->own, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    free_surrogate(s);
    return CFUST_ENOMEM;
  }
  std::vector<float> w((size_t)kMlpParams, 0.0f);
  Rng rng{seed};
  for (int l = 0; l < kMlpLayers; ++l) {
    const int kv = l == 0 ? s->F : kMlpHid;          // fan-in without padding
    const int nv = l == kMlpLayers - 1 ? s->T : kMlpHid;
    const double sd = l == kMlpLayers - 1 ? sqrt(1.0 / kv) : sqrt(2.0 / kv);
    for (int o = 0; o < nv; ++o)
      for (int i = 0; i < kv; ++i) w[mlp_w_off(l) + (int64_t)o * mlp_k(l) + i] = (float)(sd * rng.normal());
  }
  for (int c = 0; c < CFUST_SURR_STD; ++c) s->h_std[c] = (c / kMlpPad) % 2 == 1 ? 1.0f : 0.0f;
  ok = hipMemcpy(s->params, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice) ==
           hipSuccess &&
       hipMemset(s->adm, 0, kMlpParams * sizeof(float)) == hipSuccess &&
       hipMemset(s->adv, 0, kMlpParams * sizeof(float)) == hipSuccess &&
       hipMemset(s->fb_total, 0, sizeof(unsigned long long)) == hipSuccess &&
       hipMemcpy(s->stdv, s->h_std, sizeof(s->h_std), hipMemcpyHostToDevice) == hipSuccess;
  if (ok) {
    set_loss_weights(s, nullptr, nullptr);
    ok = refresh_bf16(s, nullptr) == CFUST_OK && hipDeviceSynchronize() == hipSuccess;
  }
  if (!ok) {
    free_surrogate(s);
    return CFUST_EHIP;
  }
  *out = s;
  return CFUST_OK;
}

void cfust_surrogate_destroy(cfust_surrogate* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  free_surrogate(s);
}

int cfust_surrogate_train(cfust_surrogate* s, const double* feat, const double* targ, int64_t M,
                          int epochs, int batch, double lr0, double lr1, unsigned long long seed,
                          const float* wo, const cfust_opts* o, double* loss_trace) {
  if (!s || !feat || !targ || M < 1 || epochs < 0 || batch < 64 || batch % 64 || batch > 65536 ||
      !(lr0 > 0.0) || !(lr1 >= 0.0))
    return CFUST_EINVAL;
  hipStream_t st = o ? (hipStream_t)o->stream : nullptr;
  int rc = ensure_train(s, batch);
  if (rc) return rc;
  double* nt = nullptr;
  if ((rc = network_rows(s, targ, M, st, &nt))) {
    if (nt) (void)hipFreeAsync(nt, st);
    return rc;
  }
  if (!s->have_std && (rc = set_std_from_data(s, feat, nt, M, st))) {
    (void)hipFreeAsync(nt, st);
    return rc;
  }
  const float wsum = set_loss_weights(s, wo, st);
  int64_t* idx = nullptr;
  double* lacc = nullptr;
  if (!(wsum > 0.f) || hipMallocAsync((void**)&idx, M * sizeof(int64_t), st) != hipSuccess) {
    (void)hipFreeAsync(nt, st);
    return wsum > 0.f ? CFUST_ENOMEM : CFUST_EINVAL;
  }
  if (hipMallocAsync((void**)&lacc, (epochs + 1) * sizeof(double), st) != hipSuccess) {
    (void)hipFreeAsync(idx, st);
    (void)hipFreeAsync(nt, st);
    return CFUST_ENOMEM;
  }
  (void)hipMemsetAsync(lacc, 0, (epochs + 1) * sizeof(double), st);
  // The run goes on the handle's own stream (capturable): every step is the
  // same launch sequence reading its minibatch offset, loss slot and Adam
  // step from the device counter s->dstep; with opts->graph (default) it is
  // captured once and replayed.  Each epoch takes floor(M / B) minibatches of
  // B = min(batch, M) rows of a fresh shuffle.
  if (hipStreamSynchronize(st) != hipSuccess) rc = CFUST_EHIP;
  hipStream_t ow = s->own;
  const int64_t B = std::min<int64_t>(batch, M);
  const int64_t Bp = round64(B);
  const int64_t steps = M / B;
  const int64_t total = steps * (int64_t)epochs;
  TrainStep ts{s->dstep, steps, total, B, Bp, s->adam_t, lr0, lr1};
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  auto one_step = [&]() {
    gather_step_kernel<<<(unsigned)(Bp * kMlpPad / 256), 256, 0, ow>>>(
        feat, nt, idx, ts, s->F, s->T, s->stdv, s->stdv + kMlpPad, s->stdv + 2 * kMlpPad,
        s->stdv + 3 * kMlpPad, s->tX, s->tT);
    forward_backward(s, B, Bp, wsum, lacc, 0, ow, s->dstep, steps);
    adam_step_kernel<<<(unsigned)((kMlpParams + 255) / 256), 256, 0, ow>>>(
        s->params, s->grad, s->adm, s->adv, kMlpParams, ts, b1, b2, eps);
    weights_to_bf16_kernel<<<(unsigned)((kMlpWeightsBf + 255) / 256), 256, 0, ow>>>(s->params,
                                                                                    s->wb);
    step_inc_kernel<<<1, 64, 0, ow>>>(s->dstep);
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const bool use_graph = !o || o->graph;
  if (!rc && hipMemsetAsync(s->dstep, 0, sizeof(int64_t), ow) != hipSuccess) rc = CFUST_EHIP;
  if (!rc && use_graph && total > 0) {
    if (hipStreamBeginCapture(ow, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      rc = CFUST_EHIP;
    } else {
      one_step();
      if (hipStreamEndCapture(ow, &graph) != hipSuccess ||
          hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
        rc = CFUST_EHIP;
    }
  }
  std::vector<int64_t> perm((size_t)M);
  Rng rng{seed};
  for (int ep = 0; ep < epochs && !rc; ++ep) {
    for (int64_t k = 0; k < M; ++k) perm[k] = k;
    for (int64_t k = M - 1; k > 0; --k) std::swap(perm[k], perm[rng.next() % (uint64_t)(k + 1)]);
    if (hipMemcpyAsync(idx, perm.data(), M * sizeof(int64_t), hipMemcpyHostToDevice, ow) !=
        hipSuccess) {
      rc = CFUST_EHIP;
      break;
    }
    for (int64_t k = 0; k < steps; ++k) {
      if (exec) {
        if (hipGraphLaunch(exec, ow) != hipSuccess) {
          rc = CFUST_EHIP;
          break;
        }
      } else {
        one_step();
      }
    }
    if (!rc) rc = launch_check();
    // the host permutation is rewritten next epoch: wait for the upload
    if (hipStreamSynchronize(ow) != hipSuccess && !rc) rc = CFUST_EHIP;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (hipStreamSynchronize(ow) != hipSuccess && !rc) rc = CFUST_EHIP;
  if (!rc) s->adam_t += total;
  if (!rc && loss_trace && epochs > 0) {
    std::vector<double> h((size_t)epochs);
    if (hipMemcpyAsync(h.data(), lacc, epochs * sizeof(double), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = CFUST_EHIP;
    for (int e = 0; e < epochs; ++e) loss_trace[e] = h[e] / (double)steps;
  }
  (void)hipFreeAsync(idx, st);
  (void)hipFreeAsync(lacc, st);
  (void)hipFreeAsync(nt, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = CFUST_EHIP;
  return rc;
}

int cfust_surrogate_grad(cfust_surrogate* s, const double* feat, const double* targ, int64_t M,
                         const float* wo, const cfust_opts* o, float* grad, double* loss) {
  if (!s || !feat || !targ || !grad || !loss || M < 1 || M > 65536 || !s->have_std)
    return CFUST_EINVAL;
  hipStream_t st = o ? (hipStream_t)o->stream : nullptr;
  const int64_t Bp = round64(M);
  int rc = ensure_train(s, Bp);
  if (rc) return rc;
  const float wsum = set_loss_weights(s, wo, st);
  if (!(wsum > 0.f)) return CFUST_EINVAL;
  double* nt = nullptr;
  if ((rc = network_rows(s, targ, M, st, &nt))) {
    if (nt) (void)hipFreeAsync(nt, st);
    return rc;
  }
  double* lacc = nullptr;
  if (hipMallocAsync((void**)&lacc, sizeof(double), st) != hipSuccess) {
    (void)hipFreeAsync(nt, st);
    return CFUST_ENOMEM;
  }
  (void)hipMemsetAsync(lacc, 0, sizeof(double), st);
  gather_rows_kernel<<<(unsigned)(Bp * kMlpPad / 256), 256, 0, st>>>(
      feat, nt, nullptr, 0, M, Bp, s->F, s->T, s->stdv, s->stdv + kMlpPad, s->stdv + 2 * kMlpPad,
      s->stdv + 3 * kMlpPad, s->tX, s->tT);
  forward_backward(s, M, Bp, wsum, lacc, 0, st);
  rc = launch_check();
  if (!rc && (hipMemcpyAsync(grad, s->grad, kMlpParams * sizeof(float), hipMemcpyDeviceToHost,
                             st) != hipSuccess ||
              hipMemcpyAsync(loss, lacc, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess))
    rc = CFUST_EHIP;
  (void)hipFreeAsync(lacc, st);
  (void)hipFreeAsync(nt, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = CFUST_EHIP;
  return rc;
}

int cfust_surrogate_eval(cfust_surrogate* s, const double* feat, int64_t M, const cfust_opts* o,
                         double* out) {
  if (!s || M < 0 || (M > 0 && (!feat || !out)) || !s->have_std) return CFUST_EINVAL;
  if (M == 0) return CFUST_OK;
  hipStream_t st = o ? (hipStream_t)o->stream : nullptr;
  const int64_t chunk_rows = 2 * kSurrChunkPairs;
  int rc = ensure_infer(s, std::min<int64_t>(kSurrChunkPairs, (M + 1) / 2));
  if (rc) return rc;
  for (int64_t r0 = 0; r0 < M; r0 += chunk_rows) {
    const int64_t B = std::min(chunk_rows, M - r0);
    const int64_t Bp = round64(B);
    gather_rows_kernel<<<(unsigned)(Bp * kMlpPad / 256), 256, 0, st>>>(
        feat, nullptr, nullptr, r0, B, Bp, s->F, s->T, s->stdv, s->stdv + kMlpPad,
        s->stdv + 2 * kMlpPad, s->stdv + 3 * kMlpPad, s->X, nullptr);
    mlp_infer(s, s->X, Bp, s->P, st);
    unstd_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(
        s->P, B, s->T, s->q, s->stdv + 2 * kMlpPad, s->stdv + 3 * kMlpPad, out + r0 * s->T);
  }
  rc = launch_check();
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = CFUST_EHIP;
  return rc;
}

int cfust_surrogate_get_state(const cfust_surrogate* s, float* params, float* stdv) {
  if (!s) return CFUST_EINVAL;
  if (params && hipMemcpy(params, s->params, kMlpParams * sizeof(float), hipMemcpyDeviceToHost) !=
                    hipSuccess)
    return CFUST_EHIP;
  if (stdv) memcpy(stdv, s->h_std, sizeof(s->h_std));
  return CFUST_OK;
}

int cfust_surrogate_set_state(cfust_surrogate* s, const float* params, const float* stdv) {
  if (!s) return CFUST_EINVAL;
  if (params) {
    if (hipMemcpy(s->params, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemset(s->adm, 0, kMlpParams * sizeof(float)) != hipSuccess ||
        hipMemset(s->adv, 0, kMlpParams * sizeof(float)) != hipSuccess)
      return CFUST_EHIP;
    s->adam_t = 0;
    int rc = refresh_bf16(s, nullptr);
    if (rc) return rc;
  }
  if (stdv) {
    for (int c = 0; c < CFUST_SURR_STD; ++c)
      if (!std::isfinite(stdv[c]) || ((c / kMlpPad) % 2 == 1 && !(stdv[c] > 0.f)))
        return CFUST_EINVAL;
    memcpy(s->h_std, stdv, sizeof(s->h_std));
    if (hipMemcpy(s->stdv, s->h_std, sizeof(s->h_std), hipMemcpyHostToDevice) != hipSuccess)
      return CFUST_EHIP;
    s->have_std = true;
  }
  return hipDeviceSynchronize() == hipSuccess ? CFUST_OK : CFUST_EHIP;
}

int cfust_surrogate_save(const cfust_surrogate* s, const char* path) {
  if (!s || !path) return CFUST_EINVAL;
  std::vector<float> w((size_t)kMlpParams);
  int rc = cfust_surrogate_get_state(s, w.data(), nullptr);
  if (rc) return rc;
  SurrFileHeader hd{};
  memcpy(hd.magic, "CFUSTNN1", 8);
  hd.version = 1;
  hd.q = s->q;
  hd.F = s->F;
  hd.T = s->T;
  hd.hidden = kMlpHid;
  hd.layers = kMlpLayers;
  hd.nparams = kMlpParams;
  const SurrRange& r = s->rg;
  const double rr[6] = {r.h_lo, r.h_hi, r.dof_lo, r.dof_hi, r.r_max, r.eig_min};
  memcpy(hd.range, rr, sizeof(rr));
  FILE* f = fopen(path, "wb");
  if (!f) return CFUST_EINVAL;
  bool ok = fwrite(&hd, sizeof(hd), 1, f) == 1 &&
            fwrite(s->h_std, sizeof(float), CFUST_SURR_STD, f) == (size_t)CFUST_SURR_STD &&
            fwrite(w.data(), sizeof(float), w.size(), f) == w.size();
  ok = (fclose(f) == 0) && ok;
  return ok ? CFUST_OK : CFUST_EINVAL;
}

int cfust_surrogate_load(const char* path, cfust_surrogate** out) {
  if (!path || !out) return CFUST_EINVAL;
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return CFUST_EINVAL;
  SurrFileHeader hd{};
  std::vector<float> stdv(CFUST_SURR_STD), w((size_t)kMlpParams);
  bool ok = fread(&hd, sizeof(hd), 1, f) == 1 && memcmp(hd.magic, "CFUSTNN1", 8) == 0 &&
            hd.version == 1 && hd.q >= 1 && hd.q <= kMaxQFull && hd.F == surr_feat_width(hd.q) &&
            hd.T == surr_targ_width(hd.q) && hd.hidden == kMlpHid && hd.layers == kMlpLayers &&
            hd.nparams == kMlpParams &&
            fread(stdv.data(), sizeof(float), CFUST_SURR_STD, f) == (size_t)CFUST_SURR_STD &&
            fread(w.data(), sizeof(float), w.size(), f) == w.size();
  fclose(f);
  if (!ok) return CFUST_EINVAL;
  cfust_surrogate* s = nullptr;
  int rc = cfust_surrogate_create(hd.q, hd.range, 0, &s);
  if (rc) return rc;
  if ((rc = cfust_surrogate_set_state(s, w.data(), stdv.data()))) {
    cfust_surrogate_destroy(s);
    return rc;
  }
  *out = s;
  return CFUST_OK;
}

int64_t cfust_surrogate_fallback_count(const cfust_surrogate* s) {
  if (!s) return -1;
  unsigned long long v = 0;
  if (hipMemcpy(&v, s->fb_total, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return -1;
  return (int64_t)v;
}

int cfust_surrogate_em_switch(const cfust_surrogate* s) { return s ? s->em_switch : -1; }

int cfust_surrogate_adapt(cfust_surrogate* s, const double* y, int64_t n, int p, int q, int g,
                          const double* pi, const double* mu, const double* Sigma,
                          const double* Delta, const double* nu, const double* u, int n_qmc,
                          int64_t samples, int epochs, unsigned long long seed,
                          const cfust_opts* o, double* loss, int64_t* rows) {
  if (loss) *loss = 0.0;
  if (rows) *rows = 0;
  int rc = check_dims(n, p, q, g, n_qmc);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  if (!s || !y || !pi || !mu || !Sigma || !Delta || !nu || !u || n < 1 || samples < 1 ||
      epochs < 0 || s->q != q || !s->have_std)
    return CFUST_EINVAL;
  cfust_opts oo;
  cfust_default_opts(&oo);
  oo.stream = o ? o->stream : nullptr;
  Plan pl = make_plan(0, p, q, g, 1, CFUST_FP64);
  Ws ws;
  if ((rc = acquire(pl, &oo, &ws))) return rc;
  hipStream_t st = ws.st;
  clear_status(ws, pl);
  const double* comp = ws.at<double>(pl.o_comp);
  int* status = ws.at<int>(pl.o_status);
  precompute_kernel<<<1, kPrecompThreads, precompute_lds_bytes(p, q, g), st>>>(
      p, q, g, pi, Sigma, Delta, mu, nu,
                                      ws.at<double>(pl.o_comp), status);
  // uniform sample of pairs (with replacement)
  const int64_t pairs = n * g;
  const int F = s->F, T = s->T;
  std::vector<int64_t> pick((size_t)samples);
  Rng rng{seed * 0x9E3779B97F4A7C15ull + 0x5851F42D4C957F2Dull};
  for (auto& k : pick) k = (int64_t)(rng.next() % (uint64_t)pairs);
  int64_t* pick_d = nullptr;
  double* feat_d = nullptr;
  if (hipMallocAsync((void**)&pick_d, samples * sizeof(int64_t), st) != hipSuccess ||
      hipMallocAsync((void**)&feat_d, (size_t)2 * samples * F * sizeof(double), st) !=
          hipSuccess) {
    if (pick_d) (void)hipFreeAsync(pick_d, st);
    release(&ws);
    return CFUST_ENOMEM;
  }
  (void)hipMemcpyAsync(pick_d, pick.data(), samples * sizeof(int64_t), hipMemcpyHostToDevice, st);
  const unsigned nb = (unsigned)((samples + 127) / 128);
  if (p <= 8)
    launch_features_list<8>(q, nb, st, y, p, g, mu, comp, pick_d, samples, feat_d, status);
  else
    launch_features_list<kMaxP>(q, nb, st, y, p, g, mu, comp, pick_d, samples, feat_d, status);
  std::vector<double> fh((size_t)2 * samples * F);
  rc = launch_check();
  if (!rc && hipMemcpyAsync(fh.data(), feat_d, fh.size() * sizeof(double), hipMemcpyDeviceToHost,
                            st) != hipSuccess)
    rc = CFUST_EHIP;
  if (!rc) rc = fetch_status(ws, pl, nullptr);
  (void)hipFreeAsync(pick_d, st);
  (void)hipFreeAsync(feat_d, st);
  if (rc) {
    release(&ws);
    return rc;
  }
  // rows inside the training range
  const SurrRange& r = s->rg;
  std::vector<double> hs, Rs, dofs, fs;
  for (int64_t k = 0; k < 2 * samples; ++k) {
    const double* f = fh.data() + k * F;
    bool in = f[F - 1] >= r.dof_lo && f[F - 1] <= r.dof_hi;
    for (int a = 0; a < q && in; ++a) in = f[a] >= r.h_lo && f[a] <= r.h_hi;
    for (int a = q; a < F - 1 && in; ++a) in = fabs(f[a]) <= r.r_max;
    if (!in) continue;
    fs.insert(fs.end(), f, f + F);
    hs.insert(hs.end(), f, f + q);
    dofs.push_back(f[F - 1]);
    const size_t b = Rs.size();
    Rs.resize(b + (size_t)q * q);
    int t = q;
    for (int a = 0; a < q; ++a) {
      Rs[b + a * q + a] = 1.0;
      for (int c = a + 1; c < q; ++c, ++t) {
        Rs[b + a * q + c] = f[t];
        Rs[b + c * q + a] = f[t];
      }
    }
  }
  const int64_t M = (int64_t)dofs.size();
  if (rows) *rows = M;
  if (M == 0 || epochs == 0) {
    release(&ws);
    return CFUST_OK;
  }
  double *h_d = nullptr, *R_d = nullptr, *dof_d = nullptr, *f_d = nullptr, *lab_d = nullptr;
  bool ok = hipMallocAsync((void**)&h_d, hs.size() * sizeof(double), st) == hipSuccess &&
            hipMallocAsync((void**)&R_d, Rs.size() * sizeof(double), st) == hipSuccess &&
            hipMallocAsync((void**)&dof_d, dofs.size() * sizeof(double), st) == hipSuccess &&
            hipMallocAsync((void**)&f_d, fs.size() * sizeof(double), st) == hipSuccess &&
            hipMallocAsync((void**)&lab_d, (size_t)M * T * sizeof(double), st) == hipSuccess;
  if (ok) {
    (void)hipMemcpyAsync(h_d, hs.data(), hs.size() * sizeof(double), hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(R_d, Rs.data(), Rs.size() * sizeof(double), hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(dof_d, dofs.data(), dofs.size() * sizeof(double), hipMemcpyHostToDevice,
                         st);
    (void)hipMemcpyAsync(f_d, fs.data(), fs.size() * sizeof(double), hipMemcpyHostToDevice, st);
    rc = run_ghk_batch<double>(q, M, h_d, R_d, dof_d, u, n_qmc, lab_d, st);
    if (!rc) {
      std::vector<float> wo((size_t)T, 1.0f);
      wo[0] = (float)(T - 1);
      std::vector<double> trace((size_t)epochs);
      rc = cfust_surrogate_train(s, f_d, lab_d, M, epochs, 1024, 5e-4, 1e-6, seed, wo.data(), &oo,
                                 trace.data());
      if (!rc && loss) *loss = trace[epochs - 1];
    }
  } else {
    rc = CFUST_ENOMEM;
  }
  for (double* ptr : {h_d, R_d, dof_d, f_d, lab_d})
    if (ptr) (void)hipFreeAsync(ptr, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = CFUST_EHIP;
  release(&ws);
  return rc;
}

int cfust_pair_features(const double* y, int64_t n, int p, int q, int g, const double* pi,
                        const double* mu, const double* Sigma, const double* Delta,
                        const double* nu, const cfust_opts* o, double* out) {
  int rc = check_dims(n, p, q, g, 1);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  if (q > kMaxQFull) return CFUST_EINVAL;
  if ((n > 0 && (!y || !out)) || !pi || !mu || !Sigma || !Delta || !nu) return CFUST_EINVAL;
  Plan pl = make_plan(0, p, q, g, 1, CFUST_FP64);
  Ws ws;
  cfust_opts oo;
  cfust_default_opts(&oo);
  oo.stream = o ? o->stream : nullptr;
  if ((rc = acquire(pl, &oo, &ws))) return rc;
  clear_status(ws, pl);
  const double* comp = ws.at<double>(pl.o_comp);
  int* status = ws.at<int>(pl.o_status);
  precompute_kernel<<<1, kPrecompThreads, precompute_lds_bytes(p, q, g), ws.st>>>(
      p, q, g, pi, Sigma, Delta, mu, nu,
                                         ws.at<double>(pl.o_comp), status);
  const int64_t pairs = n * g;
  const unsigned nb = (unsigned)((pairs + 127) / 128);
  if (pairs > 0) {
    if (p <= 8)
      launch_pair_features<8>(q, nb, ws.st, y, n, p, g, mu, comp, out, status);
    else
      launch_pair_features<kMaxP>(q, nb, ws.st, y, n, p, g, mu, comp, out, status);
  }
  rc = launch_check();
  int stt = fetch_status(ws, pl, nullptr);
  release(&ws);
  return rc ? rc : stt;
}

int cfust_mlp_gemm(int ta, int tb, int M, int N, int K, const unsigned short* A,
                   const unsigned short* B, float* C, void* stream) {
  if (M < 64 || N < 64 || K < 32 || M % 64 || N % 64 || K % 32 || !A || !B || !C)
    return CFUST_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  Epi ep{};
  ep.C = C;
  ep.ldc = N;
  const int lda = ta ? M : K, ldb = tb ? K : N;
  if (!ta && !tb) gemm<false, false, kEpiStore>(A, nullptr, lda, B, ldb, M, N, K, 1, ep, st);
  if (!ta && tb) gemm<false, true, kEpiStore>(A, nullptr, lda, B, ldb, M, N, K, 1, ep, st);
  if (ta && !tb) gemm<true, false, kEpiStore>(A, nullptr, lda, B, ldb, M, N, K, 1, ep, st);
  if (ta && tb) gemm<true, true, kEpiStore>(A, nullptr, lda, B, ldb, M, N, K, 1, ep, st);
  int rc = launch_check();
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = CFUST_EHIP;
  return rc;
}

}  // extern "C"
