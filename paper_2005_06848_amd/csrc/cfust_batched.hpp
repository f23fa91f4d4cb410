// Batched EM: many independent problems (random starts with their own data,
// n and g) advanced together, one iteration = one fixed sequence of kernels
// that needs no host round trip, so it can be captured in a hipGraph and
// replayed (section 3.1, Algorithm 1: parallel starts; sections 3.2-3.4 per
// start).  Per-problem state lives on the device: an active mask (cleared on
// convergence, on reaching max_iter or on an error), the status, the
// iteration counter and the log-likelihood trace.
//
// Work decomposition: pairs of all problems form one index space
// [0, sum_k n_k g_k); a persistent pair kernel pulls chunks of it from an
// atomic counter, so problems of uneven size share the GPU without a tail.
// For small batches the autotuner may split every pair's QMC points over K
// waves (bpart_kernel over the index space of (pair, slice) items, then
// bfinish_kernel per pair).
#pragma once
#include "cfust_kernels.hpp"

namespace cfust {
// every kernel, device function and table has internal linkage: each
// translation unit of the library compiles the ones it uses
namespace {

// Device view of the batch description and per-problem state.
struct BatchDev {
  int P, p, q, W, S;
  const int64_t* n_off;    // [P+1] observation offsets
  const int* g_off;        // [P+1] component offsets
  const int64_t* pair_off; // [P+1] pair offsets
  const int* blk_off;      // [P+1] statistics-block offsets
  const int64_t* per_blk;  // [P] observations per statistics block
  const int64_t* part_off; // [P+1] partial-sum offsets (doubles)
  const int* red_off;      // [P+1] reduction-wave offsets (g_k S + 1 per problem)
  int* active;             // [P]
  int* status;             // [P][2]
  int* iter;               // [P]
  double* ll_cur;          // [P]
  double* trace;           // [P][max_iter+1]
  int* n_iter;             // [P]
};

// index k with off[k] <= x < off[k+1] (off non-decreasing, off[0] = 0)
template <typename I>
__device__ __forceinline__ int find_slot(const I* off, int P, I x) {
  int lo = 0, hi = P;  // invariant: off[lo] <= x < off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ void fail_problem(const BatchDev& b, int k, int code, int comp) {
  b.status[2 * k] = code;
  b.status[2 * k + 1] = comp;
  b.active[k] = 0;
}

// one block per problem: its components' blocks (precompute_block)
__global__ void bprecompute_kernel(BatchDev b, const double* __restrict__ pi,
                                   const double* __restrict__ Sigma,
                                   const double* __restrict__ Delta,
                                   const double* __restrict__ mu, const double* __restrict__ nu,
                                   double* __restrict__ comp) {
  const int k = blockIdx.x;
  // every thread reads the flag before any thread may clear it
  const int live = b.active[k];
  __syncthreads();
  if (!live) return;
  const int c0 = b.g_off[k], g = b.g_off[k + 1] - c0;
  const int i = threadIdx.x;
  const int p = b.p, q = b.q;
  const CompLayout cl(p, q);
  if (i == 0 && !pi_on_simplex(pi + c0, g)) fail_problem(b, k, kEInval, -1);
  // LDS sized by the host for kMaxG components, when it fits
  extern __shared__ double plds[];
  const int rc = precompute_block(p, q, g, pi + c0, nu + c0, mu + (size_t)c0 * p,
                                  Sigma + (size_t)c0 * p * p, Delta + (size_t)c0 * p * q,
                                  comp + (size_t)c0 * cl.stride,
                                  precompute_lds_bytes(p, q, kMaxG) ? plds : nullptr);
  if (i < g && rc != kOk) fail_problem(b, k, rc, i);
}

template <typename T>
__global__ void bchi_kernel(BatchDev b, const double* __restrict__ comp, int comp_stride,
                            int nu_off, int G, const double* __restrict__ u, int N,
                            T* __restrict__ sA, T* __restrict__ sB, T* __restrict__ rsB,
                            T* __restrict__ tA) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)2 * G * N) return;
  int which = (int)(t / ((int64_t)G * N));
  int rem = (int)(t - (int64_t)which * G * N);
  int c = rem / N;
  int kk = rem - c * N;
  int k = find_slot(b.g_off, b.P, c);
  if (!b.active[k]) return;
  double v = comp[(size_t)c * comp_stride + nu_off];
  double dof = v + b.p + (which ? 2.0 : 0.0);
  const double x = chi2_quantile(u[(size_t)kk * (b.q + 1)], dof);
  double s = sqrt(x / dof);
  if (which == 0) {
    sA[(size_t)c * N + kk] = (T)s;
    if (tA) tA[(size_t)c * N + kk] = (T)chi_scale_tangent(x, dof, s);
  } else {
    sB[(size_t)c * N + kk] = (T)s;
    rsB[(size_t)c * N + kk] = (T)(1.0 / s);
  }
}

// Persistent pair kernel: waves take `chunk` consecutive pair indices at a
// time from *counter until the index space is exhausted (every wave exits).
// The loop and slot lookup around pair_eval cost registers.  For FP32 at
// Q = 5 the budget is held at 4 waves per SIMD (128 VGPRs): 7% faster on
// 64 problems of 5000-50000 observations than 3 waves (159 VGPRs), and the
// compiler alone picks 2.  Other Q keep the compiler's choice.  EXACT adds
// the tangent of integral A (exact E[log W | y]; tA the chi-scale tangent).
template <typename T, int Q>
constexpr int bpair_occupancy() {
  return (sizeof(T) == 4 && Q == 5) ? 4 : 1;
}

template <typename T, int Q, bool EXACT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(bpair_occupancy<T, Q>())))
void bpair_kernel(BatchDev b, const double* __restrict__ y,
                             const double* __restrict__ mu, const double* __restrict__ comp,
                             const T* __restrict__ sA, const T* __restrict__ sB,
                             const T* __restrict__ rsB, const T* __restrict__ uT,
                             const T* __restrict__ ubT, int N, double* __restrict__ pairbuf,
                             unsigned int* counter, unsigned int total, int chunk,
                             const T* __restrict__ tA) {
  const int lane = threadIdx.x & 63;
  const CompLayout cl(b.p, Q);
  constexpr int RW = record_width<Q, true>();
  static_assert(RW <= 64, "one record entry per lane");
  // Where the occupancy target is held above the compiler's choice (FP32,
  // Q = 5), the wave-uniform values needed after integral B wait in the
  // wave's LDS slot instead of registers: the spill fell from 144 to 96
  // B/lane and 50 iterations of 64 problems of 5000-50000 observations
  // from 23.56 to 22.62 s.
  constexpr bool kPark = bpair_occupancy<T, Q>() > 1;
  __shared__ double park[kPark ? 4 * (Q + 3) : 1];
  double* const slot =
      park + (kPark ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * (Q + 3) : 0);
  for (;;) {
    unsigned int base = 0;
    if (lane == 0) base = atomicAdd(counter, (unsigned int)chunk);
    base = __builtin_amdgcn_readfirstlane(base);
    if (base >= total) break;
    const unsigned int end = min(total, base + (unsigned int)chunk);
    for (unsigned int t = base; t < end; ++t) {
      const int k = find_slot(b.pair_off, b.P, (int64_t)t);
      if (!b.active[k]) continue;
      const int c0 = b.g_off[k], g = b.g_off[k + 1] - c0;
      const int64_t local = (int64_t)t - b.pair_off[k];
      const int64_t j = local / g;
      const int i = (int)(local - j * g);
      const int c = c0 + i;
      double out;
      bool ok = kOk == pair_eval<T, Q, true, EXACT, false, 0, kPark>(
                           y + (b.n_off[k] + j) * b.p, b.p, mu + (size_t)c * b.p,
                           comp + (size_t)c * cl.stride, sA + (size_t)c * N, sB + (size_t)c * N,
                           rsB + (size_t)c * N, uT, ubT, N, lane, &out,
                           EXACT ? tA + (size_t)c * N : nullptr, nullptr, nullptr, 0, 64, 1,
                           slot);
      if (!ok) {
        if (lane == 0) fail_problem(b, k, kENonFinite, -1);
        continue;
      }
      if (lane < RW) pairbuf[(size_t)t * b.W + lane] = out;
    }
  }
}

// The same index space with each pair's QMC points spread over K waves, for
// batches with too few pairs to keep every SIMD busy to the end: item
// w = t K + s is slice s of pair t, the points s 64 + lane + i 64 K of both
// integrals.  bpart_kernel pulls items from *counter and writes each item's
// exponent-aligned sums to parts[w][part_width]; bfinish_kernel (one wave
// per pair) combines a pair's K records in the order s = 0..K-1 and
// assembles the pair record as bpair_kernel does.  The results differ from
// K = 1 only in the order of the sums.
template <typename T, int Q, bool EXACT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(bpair_occupancy<T, Q>())))
void bpart_kernel(BatchDev b, const double* __restrict__ y, const double* __restrict__ mu,
                  const double* __restrict__ comp, const T* __restrict__ sA,
                  const T* __restrict__ sB, const T* __restrict__ rsB,
                  const T* __restrict__ uT, const T* __restrict__ ubT, int N, int K,
                  double* __restrict__ parts, unsigned int* counter, unsigned int total_items,
                  int chunk, const T* __restrict__ tA) {
  constexpr int PW = part_width<Q, true, EXACT>();
  const int lane = threadIdx.x & 63;
  const CompLayout cl(b.p, Q);
  for (;;) {
    unsigned int base = 0;
    if (lane == 0) base = atomicAdd(counter, (unsigned int)chunk);
    base = __builtin_amdgcn_readfirstlane(base);
    if (base >= total_items) break;
    const unsigned int end = min(total_items, base + (unsigned int)chunk);
    for (unsigned int w = base; w < end; ++w) {
      const unsigned int t = w / (unsigned int)K;
      const int s = (int)(w - t * (unsigned int)K);
      const int k = find_slot(b.pair_off, b.P, (int64_t)t);
      if (!b.active[k]) continue;
      const int c0 = b.g_off[k], g = b.g_off[k + 1] - c0;
      const int64_t local = (int64_t)t - b.pair_off[k];
      const int64_t j = local / g;
      const int c = c0 + (int)(local - j * g);
      double out;
      const bool ok = kOk == pair_eval<T, Q, true, EXACT, false, 1>(
                                 y + (b.n_off[k] + j) * b.p, b.p, mu + (size_t)c * b.p,
                                 comp + (size_t)c * cl.stride, sA + (size_t)c * N,
                                 sB + (size_t)c * N, rsB + (size_t)c * N, uT, ubT, N, lane, &out,
                                 EXACT ? tA + (size_t)c * N : nullptr, nullptr,
                                 parts + (size_t)w * PW, 64 * s, 64 * K, K);
      if (!ok && lane == 0) fail_problem(b, k, kENonFinite, -1);
    }
  }
}

template <typename T, int Q, bool EXACT = false>
__global__ __launch_bounds__(256) void bfinish_kernel(BatchDev b, const double* __restrict__ y,
                                                      const double* __restrict__ mu,
                                                      const double* __restrict__ comp, int N,
                                                      int K, const double* __restrict__ parts,
                                                      double* __restrict__ pairbuf,
                                                      unsigned int total) {
  constexpr int PW = part_width<Q, true, EXACT>();
  constexpr int RW = record_width<Q, true>();
  static_assert(RW <= 64, "one record entry per lane");
  const int lane = threadIdx.x & 63;
  const unsigned int t =
      blockIdx.x * 4u + (unsigned int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (t >= total) return;
  const int k = find_slot(b.pair_off, b.P, (int64_t)t);
  if (!b.active[k]) return;
  const CompLayout cl(b.p, Q);
  const int c0 = b.g_off[k], g = b.g_off[k + 1] - c0;
  const int64_t local = (int64_t)t - b.pair_off[k];
  const int64_t j = local / g;
  const int c = c0 + (int)(local - j * g);
  double out;
  const bool ok = kOk == pair_eval<T, Q, true, EXACT, false, 2>(
                             y + (b.n_off[k] + j) * b.p, b.p, mu + (size_t)c * b.p,
                             comp + (size_t)c * cl.stride, nullptr, nullptr, nullptr, nullptr,
                             nullptr, N, lane, &out, nullptr, nullptr,
                             const_cast<double*>(parts) + (size_t)t * K * PW, 0, 64, K);
  if (!ok) {
    if (lane == 0) fail_problem(b, k, kENonFinite, -1);
    return;
  }
  if (lane < RW) pairbuf[(size_t)t * b.W + lane] = out;
}

// statistics blocks of all problems: block x of problem k covers
// observations [(x - blk_off[k]) per_blk[k], ...) of that problem
__global__ __launch_bounds__(256) void bstats_kernel(BatchDev b, const double* __restrict__ y,
                                                     const double* __restrict__ mu,
                                                     const double* __restrict__ pairbuf, int tile,
                                                     double* __restrict__ partial,
                                                     double* __restrict__ partial_ll) {
  const int blk = blockIdx.x;
  const int k = find_slot(b.blk_off, b.P, blk);
  if (!b.active[k]) return;
  const int c0 = b.g_off[k], g = b.g_off[k + 1] - c0;
  const int GS = g * b.S;
  const int ebase = blockIdx.y * kStatsPerBlock;
  if (ebase >= GS) return;
  const int64_t n = b.n_off[k + 1] - b.n_off[k];
  const int local = blk - b.blk_off[k];
  const int64_t j0 = (int64_t)local * b.per_blk[k];
  const int64_t j1 = min(n, j0 + b.per_blk[k]);
  stats_body(y + b.n_off[k] * b.p, n, b.p, b.q, g, mu + (size_t)c0 * b.p,
             pairbuf + b.pair_off[k] * b.W, b.W, j0, j1, tile, 1, ebase, blockIdx.y == 0, true,
             partial + b.part_off[k] + (int64_t)local * GS, partial_ll + blk, nullptr, nullptr,
             nullptr, nullptr, nullptr, nullptr);
}

// one wave per (problem, statistic) plus one per problem for the log-likelihood
__global__ __launch_bounds__(64) void breduce_kernel(BatchDev b, const double* __restrict__ partial,
                                                     const double* __restrict__ partial_ll,
                                                     double* __restrict__ stats) {
  const int w = blockIdx.x;
  const int k = find_slot(b.red_off, b.P, w);
  if (!b.active[k]) return;
  const int c0 = b.g_off[k], g = b.g_off[k + 1] - c0;
  const int GS = g * b.S;
  const int e = w - b.red_off[k];
  const int nb = b.blk_off[k + 1] - b.blk_off[k];
  const int lane = threadIdx.x;
  double s = 0.0;
  if (e < GS) {
    const double* pk = partial + b.part_off[k];
    for (int x = lane; x < nb; x += 64) s += pk[(size_t)x * GS + e];
  } else {
    for (int x = lane; x < nb; x += 64) s += partial_ll[b.blk_off[k] + x];
  }
  s = wave_sum(s);
  if (lane == 0) {
    if (e < GS)
      stats[(size_t)c0 * b.S + e] = s;
    else
      b.ll_cur[k] = s;
  }
}

// record l^(t), apply Aitken's rule (Algorithm 4) and the iteration cap
__global__ void baitken_kernel(BatchDev b, int max_iter, double tol) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= b.P || !b.active[k]) return;
  const int t = b.iter[k];
  double* tr = b.trace + (size_t)k * (max_iter + 1);
  const double l2 = b.ll_cur[k];
  tr[t] = l2;
  b.n_iter[k] = t;
  bool stop = !isfinite(l2);
  if (stop) b.status[2 * k] = kENonFinite;
  if (!stop && t >= 2) {
    const double l0 = tr[t - 2], l1 = tr[t - 1];
    const double den = l1 - l0;
    const double a = den != 0.0 ? (l2 - l1) / den : 0.0;
    const double linf = l1 + (l2 - l1) / (1.0 - a);
    stop = fabs(linf - l2) < tol;
  }
  if (stop || t >= max_iter)
    b.active[k] = 0;
  else
    b.iter[k] = t + 1;
}

// one block per problem: its components' M-step (mstep_body)
__global__ void bmstep_kernel(BatchDev b, const double* __restrict__ stats, int nu_fixed,
                              int fix_delta_zero, double nu_lo, double nu_hi, double* pi,
                              double* mu, double* Sigma, double* Delta, double* nu,
                              double* __restrict__ pi_tmp, double* __restrict__ mwork) {
  const int k = blockIdx.x;
  if (!b.active[k]) return;
  const int c0 = b.g_off[k], g = b.g_off[k + 1] - c0;
  const int p = b.p, q = b.q;
  const int64_t n = b.n_off[k + 1] - b.n_off[k];
  int* st = b.status + 2 * k;
  // LDS sized by the host for the largest g of the batch, when it fits
  extern __shared__ double mlds[];
  double* wk = mstep_lds_bytes(p, q, kMaxG) ? mlds : mwork + (size_t)c0 * mstep_work_doubles(p, q);
  mstep_body(stats + (size_t)c0 * b.S, n, p, q, g, mu + (size_t)c0 * p,
             Delta + (size_t)c0 * p * q, nu + c0, nu_fixed, fix_delta_zero, nu_lo, nu_hi,
             pi + c0, mu + (size_t)c0 * p, Sigma + (size_t)c0 * p * p, Delta + (size_t)c0 * p * q,
             nu + c0, pi_tmp + c0, wk, st);
  __syncthreads();
  if (threadIdx.x == 0 && st[0] != kOk) b.active[k] = 0;
}

__global__ void binit_state_kernel(BatchDev b, int max_iter) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= b.P) return;
  b.active[k] = 1;
  b.status[2 * k] = kOk;
  b.status[2 * k + 1] = -1;
  b.iter[k] = 0;
  b.n_iter[k] = 0;
  b.ll_cur[k] = 0.0;
  double* tr = b.trace + (size_t)k * (max_iter + 1);
  for (int t = 0; t <= max_iter; ++t) tr[t] = NAN;
}

}  // namespace
}  // namespace cfust
