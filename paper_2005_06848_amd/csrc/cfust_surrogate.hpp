// E-step with the surrogate network in place of the two GHK integrals.
//
// For pair (j, i) the two integrals of eq. (2) and the truncated moments are
// standardised problems P(V <= h) with V ~ t_q(0, R_i, dof): integral A at
// h^A = D^-1 c sqrt((nu+p)/(nu+d)), dof nu+p, integral B at
// h^B = D^-1 c sqrt((nu+p+2)/(nu+d)), dof nu+p+2, where R_i is the correlation
// matrix of Lambda_i = I - Delta^T Omega^-1 Delta and D = sqrt(diag Lambda).
// The network maps the feature row (h, the q(q-1)/2 correlations above the
// diagonal of R row by row, dof) to (log P(V <= h), E[V | V <= h],
// Cov(V | V <= h) = U^T U with U upper triangular).  A pair whose features leave the
// training range is evaluated by the GHK kernel instead (QMC fallback).
#pragma once
#include "cfust_kernels.hpp"
#include "cfust_mlp.hpp"

namespace cfust {
// every kernel, device function and table has internal linkage: each
// translation unit of the library compiles the ones it uses
namespace {

// training range and standardisation, by value in kernel arguments
struct SurrRange {
  double h_lo, h_hi, dof_lo, dof_hi, r_max, eig_min;
};

// smallest eigenvalue of a symmetric m x m matrix (m <= kMaxQFull) by cyclic
// Jacobi rotations
__device__ double min_eig_sym(double* a, int m) {
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int r = 0; r < m; ++r)
      for (int c = r + 1; c < m; ++c) off += a[r * m + c] * a[r * m + c];
    if (off < 1e-30) break;
    for (int r = 0; r < m; ++r)
      for (int c = r + 1; c < m; ++c) {
        const double arc = a[r * m + c];
        if (fabs(arc) < 1e-300) continue;
        const double th = (a[c * m + c] - a[r * m + r]) / (2.0 * arc);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < m; ++k) {  // columns r, c
          const double akr = a[k * m + r], akc = a[k * m + c];
          a[k * m + r] = cs * akr - sn * akc;
          a[k * m + c] = sn * akr + cs * akc;
        }
        for (int k = 0; k < m; ++k) {  // rows r, c
          const double ark = a[r * m + k], ack = a[c * m + k];
          a[r * m + k] = cs * ark - sn * ack;
          a[c * m + k] = sn * ark + cs * ack;
        }
      }
  }
  double e = a[0];
  for (int k = 1; k < m; ++k) e = fmin(e, a[k * m + k]);
  return e;
}

// One thread per component: range test of R_i and of the two dofs, and the
// constant part of the standardised feature rows:
//   cf[i][0 .. NR)   correlations r_kl (k < l, row by row), standardised
//   cf[i][NR]        dof nu_i + p (integral A), standardised
//   cf[i][NR + 1]    dof nu_i + p + 2 (integral B), standardised
// ok[i] = 1 if the component is inside the training range.  stdv = mx | sx
// (feature column means and deviations, 64 each).
__global__ void surr_comp_kernel(int p, int q, int g, const double* __restrict__ comp,
                                 SurrRange rg, const float* __restrict__ stdv,
                                 float* __restrict__ cf, int* __restrict__ ok) {
  const int i = threadIdx.x;
  if (i >= g) return;
  const CompLayout cl(p, q);
  const double* cp = comp + (size_t)i * cl.stride;
  const double* C = cp + cl.C;
  const int NR = q * (q - 1) / 2;
  const float* mx = stdv;
  const float* sx = stdv + kMlpPad;
  double R[kMaxQFull * kMaxQFull];
  bool in = true;
  int t = 0;
  for (int k = 0; k < q; ++k)
    for (int l = 0; l < q; ++l) {
      double s = 0.0;
      for (int m = 0; m <= min(k, l); ++m) s += C[k * q + m] * C[l * q + m];
      R[k * q + l] = s;
    }
  for (int k = 0; k < q; ++k)
    for (int l = k + 1; l < q; ++l) {
      const double r = R[k * q + l];
      in = in && fabs(r) <= rg.r_max;
      cf[i * 32 + t] = (float)((r - mx[q + t]) / sx[q + t]);
      ++t;
    }
  const double v = cp[cl.nu];
  const double dA = v + p, dB = v + p + 2.0;
  in = in && dA >= rg.dof_lo && dB <= rg.dof_hi;
  cf[i * 32 + NR] = (float)((dA - mx[q + NR]) / sx[q + NR]);
  cf[i * 32 + NR + 1] = (float)((dB - mx[q + NR]) / sx[q + NR]);
  in = in && min_eig_sym(R, q) >= rg.eig_min;
  ok[i] = in ? 1 : 0;
}

// r = y_j - mu_i, squared Mahalanobis distance d under Omega_i and
// c = Delta^T Omega^-1 r (eq. (2)) in one thread; false if y_j is not
// finite.  PM >= p bounds the loops at compile time so that r and z stay in
// registers.
template <int Q, int PM>
__device__ __forceinline__ bool pair_geometry(const double* __restrict__ yj, int p,
                                              const double* __restrict__ mui,
                                              const double* __restrict__ cp, double& d,
                                              double (&c)[Q]) {
  const CompLayout cl(p, Q);
  double r[PM], z[PM];
  bool fin = true;
#pragma unroll
  for (int a = 0; a < PM; ++a) {
    r[a] = 0.0;
    z[a] = 0.0;
    if (a < p) {
      const double ya = yj[a];
      fin = fin && isfinite(ya);
      r[a] = ya - mui[a];
    }
  }
  const double* L = cp + cl.L;
  d = 0.0;
#pragma unroll
  for (int a = 0; a < PM; ++a) {
    if (a < p) {
      double t = r[a];
#pragma unroll
      for (int b = 0; b < a; ++b) t -= L[a * p + b] * z[b];
      z[a] = t / L[a * p + a];
      d += z[a] * z[a];
    }
  }
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    double t = 0.0;
#pragma unroll
    for (int a = 0; a < PM; ++a)
      if (a < p) t += cp[cl.B + a * Q + k] * r[a];
    c[k] = t;
  }
  return fin;
}

// standardised truncation points of integrals A and B (before the GHK
// scaling by 1/C_mm): h_m = c_m / D_m * sqrt((nu + p [+2]) / (nu + d))
template <int Q>
__device__ __forceinline__ void pair_bounds(const double* __restrict__ cp, int p, double d,
                                            const double (&c)[Q], double (&hA)[Q],
                                            double (&hB)[Q]) {
  const CompLayout cl(p, Q);
  const double v = cp[cl.nu];
  const double fa = sqrt((v + p) / (v + d));
  const double fb = sqrt((v + p + 2.0) / (v + d));
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    const double hb = c[m] * cp[cl.Dinv + m];
    hA[m] = hb * fa;
    hB[m] = hb * fb;
  }
}

// bf16 feature row: standardised h | constant part cf (NR + 1 values, the
// last one the row's dof) | zeros; 64 values written as 8 x 16 bytes
template <int Q>
__device__ __forceinline__ void write_feature_row(bf16* __restrict__ row, const double (&h)[Q],
                                                  const float* __restrict__ cf, float dof_std,
                                                  const float* __restrict__ mx,
                                                  const float* __restrict__ sx, bool zero) {
  constexpr int NR = Q * (Q - 1) / 2;
#pragma unroll
  for (int v8 = 0; v8 < kMlpPad / 8; ++v8) {
    bf16 pk[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int col = v8 * 8 + t;
      float x = 0.f;
      if (!zero) {
        if (col < Q)
          x = (float)((h[col] - (double)mx[col]) / (double)sx[col]);
        else if (col < Q + NR)
          x = cf[col - Q];
        else if (col == Q + NR)
          x = dof_std;
      }
      pk[t] = f2bf(x);
    }
    *reinterpret_cast<uint4*>(row + v8 * 8) = *reinterpret_cast<const uint4*>(pk);
  }
}

// One thread per pair of the chunk [c0, c0 + cn): rows 2t (integral A) and
// 2t + 1 (integral B) of X; pairs outside the training range get zero rows,
// inr[t] = 0 and an entry in list (order of the entries is arbitrary).
template <int Q, int PM>
__global__ __launch_bounds__(256) void surr_feat_kernel(
    const double* __restrict__ y, int p, int g, const double* __restrict__ mu,
    const double* __restrict__ comp, int64_t c0, int64_t cn, SurrRange rg,
    const float* __restrict__ stdv, const float* __restrict__ cf, const int* __restrict__ cok,
    bf16* __restrict__ X, unsigned char* __restrict__ inr, int64_t* __restrict__ list,
    unsigned int* __restrict__ count, int* __restrict__ status) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cn) return;
  constexpr int NR = Q * (Q - 1) / 2;
  const int64_t pair = c0 + t;
  const int64_t j = pair / g;
  const int i = (int)(pair - j * g);
  const CompLayout cl(p, Q);
  const double* cp = comp + (size_t)i * cl.stride;
  double d, c[Q], hA[Q], hB[Q];
  const bool fin = pair_geometry<Q, PM>(y + j * p, p, mu + (size_t)i * p, cp, d, c);
  if (!fin) set_status(status, kENonFinite, -1);
  pair_bounds<Q>(cp, p, d, c, hA, hB);
  bool in = fin && cok[i] != 0;
  // bounds above h_hi are lowered to h_hi (the coordinate is then nearly
  // untruncated); bounds below h_lo send the pair to the GHK path
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    hA[m] = fmin(hA[m], rg.h_hi);
    hB[m] = fmin(hB[m], rg.h_hi);
    in = in && hA[m] >= rg.h_lo && hB[m] >= rg.h_lo;
  }
  const float* cfi = cf + i * 32;
  write_feature_row<Q>(X + (size_t)(2 * t) * kMlpPad, hA, cfi, cfi[NR], stdv, stdv + kMlpPad, !in);
  write_feature_row<Q>(X + (size_t)(2 * t + 1) * kMlpPad, hB, cfi, cfi[NR + 1], stdv,
                       stdv + kMlpPad, !in);
  inr[t] = in ? 1 : 0;
  if (!in && fin) {
    const unsigned int slot = atomicAdd(count, 1u);
    list[slot] = pair;
  }
}

// One thread per in-range pair of the chunk: the pair record
//   log(pi_i f_i(y_j)) | e2 | e1 - e2 | e3[Q] | e4 (upper triangle)
// from the network outputs P (rows 2t, 2t + 1; de-standardised with my, sy),
// by the same assembly as the GHK path.
template <int Q, int PM>
__global__ __launch_bounds__(256) void surr_assemble_kernel(
    const double* __restrict__ y, int p, int g, const double* __restrict__ mu,
    const double* __restrict__ comp, int64_t c0, int64_t cn, const float* __restrict__ P,
    const float* __restrict__ stdv, const unsigned char* __restrict__ inr,
    double* __restrict__ pairbuf, int W) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cn || !inr[t]) return;
  constexpr int NT = Q * (Q + 1) / 2;
  const int64_t pair = c0 + t;
  const int64_t j = pair / g;
  const int i = (int)(pair - j * g);
  const CompLayout cl(p, Q);
  const double* cp = comp + (size_t)i * cl.stride;
  double d, c[Q];
  pair_geometry<Q, PM>(y + j * p, p, mu + (size_t)i * p, cp, d, c);
  const float* my = stdv + 2 * kMlpPad;
  const float* sy = stdv + 3 * kMlpPad;
  // integral A: log T only; integral B: the whole label row
  const double logTA =
      (double)P[(size_t)(2 * t) * kMlpPad] * (double)sy[0] + (double)my[0];
  double lb[1 + Q + NT];
  label_row(P + (size_t)(2 * t + 1) * kMlpPad, my, sy, Q, lb);
  const double logTB = lb[0];
  const double v = cp[cl.nu];
  const double aa = 0.5 * (v + p);
  const double bb = 0.5 * (v + d);
  double* rec = pairbuf + (size_t)pair * W;
  rec[0] = cp[cl.kappa] - aa * log1p(d / v) + logTA;
  const double e2 = (aa / bb) * exp(logTB - logTA);
  rec[1] = e2;
  rec[2] = cp[cl.psi_a] - log(bb) - aa / bb;
  const double sc = sqrt((v + d) / (v + p + 2.0));
  double Ds[Q], mx[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    Ds[k] = sc * cp[cl.D + k];
    mx[k] = Ds[k] * lb[1 + k];
  }
#pragma unroll
  for (int k = 0; k < Q; ++k) rec[3 + k] = e2 * (c[k] - mx[k]);
  int u = 0;
#pragma unroll
  for (int a = 0; a < Q; ++a)
#pragma unroll
    for (int b = a; b < Q; ++b) {
      const double m2 = lb[1 + Q + u];
      const double exx = c[a] * c[b] - c[a] * mx[b] - mx[a] * c[b] + Ds[a] * m2 * Ds[b];
      rec[3 + Q + u] = e2 * exx;
      ++u;
    }
  static_assert(3 + Q + NT <= 64, "record width");
}

// GHK fallback for the listed pairs: waves stride over list[0 .. *count)
template <typename T, int Q>
__global__ __launch_bounds__(256) void pair_list_kernel(
    const double* __restrict__ y, int p, int g, const double* __restrict__ mu,
    const double* __restrict__ comp, const T* __restrict__ sA, const T* __restrict__ sB,
    const T* __restrict__ rsB, const T* __restrict__ uT, const T* __restrict__ ubT, int N,
    const int64_t* __restrict__ list, const unsigned int* __restrict__ count,
    double* __restrict__ pairbuf, int W, int* status) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * 4;
  const int64_t cnt = (int64_t)count[0];
  const CompLayout cl(p, Q);
  for (int64_t e = wave; e < cnt; e += nw) {
    const int64_t pair = list[e];
    const int64_t j = pair / g;
    const int i = (int)(pair - j * g);
    double out;
    bool ok = kOk == pair_eval<T, Q, true>(y + j * p, p, mu + (size_t)i * p, comp + (size_t)i * cl.stride,
                                    sA + (size_t)i * N, sB + (size_t)i * N, rsB + (size_t)i * N,
                                    uT, ubT, N, lane, &out);
    if (!ok) {
      if (lane == 0) set_status(status, kENonFinite, -1);
      continue;
    }
    static_assert(record_width<Q, true>() <= 64, "one record entry per lane");
    if (lane < record_width<Q, true>()) pairbuf[pair * W + lane] = out;
  }
}

__global__ void fill_u64_kernel(unsigned long long* p, unsigned long long v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}
__global__ void add_count_kernel(const unsigned int* c, unsigned long long* total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) total[0] += c[0];
}

// raw feature rows of listed pairs (2 per listed pair, A then B), same
// layout as pair_features_kernel
template <int Q, int PM>
__global__ void pair_features_list_kernel(const double* __restrict__ y, int p, int g,
                                          const double* __restrict__ mu,
                                          const double* __restrict__ comp,
                                          const int64_t* __restrict__ pick, int64_t m,
                                          double* __restrict__ out, int* __restrict__ status) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  constexpr int NR = Q * (Q - 1) / 2;
  constexpr int F = Q + NR + 1;
  const int64_t pair = pick[e];
  const int64_t j = pair / g;
  const int i = (int)(pair - j * g);
  const CompLayout cl(p, Q);
  const double* cp = comp + (size_t)i * cl.stride;
  double d, c[Q], hA[Q], hB[Q];
  if (!pair_geometry<Q, PM>(y + j * p, p, mu + (size_t)i * p, cp, d, c))
    set_status(status, kENonFinite, -1);
  pair_bounds<Q>(cp, p, d, c, hA, hB);
  const double* C = cp + cl.C;
  double* oa = out + (size_t)(2 * e) * F;
  double* ob = oa + F;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    oa[k] = hA[k];
    ob[k] = hB[k];
  }
  int t = Q;
  for (int k = 0; k < Q; ++k)
    for (int l = k + 1; l < Q; ++l) {
      double sum = 0.0;
      for (int mm = 0; mm <= k; ++mm) sum += C[k * Q + mm] * C[l * Q + mm];
      oa[t] = sum;
      ob[t] = sum;
      ++t;
    }
  const double v = cp[cl.nu];
  oa[F - 1] = v + p;
  ob[F - 1] = v + p + 2.0;
}

// raw feature rows of every pair (2 per pair, A then B):
// h (Q) | correlations (NR) | dof, doubles
template <int Q, int PM>
__global__ void pair_features_kernel(const double* __restrict__ y, int64_t n, int p, int g,
                                     const double* __restrict__ mu,
                                     const double* __restrict__ comp, double* __restrict__ out,
                                     int* __restrict__ status) {
  const int64_t pair = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pair >= n * g) return;
  constexpr int NR = Q * (Q - 1) / 2;
  constexpr int F = Q + NR + 1;
  const int64_t j = pair / g;
  const int i = (int)(pair - j * g);
  const CompLayout cl(p, Q);
  const double* cp = comp + (size_t)i * cl.stride;
  double d, c[Q], hA[Q], hB[Q];
  if (!pair_geometry<Q, PM>(y + j * p, p, mu + (size_t)i * p, cp, d, c))
    set_status(status, kENonFinite, -1);
  pair_bounds<Q>(cp, p, d, c, hA, hB);
  const double* C = cp + cl.C;
  double* oa = out + (size_t)(2 * pair) * F;
  double* ob = oa + F;
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    oa[m] = hA[m];
    ob[m] = hB[m];
  }
  int t = Q;
  for (int k = 0; k < Q; ++k)
    for (int l = k + 1; l < Q; ++l) {
      double s = 0.0;
      for (int m = 0; m <= k; ++m) s += C[k * Q + m] * C[l * Q + m];
      oa[t] = s;
      ob[t] = s;
      ++t;
    }
  const double v = cp[cl.nu];
  oa[F - 1] = v + p;
  ob[F - 1] = v + p + 2.0;
}


// ---------------------------------------------------------------------------
// Surrogate check: a difference estimator of the E-step totals.  The m
// sampled observations are j_i = floor((2i + 1) n / (2m)), i < m (the same
// every call, so the corrected E-step is a smooth function of the
// parameters); the totals T (partial sums s1..s8 and the log-likelihood) of
// the network E-step are corrected by (n/m) (T_GHK - T_net) over the sample.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t check_obs(int64_t i, int64_t n, int64_t m) {
  return (2 * i + 1) * n / (2 * m);
}

// ysub[i] = y[j_i], rnet[i] = the g records of observation j_i
__global__ void check_gather_kernel(const double* __restrict__ y, int64_t n, int p,
                                    const double* __restrict__ pairbuf, int gW, int64_t m,
                                    double* __restrict__ ysub, double* __restrict__ rnet) {
  const int C = p > gW ? p : gW;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * C) return;
  const int64_t i = t / C;
  const int c = (int)(t - i * C);
  const int64_t j = check_obs(i, n, m);
  if (c < p) ysub[i * p + c] = y[j * p + c];
  if (c < gW) rnet[i * gW + c] = pairbuf[j * gW + c];
}

// cst = net statistics [GS] | net l | GHK statistics [GS] | GHK l
__global__ void check_combine_kernel(const double* __restrict__ cst, int GS, int with_stats,
                                     double scale, double* __restrict__ stats,
                                     double* __restrict__ loglik, const int* __restrict__ status) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (status[0] != kOk) return;
  if (with_stats && e < GS) stats[e] += scale * (cst[GS + 1 + e] - cst[e]);
  if (e == GS) loglik[0] += scale * (cst[2 * GS + 1] - cst[GS]);
}

}  // namespace
}  // namespace cfust
