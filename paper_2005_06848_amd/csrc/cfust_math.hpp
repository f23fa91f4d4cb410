// Device special functions for the CFUST E-step on CDNA (gfx950).
//
// Everything here runs inside the hot kernels, for FP64 and (where it is on
// the integrand path) FP32.  The normal CDF and its complement come from one
// erfc call; tails that leave the double range are carried as a mantissa and
// a power-of-two exponent so that no GHK weight ever underflows to zero.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "cfust_coeffs.hpp"

namespace cfust {
// every kernel, device function and table has internal linkage: each
// translation unit of the library compiles the ones it uses
namespace {

constexpr double kLn2 = 0.69314718055994530942;
constexpr double kSqrtHalf = 0.70710678118654752440;
constexpr double kLogSqrt2Pi = 0.91893853320467274178;
constexpr double kSqrt2Pi = 2.50662827463100050242;
constexpr double kLogPi = 1.14472988584940017414;

// ---------------------------------------------------------------------------
// precision traits of the integrand type T: ldexp and how far the weight
// accumulators may grow above their reference before it is moved.
// ---------------------------------------------------------------------------
template <typename T>
struct Prec;

template <>
struct Prec<double> {
  static __device__ __forceinline__ double ldexp_(double x, int e) { return ldexp(x, e); }
  static constexpr int kRescale = 64;  // accumulators may grow to 2^64 before re-referencing
};

template <>
struct Prec<float> {
  static __device__ __forceinline__ float ldexp_(float x, int e) { return ldexpf(x, e); }
  static constexpr int kRescale = 32;
};

// ---------------------------------------------------------------------------
// One GHK coordinate.  PhiVal holds Phi(ub) = m * 2^n with the exponent n
// carried separately (a double holding an integer), so that no truncation
// probability ever underflows, and the complement ebar = 1 - Phi(ub) with full
// relative accuracy where it can be close to 0 (ub > 0).
// ---------------------------------------------------------------------------
template <typename T>
struct PhiVal {
  T e;        // FP32: Phi(ub) as a plain value (0 when below the float range)
  T m;        // Phi(ub) = m * 2^n
  typename std::conditional<sizeof(T) == 8, double, int>::type n;
  T ebar;     // 1 - Phi(ub)
  bool neg;   // ub < 0
  T ex;       // erfcx(|ub| / sqrt 2)
};

// FP64 building blocks --------------------------------------------------------
constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2Hi = 0.69314718055994528623;   // double(ln 2)
constexpr double kLn2Lo = 2.3190468138462996154e-17; // ln 2 - kLn2Hi

// The address of a coefficient table, as a pointer into the constant address
// space that the compiler cannot see through (an empty asm on the SGPR pair).
// The table's scalar loads then stay next to their use, with immediate
// offsets from this one base: hoisted out of the point loop, the ~75 FP64
// coefficients would not fit the SGPR file and would spill into VGPR lanes.
typedef const __attribute__((address_space(4))) double* const_dptr;
template <int K>
__device__ __forceinline__ const_dptr opaque_table(const double (&c)[K]) {
  const_dptr p = (const_dptr)c;
  asm volatile("" : "+s"(p));
  return p;
}

// Horner steps acc = acc * x + c_k, k = n-1 .. 0, in one asm block, each
// coefficient taken straight from an SGPR pair as the addend of a VOP3
// v_fma_f64.  (Written as plain fma the compiler picks the two-address
// v_fmac_f64, whose addend is the destination register, and copies every
// coefficient into VGPRs first.)  The scalar loads of a block's coefficients
// complete before the block starts, behind one wait: scalar loads return out
// of order, so every wait is for all of them, and a polynomial costs one
// wait per block.  Blocks of up to 16 steps (32 SGPRs).
// Steps per block: 16 measured 2.7% faster than 8 and 1.9% faster than 12 on
// the FP64 pair kernel at p = q = 4 (fewer waits; larger blocks add SGPR
// spills to VGPR lanes)
constexpr int kHornerBlock = 16;
template <int n>
__device__ __forceinline__ double horner_block(double acc, double x, const_dptr c);

// horner_block<n>: n steps in one asm statement, operands %2 .. %(n+1) =
// c[n-1] .. c[0] (one SGPR pair each)
#define CFUST_FMA_STEP(i) "v_fma_f64 %0, %0, %1, %" #i "\n\t"
#define CFUST_HORNER_BLOCK(n, steps, ...)                                              \
  template <>                                                                          \
  __device__ __forceinline__ double horner_block<n>(double acc, double x, const_dptr c) { \
    asm(steps : "+v"(acc) : "v"(x), __VA_ARGS__);                                      \
    return acc;                                                                        \
  }

CFUST_HORNER_BLOCK(1,
                   CFUST_FMA_STEP(2),
                   "s"(c[0]))

CFUST_HORNER_BLOCK(2,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3),
                   "s"(c[1]), "s"(c[0]))

CFUST_HORNER_BLOCK(3,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3) CFUST_FMA_STEP(4),
                   "s"(c[2]), "s"(c[1]), "s"(c[0]))

CFUST_HORNER_BLOCK(4,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3) CFUST_FMA_STEP(4) CFUST_FMA_STEP(5),
                   "s"(c[3]), "s"(c[2]), "s"(c[1]), "s"(c[0]))

CFUST_HORNER_BLOCK(5,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3) CFUST_FMA_STEP(4) CFUST_FMA_STEP(5)
                   CFUST_FMA_STEP(6),
                   "s"(c[4]), "s"(c[3]), "s"(c[2]), "s"(c[1]), "s"(c[0]))

CFUST_HORNER_BLOCK(6,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3) CFUST_FMA_STEP(4) CFUST_FMA_STEP(5)
                   CFUST_FMA_STEP(6) CFUST_FMA_STEP(7),
                   "s"(c[5]), "s"(c[4]), "s"(c[3]), "s"(c[2]), "s"(c[1]), "s"(c[0]))

CFUST_HORNER_BLOCK(7,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3) CFUST_FMA_STEP(4) CFUST_FMA_STEP(5)
                   CFUST_FMA_STEP(6) CFUST_FMA_STEP(7) CFUST_FMA_STEP(8),
                   "s"(c[6]), "s"(c[5]), "s"(c[4]), "s"(c[3]), "s"(c[2]), "s"(c[1]),
                   "s"(c[0]))

CFUST_HORNER_BLOCK(8,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3) CFUST_FMA_STEP(4) CFUST_FMA_STEP(5)
                   CFUST_FMA_STEP(6) CFUST_FMA_STEP(7) CFUST_FMA_STEP(8) CFUST_FMA_STEP(9),
                   "s"(c[7]), "s"(c[6]), "s"(c[5]), "s"(c[4]), "s"(c[3]), "s"(c[2]),
                   "s"(c[1]), "s"(c[0]))

CFUST_HORNER_BLOCK(9,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3) CFUST_FMA_STEP(4) CFUST_FMA_STEP(5)
                   CFUST_FMA_STEP(6) CFUST_FMA_STEP(7) CFUST_FMA_STEP(8) CFUST_FMA_STEP(9)
                   CFUST_FMA_STEP(10),
                   "s"(c[8]), "s"(c[7]), "s"(c[6]), "s"(c[5]), "s"(c[4]), "s"(c[3]),
                   "s"(c[2]), "s"(c[1]), "s"(c[0]))

CFUST_HORNER_BLOCK(10,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3) CFUST_FMA_STEP(4) CFUST_FMA_STEP(5)
                   CFUST_FMA_STEP(6) CFUST_FMA_STEP(7) CFUST_FMA_STEP(8) CFUST_FMA_STEP(9)
                   CFUST_FMA_STEP(10) CFUST_FMA_STEP(11),
                   "s"(c[9]), "s"(c[8]), "s"(c[7]), "s"(c[6]), "s"(c[5]), "s"(c[4]),
                   "s"(c[3]), "s"(c[2]), "s"(c[1]), "s"(c[0]))

CFUST_HORNER_BLOCK(11,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3) CFUST_FMA_STEP(4) CFUST_FMA_STEP(5)
                   CFUST_FMA_STEP(6) CFUST_FMA_STEP(7) CFUST_FMA_STEP(8) CFUST_FMA_STEP(9)
                   CFUST_FMA_STEP(10) CFUST_FMA_STEP(11) CFUST_FMA_STEP(12),
                   "s"(c[10]), "s"(c[9]), "s"(c[8]), "s"(c[7]), "s"(c[6]), "s"(c[5]),
                   "s"(c[4]), "s"(c[3]), "s"(c[2]), "s"(c[1]), "s"(c[0]))

CFUST_HORNER_BLOCK(12,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3) CFUST_FMA_STEP(4) CFUST_FMA_STEP(5)
                   CFUST_FMA_STEP(6) CFUST_FMA_STEP(7) CFUST_FMA_STEP(8) CFUST_FMA_STEP(9)
                   CFUST_FMA_STEP(10) CFUST_FMA_STEP(11) CFUST_FMA_STEP(12) CFUST_FMA_STEP(13),
                   "s"(c[11]), "s"(c[10]), "s"(c[9]), "s"(c[8]), "s"(c[7]), "s"(c[6]),
                   "s"(c[5]), "s"(c[4]), "s"(c[3]), "s"(c[2]), "s"(c[1]), "s"(c[0]))

CFUST_HORNER_BLOCK(13,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3) CFUST_FMA_STEP(4) CFUST_FMA_STEP(5)
                   CFUST_FMA_STEP(6) CFUST_FMA_STEP(7) CFUST_FMA_STEP(8) CFUST_FMA_STEP(9)
                   CFUST_FMA_STEP(10) CFUST_FMA_STEP(11) CFUST_FMA_STEP(12) CFUST_FMA_STEP(13)
                   CFUST_FMA_STEP(14),
                   "s"(c[12]), "s"(c[11]), "s"(c[10]), "s"(c[9]), "s"(c[8]), "s"(c[7]),
                   "s"(c[6]), "s"(c[5]), "s"(c[4]), "s"(c[3]), "s"(c[2]), "s"(c[1]),
                   "s"(c[0]))

CFUST_HORNER_BLOCK(14,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3) CFUST_FMA_STEP(4) CFUST_FMA_STEP(5)
                   CFUST_FMA_STEP(6) CFUST_FMA_STEP(7) CFUST_FMA_STEP(8) CFUST_FMA_STEP(9)
                   CFUST_FMA_STEP(10) CFUST_FMA_STEP(11) CFUST_FMA_STEP(12) CFUST_FMA_STEP(13)
                   CFUST_FMA_STEP(14) CFUST_FMA_STEP(15),
                   "s"(c[13]), "s"(c[12]), "s"(c[11]), "s"(c[10]), "s"(c[9]), "s"(c[8]),
                   "s"(c[7]), "s"(c[6]), "s"(c[5]), "s"(c[4]), "s"(c[3]), "s"(c[2]),
                   "s"(c[1]), "s"(c[0]))

CFUST_HORNER_BLOCK(15,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3) CFUST_FMA_STEP(4) CFUST_FMA_STEP(5)
                   CFUST_FMA_STEP(6) CFUST_FMA_STEP(7) CFUST_FMA_STEP(8) CFUST_FMA_STEP(9)
                   CFUST_FMA_STEP(10) CFUST_FMA_STEP(11) CFUST_FMA_STEP(12) CFUST_FMA_STEP(13)
                   CFUST_FMA_STEP(14) CFUST_FMA_STEP(15) CFUST_FMA_STEP(16),
                   "s"(c[14]), "s"(c[13]), "s"(c[12]), "s"(c[11]), "s"(c[10]), "s"(c[9]),
                   "s"(c[8]), "s"(c[7]), "s"(c[6]), "s"(c[5]), "s"(c[4]), "s"(c[3]),
                   "s"(c[2]), "s"(c[1]), "s"(c[0]))

CFUST_HORNER_BLOCK(16,
                   CFUST_FMA_STEP(2) CFUST_FMA_STEP(3) CFUST_FMA_STEP(4) CFUST_FMA_STEP(5)
                   CFUST_FMA_STEP(6) CFUST_FMA_STEP(7) CFUST_FMA_STEP(8) CFUST_FMA_STEP(9)
                   CFUST_FMA_STEP(10) CFUST_FMA_STEP(11) CFUST_FMA_STEP(12) CFUST_FMA_STEP(13)
                   CFUST_FMA_STEP(14) CFUST_FMA_STEP(15) CFUST_FMA_STEP(16) CFUST_FMA_STEP(17),
                   "s"(c[15]), "s"(c[14]), "s"(c[13]), "s"(c[12]), "s"(c[11]), "s"(c[10]),
                   "s"(c[9]), "s"(c[8]), "s"(c[7]), "s"(c[6]), "s"(c[5]), "s"(c[4]),
                   "s"(c[3]), "s"(c[2]), "s"(c[1]), "s"(c[0]))

#undef CFUST_HORNER_BLOCK
#undef CFUST_FMA_STEP

// sum_j c[j] x^j by Horner's rule, K - 1 fma.  The coefficients are read
// through scalar loads at the point of use (opaque_table keeps the compiler
// from hoisting them out of the point loop, where they would not fit the
// SGPR file) and enter as SGPR operands.  Rounding stays at a few ulp for the
// tables used here (|x| <= 1 with decaying coefficients, or all terms of one
// sign).
template <int K>
__device__ __forceinline__ double horner(const double (&c)[K], double x) {
  static_assert(K >= 2, "horner: at least 2 coefficients");
  const const_dptr cp = opaque_table(c);
  double acc = cp[K - 1];
  // K - 1 steps: blocks of kHornerBlock, then one block of the rest
  constexpr int B = kHornerBlock;
  constexpr int kFull = (K - 1) / B, kRest = (K - 1) % B;
#pragma unroll
  for (int b = 0; b < kFull; ++b) acc = horner_block<B>(acc, x, cp + K - 1 - B - B * b);
  if constexpr (kRest > 0) acc = horner_block<kRest>(acc, x, cp);
  return acc;
}

// 1/x for x > 0 normal: hardware reciprocal plus two Newton steps.
__device__ __forceinline__ double rcp_(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// exp(x) = r * 2^n with n = rint(x / ln 2), |x| <= 2^50.  The reduction uses
// fma so that n * ln2 is subtracted exactly even for large n; exp of the
// reduced argument (|r| <= ln2/2 plus a rounding residual) by its Taylor
// polynomial of degree 13 (truncation below 1e-17).
__constant__ double kExpTaylor[14] = {
    1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720, 1.0 / 5040, 1.0 / 40320,
    1.0 / 362880, 1.0 / 3628800, 1.0 / 39916800, 1.0 / 479001600, 1.0 / 6227020800.0};

__device__ __forceinline__ double exp_split(double x, double* n) {
  double k = rint(x * kLog2e);
  double r = fma(k, -kLn2Hi, x);
  r = fma(k, -kLn2Lo, r);
  *n = k;
  return horner(kExpTaylor, r);
}

// exp(x + xl) = r * 2^n for a small correction xl (|xl| <= ulp(x)): the
// correction joins the reduced argument.
__device__ __forceinline__ double exp_split2(double x, double xl, double* n) {
  double k = rint(x * kLog2e);
  double r = fma(k, -kLn2Hi, x);
  r = fma(k, -kLn2Lo, r) + xl;
  *n = k;
  return horner(kExpTaylor, r);
}

// Natural log of x 2^e for a positive normal double x and an integer-valued
// e: x = m 2^k with m in [1/2, 1).  F_j is m with all but the top 7 bits of
// its fraction cleared (F_j = (1 + j/128) / 2), so d = m - F_j is exact and
// r = d / F_j (with 1/F_j from kLogTab) is below 1/128 in size; then
// log m = log F_j + log1p(r), log1p(r) = r + r^2 P(r) by its series to r^8
// (truncation below 5e-20), and log(x 2^e) = (k + e) ln 2 + log m.  The
// table's log F_j carries a rounding of at most 5.5e-17, so the result is
// within about 1e-16 absolute and 2e-16 relative: near x = 1 (not a case of
// the draws, whose probabilities are at most 1/2) the absolute bound rules.
__constant__ double kLog1pTail[7] = {-1.0 / 2, 1.0 / 3, -1.0 / 4, 1.0 / 5, -1.0 / 6, 1.0 / 7,
                                     -1.0 / 8};
__device__ __forceinline__ double log_(double x, double e = 0.0) {
  int k;
  const double m = frexp(x, &k);
  const unsigned hi = (unsigned)__double2hiint(m);
  const int j = (int)((hi >> 13) & 127u);
  const double F = __hiloint2double((int)(hi & ~0x1FFFu), 0);
  const double d = m - F;
  const LogTab t = kLogTab[j];
  const double r = d * t.inv;
  const double r2 = r * r;
  const double lp = fma(r2, horner(kLog1pTail, r), r);
  const double kd = (double)k + e;
  return fma(kd, kLn2Hi, fma(kd, kLn2Lo, t.lg + lp));
}

// sqrt of x > 0: hardware reciprocal square root (relative error about
// 5e-8) refined by one coupled Newton (Goldschmidt) step for sqrt(x) and
// 1/(2 sqrt(x)), which squares the error to about 4e-15, then a final
// correction on the exact residual x - g^2, which squares it again.
__device__ __forceinline__ double sqrt_(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * y;
  double g = x * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  return fma(d, h, g);
}

// Phi(ub) for FP64, branch-free: with z = |ub| / sqrt 2 and t = 2 / (2 + z),
// erfc(z) = erfcx(z) exp(-z^2) = t Q(2t - 1) exp(-z^2); the exponent of
// exp(-z^2) is kept apart.  z^2 is split into its rounded value and the exact
// residual (fma) so that exp(-z^2) keeps full relative accuracy.  With
// h = t / 2 = 1 / (2 + z): erfc(z) / 2 = h Q(4h - 1) exp(-z^2).
__device__ __forceinline__ PhiVal<double> phi_eval(double ub) {
  double z = fmin(fabs(ub) * kSqrtHalf, 1.0e7);
  double h = rcp_(2.0 + z);
  double exh = h * horner(kErfcxQ, fma(4.0, h, -1.0));  // erfcx(z) / 2
  double zz = z * z;
  double res = fma(z, z, -zz);
  double n;
  double er = exp_split2(-zz, -res, &n);
  double mh = exh * er;  // erfc(z)/2 = mh 2^n
  double small = ldexp(mh, (int)fmax(n, -1100.0));
  PhiVal<double> v;
  v.neg = ub < 0.0;
  v.e = 0.0;
  v.m = v.neg ? mh : 1.0 - small;
  v.n = v.neg ? n : 0.0;
  v.ebar = v.neg ? 1.0 - small : small;
  v.ex = exh + exh;
  return v;
}

// Lower-tail quantile from log p where p is below the rational's range
// (t > kNinvTMax, p < 1e-313): Newton on log Phi(w) - lp with erfcx.
__device__ __noinline__ double ninv_from_log(double lp) {
  double t = -2.0 * lp;
  double w = -sqrt(t - log(t) - 2.0 * kLogSqrt2Pi);
  for (int it = 0; it < 12; ++it) {
    double z = -w * kSqrtHalf;
    double ex = erfcx(z);
    double lphi = log(0.5 * ex) - z * z;
    double slope = 2.0 / (kSqrt2Pi * ex);
    double step = (lphi - lp) / slope;
    w -= step;
    if (fabs(step) <= 1e-16 * fabs(w)) break;
  }
  return w;
}

// eps = Phi^{-1}(u Phi(ub)) for FP64, branch-free outside the deep tail:
// with the lower-half probability a = u Phi(ub) (or its complement
// (1 - u) + u (1 - Phi(ub)) when u Phi(ub) > 1/2) and t = sqrt(-2 log a),
// Phi^{-1}(a) = -t + P(t)/R(t).
__device__ __forceinline__ double draw_eval(double u, double ubar, const PhiVal<double>& v) {
  double um = u * v.m;
  bool lower = v.neg || um <= 0.5;
  double a = lower ? um : fma(u, v.ebar, ubar);
  double nl = lower ? v.n : 0.0;
  double L = log_(a, nl);
  double t2 = -2.0 * L;
  double w;
  if (t2 <= kNinvTMax * kNinvTMax) {
    double t = sqrt_(t2);
    w = fma(horner(kNinvP, t), rcp_(horner(kNinvR, t)), -t);
  } else {
    w = ninv_from_log(L);
  }
  return lower ? w : -w;
}

// FP32 building blocks --------------------------------------------------------
// Same construction as FP64 with hardware v_exp_f32 / v_log_f32 / v_rcp_f32 /
// v_sqrt_f32 and single-precision fits; the exponent of Phi is an int.
constexpr float kSqrtHalfF = 0.70710678118654752f;
constexpr float kLog2eF = 1.44269504088896341f;
constexpr float kLog2eLoF = 1.925963033500011e-08f;  // log2(e) - float(log2(e))
constexpr float kLn2F = 0.69314718055994531f;

template <int K>
__device__ __forceinline__ float poly_f(const float (&c)[K], float x) {
  float r = c[K - 1];
#pragma unroll
  for (int j = K - 2; j >= 0; --j) r = fmaf(r, x, c[j]);
  return r;
}

__device__ __forceinline__ PhiVal<float> phi_eval(float ub) {
  float z = fminf(fabsf(ub) * kSqrtHalfF, 2000.0f);
  float t = 2.0f * __builtin_amdgcn_rcpf(2.0f + z);
  float ex = t * poly_f(kErfcxQf, fmaf(2.0f, t, -1.0f));
  float zz = z * z;
  float res = fmaf(z, z, -zz);
  // exp(-zz - res) = 2^k * 2^r: k = rint(-zz log2 e), r with a two-part log2 e
  float k = rintf(-zz * kLog2eF);
  float r = fmaf(-zz, kLog2eF, -k);
  r = fmaf(-zz, kLog2eLoF, r);
  r = fmaf(-res, kLog2eF, r);
  float mh = 0.5f * ex * __builtin_amdgcn_exp2f(r);  // erfc(z)/2 = mh 2^k
  int n = (int)k;
  float small = ldexpf(mh, max(n, -160));
  PhiVal<float> v;
  v.neg = ub < 0.0f;
  v.m = v.neg ? mh : 1.0f - small;
  v.n = v.neg ? n : 0;
  v.ebar = v.neg ? 1.0f - small : small;
  v.e = v.neg ? small : v.m;
  v.ex = ex;
  return v;
}

__device__ __noinline__ double deep_draw_f(double lp) { return ninv_from_log(lp); }

__device__ __forceinline__ float draw_eval(float u, float ubar, const PhiVal<float>& v) {
  float um = u * v.m;
  bool lower = v.neg || um <= 0.5f;
  float a = lower ? um : fmaf(u, v.ebar, ubar);
  float L2 = __builtin_amdgcn_logf(a) + (lower ? (float)v.n : 0.0f);  // log2 of the probability
  float t2 = (-2.0f * kLn2F) * L2;
  float w;
  if (t2 <= kNinvTMaxF * kNinvTMaxF) {
    float t = __builtin_amdgcn_sqrtf(t2);
    w = fmaf(poly_f(kNinvPf, t), __builtin_amdgcn_rcpf(poly_f(kNinvRf, t)), -t);
  } else {
    w = (float)deep_draw_f((double)L2 * kLn2);
  }
  return lower ? w : -w;
}

// ---------------------------------------------------------------------------
// Pieces of the derivative of a GHK weight (the exact E[log W | y]).
// ---------------------------------------------------------------------------
constexpr double kSqrt2OverPi = 0.79788456080286535588;  // sqrt(2 / pi)

// phi(ub) / Phi(ub) from the pieces of phi_eval, with z = |ub| / sqrt 2 and
// ex = erfcx(z): below zero Phi(ub) = ex exp(-z^2) / 2 and phi(ub) =
// exp(-z^2) / sqrt(2 pi), so the ratio is sqrt(2/pi) / ex; above zero
// ebar = 1 - Phi(ub) = ex exp(-z^2) / 2 gives phi(ub) = sqrt(2/pi) ebar / ex
// and the ratio sqrt(2/pi) ebar / (ex Phi(ub)).
__device__ __forceinline__ double mills(const PhiVal<double>& v) {
  const double num = v.neg ? 1.0 : v.ebar;
  const double den = v.neg ? v.ex : v.ex * v.m;
  return kSqrt2OverPi * num * rcp_(den);
}
__device__ __forceinline__ float mills(const PhiVal<float>& v) {
  const float num = v.neg ? 1.0f : v.ebar;
  const float den = v.neg ? v.ex : v.ex * v.m;
  return (float)kSqrt2OverPi * num * __builtin_amdgcn_rcpf(den);
}

// phi(ub) / phi(eps) = exp((eps^2 - ub^2) / 2), the argument clamped to a
// range where the result is 0 or finite.
__device__ __forceinline__ double dens_ratio(double eps, double ub) {
  const double x = fmin(fmax(0.5 * (eps - ub) * (eps + ub), -1000.0), 700.0);
  double n;
  const double r = exp_split(x, &n);
  return ldexp(r, (int)n);
}
__device__ __forceinline__ float dens_ratio(float eps, float ub) {
  const float x = fminf(fmaxf(0.5f * (eps - ub) * (eps + ub), -100.0f), 80.0f);
  return __builtin_amdgcn_exp2f(x * kLog2eF);
}

// ---------------------------------------------------------------------------
// regularised incomplete gamma and the chi-square quantile (FP64)
// ---------------------------------------------------------------------------
// Lower and upper regularised incomplete gamma P(a,x), Q(a,x): power series
// of P below x = a + 1, Lentz continued fraction of Q above.
__device__ void inc_gamma(double a, double x, double lga, double* P, double* Q) {
  if (!(x > 0.0)) {
    *P = 0.0;
    *Q = 1.0;
    return;
  }
  double lead = exp(a * log(x) - x - lga);
  if (x < a + 1.0) {
    double term = 1.0 / a;
    double sum = term;
    double ak = a;
    for (int k = 0; k < 4000; ++k) {
      ak += 1.0;
      term *= x / ak;
      sum += term;
      if (fabs(term) < 1e-17 * sum) break;
    }
    *P = lead * sum;
    *Q = 1.0 - *P;
  } else {
    const double tiny = 1e-300;
    double b = x + 1.0 - a;
    double cc = 1.0 / tiny;
    double dd = 1.0 / b;
    double f = dd;
    for (int k = 1; k < 4000; ++k) {
      double an = k * (a - k);
      b += 2.0;
      dd = fma(an, dd, b);
      if (fabs(dd) < tiny) dd = tiny;
      cc = b + an / cc;
      if (fabs(cc) < tiny) cc = tiny;
      dd = 1.0 / dd;
      double delta = dd * cc;
      f *= delta;
      if (fabs(delta - 1.0) <= 2.3e-16) break;
    }
    *Q = lead * f;
    *P = 1.0 - *Q;
  }
}

// Chi-square quantile with `dof` degrees of freedom at probability u.
// Halley iterations on the gamma CDF (or on its complement above the median)
// inside a shrinking bracket, from a Wilson-Hilferty start.
__device__ double chi2_quantile(double u, double dof) {
  double a = 0.5 * dof;
  double lga = lgamma(a);
  double z = normcdfinv(u);
  double c = 1.0 / (9.0 * a);
  double wh = 1.0 - c + z * sqrt(c);
  double x = a * wh * wh * wh;
  if (!(x > 0.0)) x = a * exp((log(u) + lgamma(a + 1.0)) / a);  // small-x series start
  if (!(x > 0.0)) x = 1e-300;
  double lo = 0.0, hi = 1e308;
  bool upper = u > 0.5;
  double target = upper ? (1.0 - u) : u;
  for (int it = 0; it < 100; ++it) {
    double P, Q;
    inc_gamma(a, x, lga, &P, &Q);
    double r = upper ? (target - Q) : (P - target);  // increasing in x
    if (r < 0.0)
      lo = x;
    else
      hi = x;
    double dens = exp((a - 1.0) * log(x) - x - lga);
    // Halley's third-order step: the density's log-derivative is
    // (a - 1)/x - 1.  About 3 evaluations of P, Q per quantile instead of
    // Newton's 3.6-4.1, and at most 8 instead of up to 24 (a wave waits for
    // its slowest lane); a step that leaves the bracket falls back below.
    double step = r / dens;
    step = step / (1.0 - 0.5 * step * ((a - 1.0) / x - 1.0));
    double xn = x - step;
    // converged: the Newton step is at rounding level, or the bracket has
    // shrunk to a few ulp (P and Q carry ~1e-15 absolute rounding)
    if (fabs(step) <= 1e-15 * x || hi - lo <= 4e-16 * x) {
      x = xn > lo && xn < hi ? xn : x;
      break;
    }
    if (!(xn > lo && xn < hi)) xn = (hi < 1e308) ? 0.5 * (lo + hi) : 4.0 * x;
    x = xn;
  }
  return 2.0 * x;
}

// Derivative of the chi-square quantile x (P(dof/2, x/2) = u) in the degrees
// of freedom.  With a = dof/2 and z = x/2, implicit differentiation gives
// dz/da = -(dP/da) / (dP/dz) and dx/d(dof) = dz/da, where
// dP/dz = z^(a-1) e^-z / Gamma(a) and, term by term from the series of P,
// dP/da = sum_k w_k (log z - psi(a+k+1)), w_k = e^-z z^(a+k) / Gamma(a+k+1).
// The terms follow by recurrence (w_k = w_{k-1} z / (a+k),
// psi(a+k+1) = psi(a+k) + 1/(a+k)) and stop past their peak once below 1e-20.
__device__ double digamma_(double x);
__device__ double chi2_quantile_ddof(double x, double dof) {
  const double a = 0.5 * dof, z = 0.5 * x, lz = log(z);
  double w = exp(a * lz - z - lgamma(a + 1.0));
  double ps = digamma_(a + 1.0);
  double sum = w * (lz - ps);
  for (int k = 1; k < 100000; ++k) {
    const double ak = a + k;
    w *= z / ak;
    ps += 1.0 / ak;
    sum += w * (lz - ps);
    if (ak > z && w < 1e-20) break;
  }
  const double dPdz = exp((a - 1.0) * lz - z - lgamma(a));
  return -sum / dPdz;
}

// Tangent of the chi scale of integral A in a' = dof'/2 at a' = a: the bounds
// of J(a') are s(a') h sqrt(a'/a) with s(a') = sqrt(x(2a') / (2a')), so the
// factor of h moves at 2 ds/d(dof) + s / dof, with
// ds/d(dof) = (dx/d(dof) / dof - x / dof^2) / (2 s).
__device__ double chi_scale_tangent(double x, double dof, double s) {
  const double dx = chi2_quantile_ddof(x, dof);
  const double ds = (dx / dof - x / (dof * dof)) / (2.0 * s);
  return 2.0 * ds + s / dof;
}

// ---------------------------------------------------------------------------
// digamma and trigamma (FP64): recurrence to x >= 8, then the asymptotic
// expansions in 1/x^2.
// ---------------------------------------------------------------------------
__device__ double digamma_(double x) {
  if (!(x > 0.0) || !(x < 1e300)) return NAN;
  double acc = 0.0;
  while (x < 8.0) {
    acc -= 1.0 / x;
    x += 1.0;
  }
  double r = 1.0 / x;
  double r2 = r * r;
  double series =
      r2 * (1.0 / 12 -
            r2 * (1.0 / 120 -
                  r2 * (1.0 / 252 -
                        r2 * (1.0 / 240 - r2 * (1.0 / 132 - r2 * (691.0 / 32760 - r2 / 12.0))))));
  return acc + log(x) - 0.5 * r - series;
}

__device__ double trigamma_(double x) {
  if (!(x > 0.0) || !(x < 1e300)) return NAN;
  double acc = 0.0;
  while (x < 8.0) {
    acc += 1.0 / (x * x);
    x += 1.0;
  }
  double r = 1.0 / x;
  double r2 = r * r;
  double series = r * (1.0 + r * (0.5 + r * (1.0 / 6 - r2 * (1.0 / 30 - r2 * (1.0 / 42 - r2 * (1.0 / 30 - r2 * 5.0 / 66))))));
  return acc + series;
}

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// value of v in lane src (src wave-uniform)
__device__ __forceinline__ double wave_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

}  // namespace
}  // namespace cfust
