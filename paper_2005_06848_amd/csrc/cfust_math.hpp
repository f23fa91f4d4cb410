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

namespace cfust {

constexpr double kLn2 = 0.69314718055994530942;
constexpr double kSqrtHalf = 0.70710678118654752440;
constexpr double kLogSqrt2Pi = 0.91893853320467274178;
constexpr double kSqrt2Pi = 2.50662827463100050242;
constexpr double kLogPi = 1.14472988584940017414;

// ---------------------------------------------------------------------------
// precision traits: the integrand type T and its tail threshold.  Below
// `deep` the lower-tail probability Phi(x) is treated in log space, chosen so
// that u * Phi(x) stays a normal number of type T for every u >= 2^-31.
// ---------------------------------------------------------------------------
template <typename T>
struct Prec;

template <>
struct Prec<double> {
  static __device__ __forceinline__ double deep() { return -36.0; }
  static __device__ __forceinline__ double erfc_(double x) { return erfc(x); }
  static __device__ __forceinline__ double ninv(double p) { return normcdfinv(p); }
  static __device__ __forceinline__ double frexp_(double x, int* e) { return frexp(x, e); }
  static __device__ __forceinline__ double ldexp_(double x, int e) { return ldexp(x, e); }
  static constexpr int kRescale = 64;  // accumulators may grow to 2^64 before re-referencing
};

template <>
struct Prec<float> {
  static __device__ __forceinline__ float deep() { return -11.0f; }
  static __device__ __forceinline__ float erfc_(float x) { return erfcf(x); }
  static __device__ __forceinline__ float ninv(float p) { return normcdfinvf(p); }
  static __device__ __forceinline__ float frexp_(float x, int* e) { return frexpf(x, e); }
  static __device__ __forceinline__ float ldexp_(float x, int e) { return ldexpf(x, e); }
  static constexpr int kRescale = 32;
};

// log Phi(x) for x far in the lower tail (x < -10), in FP64:
// Phi(x) = erfcx(z) exp(-z^2) / 2 with z = -x / sqrt(2).
__device__ __forceinline__ double log_phi_lower_tail(double x) {
  double z = -x * kSqrtHalf;
  return log(0.5 * erfcx(z)) - z * z;
}

// Lower-tail normal quantile from log p for p below the double range.
// Newton on log Phi(w) - lp; the slope phi(w)/Phi(w) equals
// 1 / (sqrt(2 pi) erfcx(-w/sqrt 2) / 2), so no exp is needed.
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

// One GHK coordinate: the truncation probability e = Phi(ub) as
// mant * 2^ex (mant in [1/2, 1)), its complement ebar = 1 - Phi(ub), and,
// in the deep lower tail, log Phi(ub) in FP64.
template <typename T>
struct Coord {
  T e, ebar, mant;
  int ex;
  bool deep;
  double lphi;
};

// Deep lower tail of norm_coord, kept out of line: it is rare and its
// log/exp/erfcx would otherwise inflate the register budget of the hot loop.
__device__ __noinline__ void deep_coord(double ub, double* mant, int* ex, double* lphi) {
  double lp = log_phi_lower_tail(ub);
  double k = floor(lp / kLn2);
  double m = exp(lp - k * kLn2);  // in [1, 2)
  *ex = (int)k + 1;
  *mant = 0.5 * m;
  *lphi = lp;
}

template <typename T>
__device__ __forceinline__ Coord<T> norm_coord(T ub) {
  Coord<T> c;
  if (ub >= Prec<T>::deep()) {
    T t = T(0.5) * Prec<T>::erfc_(fabs(ub) * T(kSqrtHalf));
    bool neg = ub < T(0);
    c.e = neg ? t : T(1) - t;
    c.ebar = neg ? T(1) - t : t;
    c.mant = Prec<T>::frexp_(c.e, &c.ex);
    c.deep = false;
    c.lphi = 0.0;
  } else {
    double m;
    deep_coord((double)ub, &m, &c.ex, &c.lphi);
    c.mant = (T)m;
    c.e = T(0);
    c.ebar = T(1);
    c.deep = true;
  }
  return c;
}

__device__ __noinline__ double deep_draw(double u, double lphi) { return ninv_from_log(log(u) + lphi); }

// Draw eps = Phi^{-1}(u Phi(ub)) by inversion.  Above 1/2 the quantile is
// taken from the complement (1 - u) + u (1 - Phi(ub)), which keeps full
// relative accuracy near 1.
template <typename T>
__device__ __forceinline__ T norm_draw(T u, T ubar, const Coord<T>& c) {
  if (c.deep) return (T)deep_draw((double)u, c.lphi);
  T pr = u * c.e;
  if (pr <= T(0.5)) return Prec<T>::ninv(pr);
  return -Prec<T>::ninv(ubar + u * c.ebar);
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
      if (fabs(delta - 1.0) < 1e-17) break;
    }
    *Q = lead * f;
    *P = 1.0 - *Q;
  }
}

// Chi-square quantile with `dof` degrees of freedom at probability u.
// Newton iterations on the gamma CDF (or on its complement above the median)
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
  for (int it = 0; it < 400; ++it) {
    double P, Q;
    inc_gamma(a, x, lga, &P, &Q);
    double r = upper ? (target - Q) : (P - target);  // increasing in x
    if (r < 0.0)
      lo = x;
    else
      hi = x;
    double dens = exp((a - 1.0) * log(x) - x - lga);
    double xn = x - r / dens;
    if (!(xn > lo && xn < hi)) xn = (hi < 1e308) ? 0.5 * (lo + hi) : 4.0 * x;
    double dx = fabs(xn - x);
    x = xn;
    if (dx <= 1e-15 * x) break;
  }
  return 2.0 * x;
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

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

}  // namespace cfust
