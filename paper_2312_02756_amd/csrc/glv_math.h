// Elementary functions for the conversion of a (pt, eta, phi) vector to
// Cartesian components on gfx950, written for this library:
//
//   sincos  Cody and Waite's additive argument reduction by pi/2 (Cody & Waite,
//           "Software Manual for the Elementary Functions", 1980), with the
//           multiples of pi/2 subtracted by fused multiply-adds against a
//           three-part split of pi/2, then Taylor polynomials of sin and cos on
//           |r| <= pi/4 (truncation below 1e-18 relative in FP64, 1e-9 in FP32);
//   exp     the same reduction by ln 2 (two-part split) and the Taylor
//           polynomial of e^r on |r| <= ln2/2, scaled by 2^k;
//   sinh / cosh from one exp and one reciprocal; sinh by its odd Taylor
//           polynomial for |x| < 1/2, where e^x - e^-x would cancel;
//   log     (FP64) x = m 2^e with m in [sqrt(1/2), sqrt(2)), log m = 2 atanh s,
//           s = (m - 1)/(m + 1), by the odd Taylor series of atanh (|s| <= 0.172,
//           truncation below 2^-60 relative), e ln 2 added in two parts;
//   asinh   (FP64) odd Taylor polynomial for |x| < 1/8; log1p(|x| + x^2 /
//           (1 + sqrt(1 + x^2))) below 2^28, the log1p as log w plus the
//           first-order correction for the rounding of w = 1 + u; log 2|x|
//           beyond.  Within 3 ulp (checked against 200-bit references).
//
// Split constants are the leading double / float of pi/2 and ln 2 and the
// remainders; Taylor coefficients are 1/n!, written as quotients the compiler
// folds exactly.
//
// Range.  The multiples k of pi/2 are removed with exact products inside the
// fused multiply-adds, so the reduced argument carries an absolute error of
// about |k| 2^-107 plus one rounding: within an ulp of the result for
// |x| < 2^40 rad in FP64 (2^20 in FP32), which is where the quadrant k is
// found exactly.  Beyond that (never for an azimuth) accuracy degrades.
// exp overflows to inf / underflows to 0 on its own (so sinh and cosh of
// |x| > 709.78 are +-inf, a little early near the double limit); NaN
// propagates.  There is no fallback to library code, so no call sites.
#pragma once

#include <hip/hip_runtime.h>

namespace glv {

// ------------------------------------------------------------------- FP64

// FP64 constants.  gfx9 has no 64-bit literals, so each one occupies a
// scalar-register pair, and the compiler hoists them to the top of the
// kernel.  That is right for the hot path, but on a rarely taken FP64 branch
// (the FP64 redo of an FP32 item) the hoisted constants would stay live
// across the whole kernel.  With kCold the value is marked as produced at
// its point of use (the asm statement emits nothing), which keeps it there.
template <bool kCold>
__device__ __forceinline__ double kd(double c) {
  if constexpr (kCold) asm volatile("" : "+s"(c));
  return c;
}

template <bool kCold = false>
__device__ __forceinline__ double poly_sin_d(double r) {
  const double z = r * r;
  double p = kd<kCold>(-1.0 / 355687428096000.0);  // -1/17!
  p = fma(p, z, kd<kCold>(1.0 / 1307674368000.0));
  p = fma(p, z, kd<kCold>(-1.0 / 6227020800.0));
  p = fma(p, z, kd<kCold>(1.0 / 39916800.0));
  p = fma(p, z, kd<kCold>(-1.0 / 362880.0));
  p = fma(p, z, kd<kCold>(1.0 / 5040.0));
  p = fma(p, z, kd<kCold>(-1.0 / 120.0));
  p = fma(p, z, kd<kCold>(1.0 / 6.0));
  // sin r = r - r^3 (1/6 - r^2/120 + ...)
  return fma(-r * z, p, r);
}

template <bool kCold = false>
__device__ __forceinline__ double poly_cos_d(double r) {
  const double z = r * r;
  double p = kd<kCold>(1.0 / 20922789888000.0);  // 1/16!
  p = fma(p, z, kd<kCold>(-1.0 / 87178291200.0));
  p = fma(p, z, kd<kCold>(1.0 / 479001600.0));
  p = fma(p, z, kd<kCold>(-1.0 / 3628800.0));
  p = fma(p, z, kd<kCold>(1.0 / 40320.0));
  p = fma(p, z, kd<kCold>(-1.0 / 720.0));
  p = fma(p, z, kd<kCold>(1.0 / 24.0));
  p = fma(p, z, -0.5);
  return fma(z, p, 1.0);
}

template <bool kCold = false>
__device__ __forceinline__ void fast_sincos(double x, double* s, double* c) {
  const double kn = rint(x * kd<kCold>(0.6366197723675814));  // x * 2/pi
  double r = fma(-kn, kd<kCold>(1.5707963267948966), x);
  r = fma(-kn, kd<kCold>(6.123233995736766e-17), r);
  r = fma(-kn, kd<kCold>(-1.4973849048591698e-33), r);
  const double sr = poly_sin_d<kCold>(r), cr = poly_cos_d<kCold>(r);
  const int q = (int)(kn - 4.0 * floor(0.25 * kn));  // k mod 4, exact
  const double ss = (q & 1) ? cr : sr;
  const double cc = (q & 1) ? sr : cr;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}

// e^x for |x| <= 709; overflows to inf beyond, underflows to 0.
template <bool kCold = false>
__device__ __forceinline__ double fast_exp(double x) {
  const double kn = rint(x * kd<kCold>(1.4426950408889634));  // x / ln2
  double r = fma(-kn, kd<kCold>(0.6931471805599453), x);
  r = fma(-kn, kd<kCold>(2.3190468138462996e-17), r);
  double p = kd<kCold>(1.0 / 6227020800.0);  // 1/13!
  p = fma(p, r, kd<kCold>(1.0 / 479001600.0));
  p = fma(p, r, kd<kCold>(1.0 / 39916800.0));
  p = fma(p, r, kd<kCold>(1.0 / 3628800.0));
  p = fma(p, r, kd<kCold>(1.0 / 362880.0));
  p = fma(p, r, kd<kCold>(1.0 / 40320.0));
  p = fma(p, r, kd<kCold>(1.0 / 5040.0));
  p = fma(p, r, kd<kCold>(1.0 / 720.0));
  p = fma(p, r, kd<kCold>(1.0 / 120.0));
  p = fma(p, r, kd<kCold>(1.0 / 24.0));
  p = fma(p, r, kd<kCold>(1.0 / 6.0));
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)kn);
}

// sinh(x) for |x| < 1/2 (odd Taylor polynomial to x^15).
template <bool kCold = false>
__device__ __forceinline__ double poly_sinh_d(double x) {
  const double z = x * x;
  double p = kd<kCold>(1.0 / 1307674368000.0);  // 1/15!
  p = fma(p, z, kd<kCold>(1.0 / 6227020800.0));
  p = fma(p, z, kd<kCold>(1.0 / 39916800.0));
  p = fma(p, z, kd<kCold>(1.0 / 362880.0));
  p = fma(p, z, kd<kCold>(1.0 / 5040.0));
  p = fma(p, z, kd<kCold>(1.0 / 120.0));
  p = fma(p, z, kd<kCold>(1.0 / 6.0));
  return fma(x * z, p, x);
}

template <bool kCold = false>
__device__ __forceinline__ void fast_sinhcosh(double x, double* sh, double* ch) {
  const double e = fast_exp<kCold>(x);
  const double ei = 1.0 / e;
  *ch = 0.5 * (e + ei);
  *sh = (fabs(x) < 0.5) ? poly_sinh_d<kCold>(x) : 0.5 * (e - ei);
}

// log(x); x = 0 gives -inf, +inf gives +inf, x < 0 and NaN give NaN.  log
// and asinh are used only once per leg, never in an inner loop, so their
// constants are always materialized at their use (kd<true>) rather than held
// in scalar registers for the whole kernel.
template <bool kCold = false>
__device__ __forceinline__ double fast_log(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);  // [1/2, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  if (m < kd<true>(0.7071067811865476)) {
    m = 2.0 * m;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double p = kd<true>(1.0 / 23.0);
  p = fma(p, z, kd<true>(1.0 / 21.0));
  p = fma(p, z, kd<true>(1.0 / 19.0));
  p = fma(p, z, kd<true>(1.0 / 17.0));
  p = fma(p, z, kd<true>(1.0 / 15.0));
  p = fma(p, z, kd<true>(1.0 / 13.0));
  p = fma(p, z, kd<true>(1.0 / 11.0));
  p = fma(p, z, kd<true>(1.0 / 9.0));
  p = fma(p, z, kd<true>(1.0 / 7.0));
  p = fma(p, z, kd<true>(1.0 / 5.0));
  p = fma(p, z, kd<true>(1.0 / 3.0));
  const double t = 2.0 * s;
  const double lm = fma(t * z, p, t);  // log m
  const double de = (double)e;
  const double r = fma(de, kd<true>(0.6931471805599453), fma(de, kd<true>(2.3190468138462996e-17), lm));
  if (x > 0.0 && x < __builtin_huge_val()) return r;
  return (x == 0.0) ? -__builtin_huge_val() : ((x == __builtin_huge_val()) ? x : __builtin_nan(""));
}

template <bool kCold = false>
__device__ __forceinline__ double fast_asinh(double x) {
  const double ax = fabs(x);
  double r;
  if (ax < 0.125) {
    const double z = ax * ax;
    double p = kd<true>(-12155.0 / 1245184.0);  // coefficient of x^19
    p = fma(p, z, kd<true>(6435.0 / 557056.0));
    p = fma(p, z, kd<true>(-143.0 / 10240.0));
    p = fma(p, z, kd<true>(231.0 / 13312.0));
    p = fma(p, z, kd<true>(-63.0 / 2816.0));
    p = fma(p, z, kd<true>(35.0 / 1152.0));
    p = fma(p, z, kd<true>(-5.0 / 112.0));
    p = fma(p, z, kd<true>(3.0 / 40.0));
    p = fma(p, z, kd<true>(-1.0 / 6.0));
    r = fma(ax * z, p, ax);
  } else if (ax < kd<true>(268435456.0)) {  // 2^28
    const double z = ax * ax;
    const double u = ax + z / (1.0 + sqrt(1.0 + z));
    const double w = 1.0 + u;
    r = fast_log<kCold>(w) + (u - (w - 1.0)) / w;
  } else {
    r = fast_log<kCold>(ax) + kd<true>(0.6931471805599453);
  }
  return copysign(r, x);
}

// ------------------------------------------------------------------- FP32

__device__ __forceinline__ float poly_sin_f(float r) {
  const float z = r * r;
  float p = 1.0f / 362880.0f;  // 1/9!
  p = fmaf(p, z, -1.0f / 5040.0f);
  p = fmaf(p, z, 1.0f / 120.0f);
  p = fmaf(p, z, -1.0f / 6.0f);
  return fmaf(r * z, p, r);
}

__device__ __forceinline__ float poly_cos_f(float r) {
  const float z = r * r;
  float p = -1.0f / 3628800.0f;  // -1/10!
  p = fmaf(p, z, 1.0f / 40320.0f);
  p = fmaf(p, z, -1.0f / 720.0f);
  p = fmaf(p, z, 1.0f / 24.0f);
  p = fmaf(p, z, -0.5f);
  return fmaf(z, p, 1.0f);
}

__device__ __forceinline__ void fast_sincos(float x, float* s, float* c) {
  const float kf = rintf(x * 0.63661975f);
  float r = fmaf(-kf, 1.5707964f, x);
  r = fmaf(-kf, -4.371139e-08f, r);
  r = fmaf(-kf, -1.7151245e-15f, r);
  const float sr = poly_sin_f(r), cr = poly_cos_f(r);
  const int q = (int)(kf - 4.0f * floorf(0.25f * kf));
  const float ss = (q & 1) ? cr : sr;
  const float cc = (q & 1) ? sr : cr;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}

__device__ __forceinline__ float fast_exp(float x) {
  const float kf = rintf(x * 1.442695f);
  float r = fmaf(-kf, 0.6931472f, x);
  r = fmaf(-kf, -1.9046542e-09f, r);
  float p = 1.0f / 40320.0f;  // 1/8!
  p = fmaf(p, r, 1.0f / 5040.0f);
  p = fmaf(p, r, 1.0f / 720.0f);
  p = fmaf(p, r, 1.0f / 120.0f);
  p = fmaf(p, r, 1.0f / 24.0f);
  p = fmaf(p, r, 1.0f / 6.0f);
  p = fmaf(p, r, 0.5f);
  p = fmaf(p, r, 1.0f);
  p = fmaf(p, r, 1.0f);
  return ldexpf(p, (int)kf);
}

__device__ __forceinline__ float poly_sinh_f(float x) {
  const float z = x * x;
  float p = 1.0f / 362880.0f;  // 1/9!
  p = fmaf(p, z, 1.0f / 5040.0f);
  p = fmaf(p, z, 1.0f / 120.0f);
  p = fmaf(p, z, 1.0f / 6.0f);
  return fmaf(x * z, p, x);
}

__device__ __forceinline__ void fast_sinhcosh(float x, float* sh, float* ch) {
  const float e = fast_exp(x);
  const float ei = 1.0f / e;
  *ch = 0.5f * (e + ei);
  *sh = (fabsf(x) < 0.5f) ? poly_sinh_f(x) : 0.5f * (e - ei);
}

// The same with e^-x from the hardware reciprocal (within 1 ulp) instead of a
// correctly rounded quotient: about half an ulp more in sinh and cosh, for
// the compensated path, whose error bound budgets for it.
__device__ __forceinline__ void fast_sinhcosh_rcp(float x, float* sh, float* ch) {
  const float e = fast_exp(x);
  const float ei = __builtin_amdgcn_rcpf(e);
  *ch = 0.5f * (e + ei);
  *sh = (fabsf(x) < 0.5f) ? poly_sinh_f(x) : 0.5f * (e - ei);
}

// sinh x for |x| <= 4 by its odd Taylor polynomial to x^19 (the next term is
// below 1e-9 of sinh x there), no reduction and no exponential: relative
// error within 3.5 * 2^-24 in an FP32 emulation over 6 M points (growing with
// |x|: 1.3 * 2^-24 below 1, 1.8 * 2^-24 below 2), against 3.9 * 2^-24 for the
// exp route.  Every coefficient is positive, so the Horner steps do not cancel.
__device__ __forceinline__ float poly_sinh19_f(float x) {
  const float z = x * x;
  float p = (float)(1.0 / 121645100408832000.0);  // 1/19!
  p = fmaf(p, z, (float)(1.0 / 355687428096000.0));
  p = fmaf(p, z, (float)(1.0 / 1307674368000.0));
  p = fmaf(p, z, (float)(1.0 / 6227020800.0));
  p = fmaf(p, z, (float)(1.0 / 39916800.0));
  p = fmaf(p, z, (float)(1.0 / 362880.0));
  p = fmaf(p, z, (float)(1.0 / 5040.0));
  p = fmaf(p, z, (float)(1.0 / 120.0));
  p = fmaf(p, z, (float)(1.0 / 6.0));
  return fmaf(x * z, p, x);
}

// sin x for |x| <= pi/2 by its odd Taylor polynomial to x^13 (the next term
// is below 7e-12 there): no argument reduction.  Within 1.7 ulp on the
// interval (an FP32 emulation over 220,000 points, the worst next to pi/2).
__device__ __forceinline__ float sin_half_range(float x) {
  const float z = x * x;
  float p = 1.0f / 6227020800.0f;  // 1/13!
  p = fmaf(p, z, -1.0f / 39916800.0f);
  p = fmaf(p, z, 1.0f / 362880.0f);
  p = fmaf(p, z, -1.0f / 5040.0f);
  p = fmaf(p, z, 1.0f / 120.0f);
  p = fmaf(p, z, -1.0f / 6.0f);
  return fmaf(x * z, p, x);
}

}  // namespace glv
