// Device-side building blocks shared by the gfx950 kernels: SoA column
// bundles, streaming (non-temporal) 16-byte loads/stores, the coordinate
// conversions of a 4D vector (GenVectorX Sec. 3.1: Cartesian and
// pt/eta/phi systems, templated on the scalar type) and the mass of a
// Cartesian vector (Fig. 1: the mass of the summed pair).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "glv.h"
#include "glv_math.h"

namespace glv {

template <typename T>
struct Cols4 {
  const T* c[4];
};
template <typename T>
struct Cols3 {
  const T* c[3];
};
template <typename T>
struct OutCols4 {
  T* c[4];
};
template <typename T>
struct OutCols3 {
  T* c[3];
};

// 16 bytes per lane per column: 2 doubles or 4 floats.
template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int N = 2;
};
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int N = 4;
};

// A pack of V consecutive elements of one column.
template <typename T, int V>
struct Pack {
  T v[V];
};

// Streaming load of elements [V*i, V*i + V) of column p.  The data is read
// once per launch, so it bypasses the caches' retention (non-temporal).
template <typename T, int V>
__device__ __forceinline__ Pack<T, V> load_pack(const T* __restrict__ p, int64_t i) {
  Pack<T, V> r;
  if constexpr (V == 1) {
    r.v[0] = __builtin_nontemporal_load(p + i);
  } else {
    static_assert(V == Vec16<T>::N, "vector width must be 16 bytes");
    typedef typename Vec16<T>::type VT;
    VT x = __builtin_nontemporal_load(reinterpret_cast<const VT*>(p) + i);
#pragma unroll
    for (int k = 0; k < V; ++k) r.v[k] = x[k];
  }
  return r;
}

template <typename T, int V>
__device__ __forceinline__ void store_pack(T* __restrict__ p, int64_t i, const Pack<T, V>& r) {
  if constexpr (V == 1) {
    __builtin_nontemporal_store(r.v[0], p + i);
  } else {
    typedef typename Vec16<T>::type VT;
    VT x;
#pragma unroll
    for (int k = 0; k < V; ++k) x[k] = r.v[k];
    __builtin_nontemporal_store(x, reinterpret_cast<VT*>(p) + i);
  }
}

// ------------------------------------------------------------ histogram

// Equal bins of [lo, hi) with under- and overflow counters.
struct HistSpec {
  double lo, hi, s;  // s = n_bins / (hi - lo), formed on the host
  int64_t nb;
};

// Counters (bins plus under- and overflow) a workgroup keeps in LDS: 32 KiB.
constexpr int kHistLdsSlots = 8192;

// Counter slot of v: 0 below lo, nb + 1 at or above hi, else
// 1 + floor((v - lo) s) clamped to nb; -1 for NaN (not counted).  Evaluated
// in binary64 without contraction, as the definition states.
__device__ __forceinline__ int64_t hist_slot(double v, const HistSpec& h) {
#pragma clang fp contract(off)
  if (v != v) return -1;
  if (v < h.lo) return 0;
  if (v >= h.hi) return h.nb + 1;
  const int64_t b = (int64_t)floor((v - h.lo) * h.s);
  return 1 + (b < h.nb - 1 ? b : h.nb - 1);
}

// ------------------------------------------------------------ scalar math

// FP64 square root: the hardware reciprocal square root y ~ 1/sqrt(x)
// (relative error below 2^-22), one Goldschmidt step (g -> sqrt x,
// h -> 1/(2 sqrt x), error ~2^-45) and one Newton correction of g from the
// residual x - g^2 formed by a fused multiply-add (error ~2^-90 before the
// final rounding).  The result is the correctly rounded root unless that lies
// within ~2^-90 (relative) of a rounding midpoint; the compiler's expansion
// adds a second correction and subnormal scaling, seven more instructions on
// the pair loops.  0 and +inf pass through, NaN propagates, x < 0 gives NaN;
// subnormal x (never a mass squared here) may lose a few bits.
__device__ __forceinline__ double d_sqrt(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  g = fma(fma(-g, g, x), h, g);
  return (x == 0.0 || x == __builtin_huge_val()) ? x : g;
}
__device__ __forceinline__ float d_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double d_abs(double x) { return fabs(x); }
// a * b + c with one rounding, either precision: written out where a sum of
// products must fuse the same way in every kernel that evaluates it.
__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ float d_abs(float x) { return fabsf(x); }

// ------------------------------------------------------------ conversion

// sincos / sinhcosh of either precision.  kPin (FP64 only) materializes the
// polynomial constants at their use: for conversions done once per particle
// in a kernel whose hot loop is elsewhere, so that the constants are not
// hoisted into registers held across that loop.
template <bool kPin, typename T>
__device__ __forceinline__ void sincos_t(T x, T* s, T* c) {
  if constexpr (sizeof(T) == 8)
    fast_sincos<kPin>(x, s, c);
  else
    fast_sincos(x, s, c);
}
template <bool kPin, typename T>
__device__ __forceinline__ void sinhcosh_t(T x, T* sh, T* ch) {
  if constexpr (sizeof(T) == 8)
    fast_sinhcosh<kPin>(x, sh, ch);
  else
    fast_sinhcosh(x, sh, ch);
}

// E = sqrt((pt cosh eta)^2 + M^2) from pc = pt cosh eta, with one explicit
// fused multiply-add, so that every conversion forms it bitwise alike.
template <typename T>
__device__ __forceinline__ T energy_of(T pc, T m) {
  if constexpr (sizeof(T) == 8)
    return d_sqrt(fma(pc, pc, m * m));
  else
    return d_sqrt(fmaf(pc, pc, m * m));
}

// E = sqrt(px^2 + py^2 + pz^2 + M^2) of a PxPyPzM vector, with explicit
// fused multiply-adds, so that every kernel forms it bitwise alike.
template <typename T>
__device__ __forceinline__ T energy_cart(T px, T py, T pz, T m) {
  if constexpr (sizeof(T) == 8)
    return d_sqrt(fma(px, px, fma(py, py, fma(pz, pz, m * m))));
  else
    return d_sqrt(fmaf(px, px, fmaf(py, py, fmaf(pz, pz, m * m))));
}

// Cartesian (px, py, pz, E) of one vector given in COORDS.
template <int COORDS, typename T, bool kPin = false>
__device__ __forceinline__ void to_cart(T c0, T c1, T c2, T c3, T v[4]) {
  if constexpr (COORDS == GLV_PXPYPZE || COORDS == GLV_PXPYPZM) {
    v[0] = c0;
    v[1] = c1;
    v[2] = c2;
    v[3] = (COORDS == GLV_PXPYPZE) ? c3 : energy_cart(c0, c1, c2, c3);
  } else {
    T s, c, sh, ch;
    sincos_t<kPin>(c2, &s, &c);
    sinhcosh_t<kPin>(c1, &sh, &ch);
    v[0] = c0 * c;
    v[1] = c0 * s;
    v[2] = c0 * sh;
    if constexpr (COORDS == GLV_PTETAPHIM) {
      T pc = c0 * ch;
      v[3] = energy_of(pc, c3);
    } else {
      v[3] = c3;
    }
  }
}

// Conversion together with the pieces its Jacobian needs.
template <typename T>
struct LegJ {
  T v[4];            // px, py, pz, E
  T cp, sp, sh, ch;  // cos phi, sin phi, sinh eta, cosh eta
};

template <int COORDS, typename T, bool kPin = false>
__device__ __forceinline__ LegJ<T> to_cart_j(T c0, T c1, T c2, T c3) {
  LegJ<T> L;
  if constexpr (COORDS == GLV_PXPYPZE || COORDS == GLV_PXPYPZM) {
    L.v[0] = c0;
    L.v[1] = c1;
    L.v[2] = c2;
    L.v[3] = (COORDS == GLV_PXPYPZE) ? c3 : energy_cart(c0, c1, c2, c3);
    L.cp = L.sp = L.sh = L.ch = T(0);
  } else {
    sincos_t<kPin>(c2, &L.sp, &L.cp);
    sinhcosh_t<kPin>(c1, &L.sh, &L.ch);
    L.v[0] = c0 * L.cp;
    L.v[1] = c0 * L.sp;
    L.v[2] = c0 * L.sh;
    if constexpr (COORDS == GLV_PTETAPHIM) {
      T pc = c0 * L.ch;
      L.v[3] = energy_of(pc, c3);
    } else {
      L.v[3] = c3;
    }
  }
  return L;
}

// Chain u = dL/d(px, py, pz, E) of one vector to its own coordinates.
template <int COORDS, typename T>
__device__ __forceinline__ void chain_coords(const LegJ<T>& L, T c0, T c3, const T u[4], T g[4]) {
  if constexpr (COORDS == GLV_PXPYPZE) {
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = u[k];
  } else if constexpr (COORDS == GLV_PXPYPZM) {
    // E = sqrt(|p|^2 + M^2): dE/dp_k = p_k/E, dE/dM = M/E
    const T e = L.v[3];
    const T ue = (e > T(0)) ? u[3] / e : T(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) g[k] = u[k] + ue * L.v[k];
    g[3] = ue * c3;
  } else {
    T pt = c0;
    T g0 = u[0] * L.cp + u[1] * L.sp + u[2] * L.sh;
    T g1 = u[2] * pt * L.ch;
    T g2 = u[1] * L.v[0] - u[0] * L.v[1];
    T g3;
    if constexpr (COORDS == GLV_PTETAPHIM) {
      // E = sqrt((pt ch)^2 + M^2): dE/dpt = pt ch^2/E, dE/deta = pt^2 sh ch/E, dE/dM = M/E
      T e = L.v[3];
      T ue = (e > T(0)) ? u[3] / e : T(0);
      g0 += ue * pt * L.ch * L.ch;
      g1 += ue * pt * pt * L.sh * L.ch;
      g3 = ue * c3;
    } else {
      g3 = u[3];
    }
    g[0] = g0;
    g[1] = g1;
    g[2] = g2;
    g[3] = g3;
  }
}

// w = a + b componentwise, each sum rounded on its own: no multiply-add may
// fuse one leg's product (pt cos(phi), ...) into the sum, so the pair mass
// is bitwise symmetric in its two legs.
template <typename T>
__device__ __forceinline__ void add4(const T a[4], const T b[4], T w[4]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = a[k] + b[k];
}

// Mass of a Cartesian vector: q = E^2 - |P|^2, m = sqrt(q) or -sqrt(-q).
template <typename T>
__device__ __forceinline__ T mass_of(const T w[4]) {
  T q = w[3] * w[3] - w[0] * w[0] - w[1] * w[1] - w[2] * w[2];
  // one square root of |q|, then q's sign bit (one instruction).  q is never
  // -0: E^2 is +0 or positive and each product subtracted after it leaves
  // +0 where it cancels exactly, so a zero q still gives +0.
  return __builtin_copysign(d_sqrt(d_abs(q)), q);
}

// 1/sqrt(a) for a > 0: the hardware reciprocal square root (relative error
// below 2^-22 in FP64, about 1 ulp in FP32) refined by Newton steps
// y <- y + y (1 - a y^2)/2, each of which squares the relative error (times
// 3/2): two in FP64, one in FP32.  Within about an ulp; a = +inf gives NaN.
__device__ __forceinline__ double inv_sqrt(double a) {
  double y = __builtin_amdgcn_rsq(a);
  y = fma(0.5 * y, fma(-a * y, y, 1.0), y);
  return fma(0.5 * y, fma(-a * y, y, 1.0), y);
}
__device__ __forceinline__ float inv_sqrt(float a) {
  const float y = __builtin_amdgcn_rsqf(a);
  return fmaf(0.5f * y, fmaf(-a * y, y, 1.0f), y);
}

// g / |m| for the mass of w, with 1/|m| = 1/sqrt|q| taken directly (no
// square root, no division on the gradient path); zero where q = 0 (m = 0).
// The same expression for q as mass_of.
template <typename T>
__device__ __forceinline__ T pair_coef(const T w[4], T g) {
  const T q = w[3] * w[3] - w[0] * w[0] - w[1] * w[1] - w[2] * w[2];
  const T a = d_abs(q);
  const T r = inv_sqrt(a);  // evaluated for every lane: a select, not a branch
  return (a > T(0)) ? g * r : T(0);
}

// u = g dm/d(px, py, pz, E) for the mass of w: (-P, E) g / |m|.
template <typename T>
__device__ __forceinline__ void dmass(const T w[4], T g, T u[4]) {
  const T s = pair_coef(w, g);
  u[0] = -w[0] * s;
  u[1] = -w[1] * s;
  u[2] = -w[2] * s;
  u[3] = w[3] * s;
}

// ------------------------------------------------- conversion, either way

__device__ __forceinline__ double hypot_t(double x, double y) { return ::hypot(x, y); }
__device__ __forceinline__ float hypot_t(float x, float y) { return ::hypotf(x, y); }
__device__ __forceinline__ double atan2_t(double y, double x) { return ::atan2(y, x); }
__device__ __forceinline__ float atan2_t(float y, float x) { return ::atan2f(y, x); }
__device__ __forceinline__ double asinh_t(double x) { return fast_asinh<false>(x); }
__device__ __forceinline__ float asinh_t(float x) { return ::asinhf(x); }

// Coordinates TO of a Cartesian vector v = (px, py, pz, E), the inverse of
// to_cart (Sec. 3.1: a 4D vector in any of its systems): pt = hypot(px, py),
// eta = asinh(pz / pt), phi = atan2(py, px), and M = mass_of(v) (the pair
// mass's sign convention) or E; PxPyPzM keeps (px, py, pz) and takes that M.
// On the beam axis (pt = 0) eta is +-inf by the sign of pz, 0 for pz = 0.
template <int TO, typename T>
__device__ __forceinline__ void from_cart(const T v[4], T c[4]) {
  if constexpr (TO == GLV_PXPYPZE || TO == GLV_PXPYPZM) {
#pragma unroll
    for (int k = 0; k < 3; ++k) c[k] = v[k];
    c[3] = (TO == GLV_PXPYPZE) ? v[3] : mass_of(v);
  } else {
    const T pt = hypot_t(v[0], v[1]);
    c[0] = pt;
    const T inf = __builtin_huge_val();
    c[1] = (pt > T(0)) ? asinh_t(v[2] / pt) : ((v[2] > T(0)) ? inf : ((v[2] < T(0)) ? -inf : T(0)));
    c[2] = atan2_t(v[1], v[0]);
    if constexpr (TO == GLV_PTETAPHIM)
      c[3] = mass_of(v);
    else
      c[3] = v[3];
  }
}

// u = (d c / d v)^T gc for c = from_cart<TO>(v): d pt = (px, py, 0, 0)/pt,
// d eta = (-pz px, -pz py, pt^2, 0)/(pt^2 p) with p = |(px, py, pz)|,
// d phi = (-py, px, 0, 0)/pt^2, d M = (-P, E)/|M| (zero where M = 0) or
// d E = (0, 0, 0, 1); on the beam axis the pt, eta and phi rows are zero.
// PxPyPzM: the identity rows of px, py, pz and the d M row.
template <int TO, typename T>
__device__ __forceinline__ void dcoords_dcart(const T v[4], const T gc[4], T u[4]) {
  if constexpr (TO == GLV_PXPYPZE) {
#pragma unroll
    for (int k = 0; k < 4; ++k) u[k] = gc[k];
  } else if constexpr (TO == GLV_PXPYPZM) {
    const T s = pair_coef(v, gc[3]);  // gc[3] / |M|
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = gc[k] - s * v[k];
    u[3] = s * v[3];
  } else {
    const T pt = hypot_t(v[0], v[1]);
    const T p = d_sqrt(pt * pt + v[2] * v[2]);
    const bool off_axis = pt > T(0);
    const T ipt = off_axis ? T(1) / pt : T(0);
    const T ip = off_axis ? T(1) / p : T(0);
    const T ipt2 = ipt * ipt;
    const T a = gc[0] * ipt - gc[1] * v[2] * ipt2 * ip;  // common factor of px and py (pt and eta rows)
    const T b = gc[2] * ipt2;                               // phi row
    u[0] = a * v[0] - b * v[1];
    u[1] = a * v[1] + b * v[0];
    u[2] = gc[1] * ip;
    if constexpr (TO == GLV_PTETAPHIM) {
      const T s = pair_coef(v, gc[3]);  // gc[3] / |M|
      u[0] -= s * v[0];
      u[1] -= s * v[1];
      u[2] -= s * v[2];
      u[3] = s * v[3];
    } else {
      u[3] = gc[3];
    }
  }
}

// ------------------------------------------------- cancellation-free mass

// sinh alone: FP64 small arguments by the odd polynomial, else from one exp;
// FP32 by the odd polynomial up to |x| = 4 (one path for every argument of a
// collider pair's half rapidity difference), else from one exp.
template <bool kCold = false>
__device__ __forceinline__ double fast_sinh(double x) {
  if (fabs(x) < 0.5) return poly_sinh_d<kCold>(x);
  double sh, ch;
  fast_sinhcosh<kCold>(x, &sh, &ch);
  return sh;
}
__device__ __forceinline__ float fast_sinh(float x) {
  if (fabsf(x) <= 4.0f) return poly_sinh19_f(x);
  float sh, ch;
  fast_sinhcosh_rcp(x, &sh, &ch);
  return sh;
}

// asinh of the small argument of delta.  FP32: for |x| < 1/8 the Taylor
// series x - x^3/6 + 3x^5/40 - 5x^7/112 (next term below 2e-9 relative);
// otherwise, and always in FP64, the device library's asinh.
template <bool kCold>
__device__ __forceinline__ double small_asinh(double x) {
  return fast_asinh<kCold>(x);
}
template <bool kCold>
__device__ __forceinline__ float small_asinh(float x) {
  if (!(fabsf(x) < 0.125f)) return asinhf(x);
  const float z = x * x;
  float p = fmaf(z, -5.0f / 112.0f, 3.0f / 40.0f);
  p = fmaf(p, z, -1.0f / 6.0f);
  return fmaf(x * z, p, x);
}

// pi split into the nearest T and the remainder.
template <typename T>
struct Pi;
template <>
struct Pi<double> {
  static constexpr double hi = 3.141592653589793116;
  static constexpr double lo = 1.2246467991473532e-16;
};
template <>
struct Pi<float> {
  static constexpr float hi = 3.14159274101257324f;
  static constexpr float lo = -8.74227765734758577e-08f;
};

// a - b reduced to (-pi, pi]; next to the seam both angles are moved by the
// head of pi separately (exact subtractions), then the tail is applied.
template <typename T>
__device__ __forceinline__ T dphi_reduced(T a, T b) {
  T d = a - b;
  if (d > Pi<T>::hi) return ((a - Pi<T>::hi) - (b + Pi<T>::hi)) - T(2) * Pi<T>::lo;
  if (d <= -Pi<T>::hi) return ((a + Pi<T>::hi) - (b - Pi<T>::hi)) + T(2) * Pi<T>::lo;
  return d;
}

// Square root and quotient of the compensated path.  In FP32 the hardware
// square root (within 1 ulp) and a times the hardware reciprocal (within
// 2 ulp), where the compiler's correctly rounded expansions take about ten
// instructions each; the error bound below budgets for the difference.  In
// FP64 the ordinary ones.
template <typename T>
__device__ __forceinline__ T sqrt_budgeted(T x) {
  if constexpr (sizeof(T) == 4)
    return __builtin_amdgcn_sqrtf(x);
  else
    return d_sqrt(x);
}
template <typename T>
__device__ __forceinline__ T div_budgeted(T a, T b) {
  if constexpr (sizeof(T) == 4)
    return a * __builtin_amdgcn_rcpf(b);
  else
    return a / b;
}

// Rounding units granted in the compensated error bound to the
// multiplicative factors of the pair terms, and (times |delta|) to each
// leg's rapidity shift delta: 16 each for products and quotients of
// accurately computed factors, plus 4 for the FP32 hardware square roots
// (mT, E) and reciprocals (the quotients of delta and of mT - pt, e^-x in
// sinh and cosh), the unreduced sine of the half azimuth difference
// (1.7 ulp) and the unreduced sinh of the half rapidity difference (3.5 units)
// that replace correctly rounded ones.
constexpr float kFactorUnits = 20.0f;
constexpr float kDeltaUnits = 20.0f;

// Per-leg terms: pt, eta, phi, M^2, mT = sqrt(pt^2 + M^2),
// delta = y - eta = -asinh(M^2 sinh(eta) / (mT (pt cosh(eta) + E))) and
// dmt = mT - pt = M^2 / (mT + pt) (formed without the cancellation).
template <typename T>
struct LegC {
  T pt, eta, phi, m2, mt, delta, dmt;
};

// mT, delta and mT - pt of a leg from pt, M^2, sinh(eta), pt cosh(eta) and E
// (pt^2 + M^2 with one explicit fused multiply-add, so that every kernel forms
// mT alike).  The two quotients are budgeted ones (a times the hardware
// reciprocal in FP32).
template <typename T, bool kCold = false>
__device__ __forceinline__ void leg_shift(T pt, T mm, T sh, T pc, T e, T* mt, T* delta, T* dmt) {
#pragma clang fp contract(off)
  if constexpr (sizeof(T) == 8)
    *mt = sqrt_budgeted(fma(pt, pt, mm));
  else
    *mt = sqrt_budgeted(fmaf(pt, pt, mm));
  const T den = *mt * (pc + e);
  *delta = (den > T(0)) ? -small_asinh<kCold>(div_budgeted(mm * sh, den)) : T(0);
  *dmt = (mm > T(0)) ? div_budgeted(mm, *mt + pt) : T(0);
}

// Compensated leg terms together with the Cartesian vector of a
// (pt, eta, phi, M) particle, sharing sinh, cosh and E with the conversion
// (v is bitwise what to_cart gives).
template <typename T>
__device__ __forceinline__ LegC<T> comp_leg_cart(T pt, T eta, T phi, T mass, T v[4]) {
  T sn, cs, sh, ch;
  sincos_t<true>(phi, &sn, &cs);
  sinhcosh_t<true>(eta, &sh, &ch);
  const T pc = pt * ch;
  v[0] = pt * cs;
  v[1] = pt * sn;
  v[2] = pt * sh;
  v[3] = energy_of(pc, mass);
  LegC<T> L;
  L.pt = pt;
  L.eta = eta;
  L.phi = phi;
  L.m2 = mass * mass;
  leg_shift<T>(pt, L.m2, sh, pc, v[3], &L.mt, &L.delta, &L.dmt);
  return L;
}

// kCold: this evaluation is the rarely taken FP64 redo of an FP32 item.
template <typename T, bool kCold = false>
__device__ __forceinline__ LegC<T> comp_leg(T pt, T eta, T phi, T mass) {
  LegC<T> L;
  L.pt = pt;
  L.eta = eta;
  L.phi = phi;
  T mm = mass * mass;
  L.m2 = mm;
  T sh, ch;
  if constexpr (sizeof(T) == 8)
    fast_sinhcosh<kCold>(eta, &sh, &ch);
  else
    fast_sinhcosh_rcp(eta, &sh, &ch);
  T pc = pt * ch;
  T e = sqrt_budgeted(fma_t(pc, pc, mm));
  leg_shift<T, kCold>(pt, mm, sh, pc, e, &L.mt, &L.delta, &L.dmt);
  return L;
}


// Relative-error bound (units of u32) above which an FP32 pair is redone in
// FP64: 2^-18 / 2^-24 = 64.
constexpr float kFallbackUnits = 64.0f;

// sin^2 of half the azimuth difference d.  In FP32 the unreduced polynomial
// while |d/2| <= pi/2 (always, for azimuths in [-pi, pi] after the seam
// reduction), otherwise the reduced sine.
template <typename T, bool kCold>
__device__ __forceinline__ T sin2_half(T d) {
  T s, c;
  if constexpr (sizeof(T) == 8) {
    fast_sincos<kCold>(T(0.5) * d, &s, &c);
  } else {
    const float h = 0.5f * d;
    if (fabsf(h) <= 1.5707964f)
      s = sin_half_range(h);
    else
      fast_sincos(h, &s, &c);
  }
  return s * s;
}

// Pair m^2 = Ma^2 + Mb^2 + 2 (t1 + t2 + t3) (all terms >= 0); *k receives
// t1 + t2 + t3 = E_a E_b - p_a.p_b.  If `redo` is not NULL it is set when a
// bound on the relative error of m^2 exceeds kFallbackUnits rounding units:
// every term is a product/quotient of accurately computed positive factors
// (kFactorUnits covers them) except the rapidity difference dy, whose
// absolute error is a few units of |d1| + |d2| + |dy| plus that of the
// deltas; t1 moves with dy as 2 mTa mTb |sinh dy| = 4 mTa mTb |s1| cosh(dy/2),
// taken at most as 4 mTa mTb |s1| (1 + |s1|).  A NaN bound asks for the redo.
template <typename T, bool kCold = false>
__device__ __forceinline__ T comp_pair_m2(const LegC<T>& a, const LegC<T>& b, T* k, bool* redo) {
  // no implicit contraction: every kernel (packed or not, staged or not)
  // rounds these terms alike; the one fused product is written out
#pragma clang fp contract(off)
  T d1 = a.eta - b.eta;
  T d2 = a.delta - b.delta;
  T dy = d1 + d2;
  T s1;
  if constexpr (sizeof(T) == 8)
    s1 = fast_sinh<kCold>(T(0.5) * dy);
  else
    s1 = fast_sinh(T(0.5) * dy);
  const T mm = a.mt * b.mt;
  T t1 = (T(2) * mm) * (s1 * s1);
  T t2 = (T(2) * (a.pt * b.pt)) * sin2_half<T, kCold>(dphi_reduced(a.phi, b.phi));
  // mTa mTb - pta ptb = (mTa - pta) mTb + pta (mTb - ptb): two terms >= 0
  T t3 = fma_t(a.dmt, b.mt, a.pt * b.dmt);
  T kk = (t1 + t2) + t3;
  T m2 = (a.m2 + b.m2) + T(2) * kk;
  *k = kk;
  if (redo) {
    T edy = ((d_abs(d1) + d_abs(d2)) + d_abs(dy)) + T(kDeltaUnits) * (d_abs(a.delta) + d_abs(b.delta));
    const T as1 = d_abs(s1);
    T sens = (T(4) * mm) * (as1 * (T(1) + as1));  // >= 2 * d(t1)/d(dy)
    // bound = sens edy / m2 + kFactorUnits > kFallbackUnits, for m2 > 0
    *redo = (m2 > T(0)) && !(sens * edy <= T(kFallbackUnits - kFactorUnits) * m2);
  }
  return m2;
}

// ------------------------------------- reverse mode of the cancellation-free mass

// A leg of the compensated form with the pieces its reverse mode needs.
template <typename T>
struct LegCJ {
  LegC<T> c;
  T mass, sh, ch, e;  // M as given, sinh(eta), cosh(eta), E
};

template <typename T>
__device__ __forceinline__ LegCJ<T> comp_leg_j(T pt, T eta, T phi, T mass) {
  LegCJ<T> L;
  L.c.pt = pt;
  L.c.eta = eta;
  L.c.phi = phi;
  L.mass = mass;
  const T mm = mass * mass;
  L.c.m2 = mm;
  if constexpr (sizeof(T) == 8)
    fast_sinhcosh<false>(eta, &L.sh, &L.ch);
  else
    fast_sinhcosh_rcp(eta, &L.sh, &L.ch);
  const T pc = pt * L.ch;
  L.e = sqrt_budgeted(fma_t(pc, pc, mm));
  leg_shift<T, false>(pt, mm, L.sh, pc, L.e, &L.c.mt, &L.c.delta, &L.c.dmt);
  return L;
}

// m dm/d(pt, eta, phi, M) of leg a with partner b, from K = E_a E_b - p_a.p_b
// = mTa mTb cosh(dy) - pta ptb cos(dphi) and m dm = Ma dMa + Mb dMb + dK:
//   dK/dpta  = (pta mTb / mTa) 2 sinh^2(dy/2) + ptb 2 sin^2(dphi/2)
//              + (pta^2 Mb^2 - ptb^2 Ma^2) / ((pta mTb + ptb mTa) mTa)
//              + mTa mTb sinh(dy) dya/dpta
//   dK/detaa = mTa mTb sinh(dy) pta cosh(etaa) / Ea
//   dK/dphia = pta ptb sin(dphi)
//   dK/dMa   = (Ma / mTa) mTb cosh(dy) + mTa mTb sinh(dy) dya/dMa
// with dy/dpt = sinh(eta) M^2 / (mT^2 E) and dy/dM = -pt sinh(eta) M / (mT^2 E)
// at fixed eta (from sinh y = pt sinh(eta) / mT).  The first row regroups
// mTb pta/mTa cosh(dy) - ptb cos(dphi), which cancels for nearly collinear
// pairs, into terms of the forward form; only its third term is a signed
// difference, of two squares products.  shdy = sinh(dy), sdphi = sin(dphi)
// as seen from leg a.  Legs with mT = 0 (pt = M = 0) get zero rows.
template <typename T>
__device__ __forceinline__ void comp_leg_rows(const LegCJ<T>& a, const LegCJ<T>& b, T sh2, T chdy, T shdy, T cf1,
                                              T sdphi, T g[4]) {
#pragma clang fp contract(off)
  const T imt = (a.c.mt > T(0)) ? div_budgeted(T(1), a.c.mt) : T(0);
  const T ie = (a.e > T(0)) ? div_budgeted(T(1), a.e) : T(0);
  const T pp = a.c.mt * b.c.mt;
  const T w = pp * shdy * ie * imt * imt;  // mTa mTb sinh(dy) / (mTa^2 Ea)
  const T sden = (a.c.pt * b.c.mt + b.c.pt * a.c.mt) * a.c.mt;
  const T diff = (sden > T(0)) ? div_budgeted(a.c.pt * a.c.pt * b.c.m2 - b.c.pt * b.c.pt * a.c.m2, sden) : T(0);
  g[0] = a.c.pt * b.c.mt * imt * sh2 + b.c.pt * cf1 + diff + w * a.sh * a.c.m2;
  g[1] = pp * shdy * a.c.pt * a.ch * ie;
  g[2] = a.c.pt * b.c.pt * sdphi;
  g[3] = a.mass + a.mass * imt * b.c.mt * chdy - w * a.c.pt * a.sh * a.mass;
}

// Both legs' gradients of the cancellation-free pair mass times gm.
template <typename T>
__device__ __forceinline__ void comp_pair_vjp(const LegCJ<T>& a, const LegCJ<T>& b, T gm, T ga[4], T gb[4]) {
#pragma clang fp contract(off)
  const T dy = (a.c.eta - b.c.eta) + (a.c.delta - b.c.delta);
  T s1;
  if constexpr (sizeof(T) == 8)
    s1 = fast_sinh<false>(T(0.5) * dy);
  else
    s1 = fast_sinh(T(0.5) * dy);
  const T c1 = sqrt_budgeted(T(1) + s1 * s1);
  const T sh2 = T(2) * s1 * s1;  // cosh(dy) - 1
  const T shdy = T(2) * s1 * c1;
  const T chdy = T(1) + sh2;
  const T h = T(0.5) * dphi_reduced(a.c.phi, b.c.phi);
  // sine and cosine of the half difference from the reduced sincos: its
  // reduction by pi/2 keeps cos(h) accurate next to |h| = pi/2, where
  // sqrt(1 - sin^2) would cancel (sin(dphi) of nearly back-to-back legs)
  T hs, hc;
  if constexpr (sizeof(T) == 8)
    fast_sincos<false>(h, &hs, &hc);
  else
    fast_sincos(h, &hs, &hc);
  const T cf1 = T(2) * hs * hs;  // 1 - cos(dphi)
  const T sdphi = T(2) * hs * hc;
  // m^2 of the forward form from the same pieces: t1 = mTa mTb (cosh dy - 1),
  // t2 = pta ptb (1 - cos dphi), t3 = (mTa - pta) mTb + pta (mTb - ptb)
  const T t3 = fma_t(a.c.dmt, b.c.mt, a.c.pt * b.c.dmt);
  const T m2 = (a.c.m2 + b.c.m2) + T(2) * (((a.c.mt * b.c.mt) * sh2 + (a.c.pt * b.c.pt) * cf1) + t3);
  const T s = (m2 > T(0)) ? gm * inv_sqrt(m2) : T(0);
  T ra[4], rb[4];
  comp_leg_rows<T>(a, b, sh2, chdy, shdy, cf1, sdphi, ra);
  comp_leg_rows<T>(b, a, sh2, chdy, -shdy, cf1, -sdphi, rb);
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    ga[k2] = s * ra[k2];
    gb[k2] = s * rb[k2];
  }
}

}  // namespace glv
