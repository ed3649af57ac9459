// Element-wise gfx950 kernels over SoA columns: pair invariant mass (plain
// and cancellation-free), its reverse mode, and the Lorentz boost with its
// reverse mode (GenVectorX Sec. 4.1: InvariantMasses and ApplyBoost, one
// independent result per item), coordinate conversion, and general Lorentz
// transformations and rotations (Sec. 3.1) with their reverse modes.
//
// Every op streams its columns exactly once, so the kernels are built for
// HBM bandwidth: each lane moves 16 bytes per column per step (2 doubles or
// 4 floats) with non-temporal loads and stores, one wavefront covers a
// contiguous 1 KiB of every column, and the grid has one lane per pack (a
// grid-stride loop only takes over beyond 2^31 workgroups).  Columns not
// aligned to 16 bytes take the same code with one element per lane.
#include "glv_device.h"
#include "glv_launch.h"

namespace glv {
namespace {

// Workgroup sizes (measured on MI355X: the streaming kernels run fastest with
// 128 threads, the ALU-heavier compensated mass with 256).
constexpr int kBlockStream = 128;
constexpr int kBlockAlu = 256;

// ---------------------------------------------------------------- driver

// Runs op.run<V>(i) over packs i in [0, n / V), then op.run<1>(t) over the
// tail elements t in [V (n / V), n).  run() returns how many of its items
// were recomputed in FP64; the total is added to *counter (one atomic per
// wavefront with a non-zero count).
template <typename Op, int V>
__global__ __launch_bounds__(Op::kBlock) void k_stream(Op op, int64_t n, unsigned long long* counter) {
  const int64_t nv = n / V;
  const int64_t stride = (int64_t)gridDim.x * Op::kBlock;
  const int64_t tid = (int64_t)blockIdx.x * Op::kBlock + threadIdx.x;
  unsigned cnt = 0;
  for (int64_t i = tid; i < nv; i += stride) cnt += op.template run<V>(i);
  if constexpr (V > 1) {
    const int64_t t = nv * V + tid;
    if (t < n) cnt += op.template run<1>(t);
  }
  if constexpr (Op::kCounts) {
    if (counter) {
      // wavefront sum, then lane 0 adds it with one vector atomic
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
      if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(counter, (unsigned long long)cnt);
    }
  }
}

template <typename Op, int V>
hipError_t run_stream(const Op& op, int64_t n, unsigned long long* counter, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t packs = n / V;
  int64_t blocks = (packs + Op::kBlock - 1) / Op::kBlock;
  if (blocks < 1) blocks = 1;
  if (blocks > 0x7fffffff) blocks = 0x7fffffff;
  hipLaunchKernelGGL((k_stream<Op, V>), dim3((unsigned)blocks), dim3(Op::kBlock), 0, s, op, n, counter);
  return hipGetLastError();
}

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <typename T, typename Op>
hipError_t dispatch_width(const Op& op, bool all_aligned, int64_t n, unsigned long long* counter,
                          hipStream_t s) {
  if (all_aligned) return run_stream<Op, Vec16<T>::N>(op, n, counter, s);
  return run_stream<Op, 1>(op, n, counter, s);
}

// ------------------------------------------------ mass -> histogram, fused

// Pair masses binned as they are computed, never stored: the mass op's
// masses<V>() over packs (grid-stride), each mass's counter slot in binary64
// (hist_slot), counters in LDS per workgroup merged into the global ones
// with one atomic per non-empty slot; with more slots than LDS holds, one
// global atomic per mass.
constexpr int kFusedHistBlock = 512;

template <typename Op, int V, bool kLds>
__global__ __launch_bounds__(kFusedHistBlock) void k_mass_hist(Op op, int64_t n, HistSpec h,
                                                               unsigned long long* __restrict__ counts,
                                                               unsigned long long* fb) {
  __shared__ unsigned int bins[kLds ? kHistLdsSlots : 1];
  const int nslot = (int)h.nb + 2;
  if constexpr (kLds) {
    for (int b = threadIdx.x; b < nslot; b += kFusedHistBlock) bins[b] = 0;
    __syncthreads();
  }
  auto count = [&](double v) {
    const int64_t sl = hist_slot(v, h);
    if (sl >= 0) {
      if constexpr (kLds)
        atomicAdd(&bins[sl], 1u);
      else
        atomicAdd(&counts[sl], 1ull);
    }
  };
  const int64_t nv = n / V;
  const int64_t stride = (int64_t)gridDim.x * kFusedHistBlock;
  const int64_t tid = (int64_t)blockIdx.x * kFusedHistBlock + threadIdx.x;
  unsigned cnt = 0;
  for (int64_t i = tid; i < nv; i += stride) {
    Pack<typename Op::Scalar, V> m;
    cnt += op.template masses<V>(i, m);
#pragma unroll
    for (int e = 0; e < V; ++e) count((double)m.v[e]);
  }
  if constexpr (V > 1) {
    const int64_t t = nv * V + tid;
    if (t < n) {
      Pack<typename Op::Scalar, 1> m;
      cnt += op.template masses<1>(t, m);
      count((double)m.v[0]);
    }
  }
  if constexpr (Op::kCounts) {
    if (fb) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
      if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(fb, (unsigned long long)cnt);
    }
  }
  if constexpr (kLds) {
    __syncthreads();
    for (int b = threadIdx.x; b < nslot; b += kFusedHistBlock)
      if (bins[b]) atomicAdd(&counts[b], (unsigned long long)bins[b]);
  }
}

// ------------------------------------------------------------ pair mass

// masses<V>(i, out) evaluates the masses of pack i (returning the number of
// FP64 redos); run<V>(i) stores them.  The fused histogram kernel calls
// masses<V> too, so both see bitwise the same masses.
template <typename T, int COORDS>
struct MassPlain {
  using Scalar = T;
  static constexpr bool kCounts = false;
  static constexpr int kBlock = kBlockStream;
  Cols4<T> a, b;
  T* m;
  template <int V>
  __device__ __forceinline__ unsigned masses(int64_t i, Pack<T, V>& out) const {
    Pack<T, V> pa[4], pb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      pa[k] = load_pack<T, V>(a.c[k], i);
      pb[k] = load_pack<T, V>(b.c[k], i);
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
      T va[4], vb[4], w[4];
      to_cart<COORDS>(pa[0].v[e], pa[1].v[e], pa[2].v[e], pa[3].v[e], va);
      to_cart<COORDS>(pb[0].v[e], pb[1].v[e], pb[2].v[e], pb[3].v[e], vb);
      add4<T>(va, vb, w);
      out.v[e] = mass_of(w);
    }
    return 0;
  }
  template <int V>
  __device__ __forceinline__ unsigned run(int64_t i) const {
    Pack<T, V> out;
    const unsigned c = masses<V>(i, out);
    store_pack<T, V>(m, i, out);
    return c;
  }
};

// Cancellation-free pair mass of PtEtaPhiM legs.  FP32 items whose running
// error bound exceeds kFallbackUnits are recomputed in FP64.
template <typename T>
struct MassComp {
  using Scalar = T;
  static constexpr bool kCounts = true;
  static constexpr int kBlock = kBlockAlu;
  Cols4<T> a, b;
  T* m;
  template <int V>
  __device__ __forceinline__ unsigned run(int64_t i) const {
    Pack<T, V> out;
    const unsigned c = masses<V>(i, out);
    store_pack<T, V>(m, i, out);
    return c;
  }
  template <int V>
  __device__ __forceinline__ unsigned masses(int64_t i, Pack<T, V>& out) const {
    Pack<T, V> pa[4], pb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      pa[k] = load_pack<T, V>(a.c[k], i);
      pb[k] = load_pack<T, V>(b.c[k], i);
    }
    unsigned cnt = 0;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      LegC<T> la = comp_leg<T>(pa[0].v[e], pa[1].v[e], pa[2].v[e], pa[3].v[e]);
      LegC<T> lb = comp_leg<T>(pb[0].v[e], pb[1].v[e], pb[2].v[e], pb[3].v[e]);
      T k;
      if constexpr (sizeof(T) == 4) {
        bool redo;
        T m2 = comp_pair_m2<T>(la, lb, &k, &redo);
        if (redo) {
          LegC<double> da = comp_leg<double, true>(pa[0].v[e], pa[1].v[e], pa[2].v[e], pa[3].v[e]);
          LegC<double> db = comp_leg<double, true>(pb[0].v[e], pb[1].v[e], pb[2].v[e], pb[3].v[e]);
          double kd;
          double m2d = comp_pair_m2<double, true>(da, db, &kd, nullptr);
          out.v[e] = (T)sqrt(m2d);
          ++cnt;
        } else {
          out.v[e] = sqrt_budgeted(m2);
        }
      } else {
        out.v[e] = d_sqrt(comp_pair_m2<T>(la, lb, &k, nullptr));
      }
    }
    return cnt;
  }
};

// Reverse mode: recompute the legs, then (-P, E)/|m| chained per leg.
template <typename T, int COORDS>
struct MassBwd {
  static constexpr bool kCounts = false;
  static constexpr int kBlock = kBlockStream;
  Cols4<T> a, b;
  const T* gm;
  OutCols4<T> ga, gb;
  template <int V>
  __device__ __forceinline__ unsigned run(int64_t i) const {
    Pack<T, V> pa[4], pb[4], pg, oa[4], ob[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      pa[k] = load_pack<T, V>(a.c[k], i);
      pb[k] = load_pack<T, V>(b.c[k], i);
    }
    pg = load_pack<T, V>(gm, i);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      LegJ<T> la = to_cart_j<COORDS, T>(pa[0].v[e], pa[1].v[e], pa[2].v[e], pa[3].v[e]);
      LegJ<T> lb = to_cart_j<COORDS, T>(pb[0].v[e], pb[1].v[e], pb[2].v[e], pb[3].v[e]);
      T w[4], u[4], g[4];
      add4<T>(la.v, lb.v, w);
      dmass<T>(w, pg.v[e], u);
      chain_coords<COORDS, T>(la, pa[0].v[e], pa[3].v[e], u, g);
#pragma unroll
      for (int k = 0; k < 4; ++k) oa[k].v[e] = g[k];
      chain_coords<COORDS, T>(lb, pb[0].v[e], pb[3].v[e], u, g);
#pragma unroll
      for (int k = 0; k < 4; ++k) ob[k].v[e] = g[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      store_pack<T, V>(ga.c[k], i, oa[k]);
      store_pack<T, V>(gb.c[k], i, ob[k]);
    }
    return 0;
  }
};

// Reverse mode of the cancellation-free pair mass (PtEtaPhiM legs): the
// gradient rows built from the forward form's own terms.
template <typename T>
struct MassCompBwd {
  static constexpr bool kCounts = false;
  // 128 threads: 196 against 205 us for 2^24 FP32 pairs at 256
  static constexpr int kBlock = kBlockStream;
  Cols4<T> a, b;
  const T* gm;
  OutCols4<T> ga, gb;
  template <int V>
  __device__ __forceinline__ unsigned run(int64_t i) const {
    Pack<T, V> pa[4], pb[4], pg, oa[4], ob[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      pa[k] = load_pack<T, V>(a.c[k], i);
      pb[k] = load_pack<T, V>(b.c[k], i);
    }
    pg = load_pack<T, V>(gm, i);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const LegCJ<T> la = comp_leg_j<T>(pa[0].v[e], pa[1].v[e], pa[2].v[e], pa[3].v[e]);
      const LegCJ<T> lb = comp_leg_j<T>(pb[0].v[e], pb[1].v[e], pb[2].v[e], pb[3].v[e]);
      T ra[4], rb[4];
      comp_pair_vjp<T>(la, lb, pg.v[e], ra, rb);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        oa[k].v[e] = ra[k];
        ob[k].v[e] = rb[k];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      store_pack<T, V>(ga.c[k], i, oa[k]);
      store_pack<T, V>(gb.c[k], i, ob[k]);
    }
    return 0;
  }
};

// ------------------------------------------------------------ conversion

// Coordinates TO of vectors given in FROM (through the Cartesian components;
// FROM == TO copies).
template <typename T, int FROM, int TO>
struct Convert {
  static constexpr bool kCounts = false;
  static constexpr int kBlock = kBlockStream;
  Cols4<T> in;
  OutCols4<T> out;
  template <int V>
  __device__ __forceinline__ unsigned run(int64_t i) const {
    Pack<T, V> pc[4], po[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) pc[k] = load_pack<T, V>(in.c[k], i);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      if constexpr (FROM == TO) {
#pragma unroll
        for (int k = 0; k < 4; ++k) po[k].v[e] = pc[k].v[e];
      } else {
        T v[4], c[4];
        to_cart<FROM>(pc[0].v[e], pc[1].v[e], pc[2].v[e], pc[3].v[e], v);
        from_cart<TO, T>(v, c);
#pragma unroll
        for (int k = 0; k < 4; ++k) po[k].v[e] = c[k];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) store_pack<T, V>(out.c[k], i, po[k]);
    return 0;
  }
};

// Reverse mode: the Cartesian gradient of the target coordinates, chained
// back through the source conversion's Jacobian; FROM == TO passes through.
template <typename T, int FROM, int TO>
struct ConvertBwd {
  static constexpr bool kCounts = false;
  static constexpr int kBlock = kBlockStream;
  Cols4<T> in, gout;
  OutCols4<T> gin;
  template <int V>
  __device__ __forceinline__ unsigned run(int64_t i) const {
    Pack<T, V> pc[4], pg[4], po[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      pg[k] = load_pack<T, V>(gout.c[k], i);
      if constexpr (FROM != TO) pc[k] = load_pack<T, V>(in.c[k], i);
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
      if constexpr (FROM == TO) {
#pragma unroll
        for (int k = 0; k < 4; ++k) po[k].v[e] = pg[k].v[e];
      } else {
        const LegJ<T> L = to_cart_j<FROM, T>(pc[0].v[e], pc[1].v[e], pc[2].v[e], pc[3].v[e]);
        T gc[4], u[4], g[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) gc[k] = pg[k].v[e];
        dcoords_dcart<TO, T>(L.v, gc, u);
        chain_coords<FROM, T>(L, pc[0].v[e], pc[3].v[e], u, g);
#pragma unroll
        for (int k = 0; k < 4; ++k) po[k].v[e] = g[k];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) store_pack<T, V>(gin.c[k], i, po[k]);
    return 0;
  }
};

// ----------------------------------------------------------------- boost

// gamma and kappa = gamma^2/(1 + gamma) from the velocity, formed in FP64
// (for FP32 data the rounding of beta^2 would otherwise be magnified by
// gamma^2 in 1 - beta^2).
struct BoostCoef {
  double g, k;
};
__device__ __forceinline__ BoostCoef boost_coef(double bx, double by, double bz) {
  double b2 = bx * bx + by * by + bz * bz;
  double g = 1.0 / sqrt(1.0 - b2);
  return {g, g * g / (1.0 + g)};
}

template <typename T, int BSTRIDE>
struct BoostFwd {
  static constexpr bool kCounts = false;
  static constexpr int kBlock = kBlockStream;
  Cols4<T> x;
  Cols3<T> beta;
  OutCols4<T> y;
  template <int V>
  __device__ __forceinline__ unsigned run(int64_t i) const {
    Pack<T, V> px[4], pb[3], out[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) px[k] = load_pack<T, V>(x.c[k], i);
    if constexpr (BSTRIDE == 1) {
#pragma unroll
      for (int k = 0; k < 3; ++k) pb[k] = load_pack<T, V>(beta.c[k], i);
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        T v = beta.c[k][0];
#pragma unroll
        for (int e = 0; e < V; ++e) pb[k].v[e] = v;
      }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
      T bx = pb[0].v[e], by = pb[1].v[e], bz = pb[2].v[e];
      BoostCoef c = boost_coef(bx, by, bz);
      T g = (T)c.g, kap = (T)c.k;
      T p0 = px[0].v[e], p1 = px[1].v[e], p2 = px[2].v[e], en = px[3].v[e];
      T sdot = bx * p0 + by * p1 + bz * p2;
      T cc = kap * sdot + g * en;
      out[3].v[e] = g * (en + sdot);
      out[0].v[e] = p0 + cc * bx;
      out[1].v[e] = p1 + cc * by;
      out[2].v[e] = p2 + cc * bz;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) store_pack<T, V>(y.c[k], i, out[k]);
    return 0;
  }
};

// Reverse mode of the boost: grad_x = L(beta) grad_y; grad_beta in closed form.
template <typename T, int BSTRIDE, bool WANT_GB>
struct BoostBwd {
  static constexpr bool kCounts = false;
  static constexpr int kBlock = kBlockStream;
  Cols4<T> x;
  Cols3<T> beta;
  Cols4<T> gy;
  OutCols4<T> gx;
  OutCols3<T> gb;
  template <int V>
  __device__ __forceinline__ unsigned run(int64_t i) const {
    Pack<T, V> px[4], pb[3], pg[4], ox[4], ob[3];
#pragma unroll
    for (int k = 0; k < 4; ++k) pg[k] = load_pack<T, V>(gy.c[k], i);
    if constexpr (WANT_GB) {
#pragma unroll
      for (int k = 0; k < 4; ++k) px[k] = load_pack<T, V>(x.c[k], i);
    }
    if constexpr (BSTRIDE == 1) {
#pragma unroll
      for (int k = 0; k < 3; ++k) pb[k] = load_pack<T, V>(beta.c[k], i);
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        T v = beta.c[k][0];
#pragma unroll
        for (int e = 0; e < V; ++e) pb[k].v[e] = v;
      }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
      T b[3] = {pb[0].v[e], pb[1].v[e], pb[2].v[e]};
      BoostCoef c = boost_coef(b[0], b[1], b[2]);
      T g = (T)c.g, kap = (T)c.k;
      T gp[3] = {pg[0].v[e], pg[1].v[e], pg[2].v[e]};
      T ge = pg[3].v[e];
      T gdb = gp[0] * b[0] + gp[1] * b[1] + gp[2] * b[2];
      T cc = kap * gdb + g * ge;
      ox[3].v[e] = g * (ge + gdb);
#pragma unroll
      for (int d = 0; d < 3; ++d) ox[d].v[e] = gp[d] + cc * b[d];
      if constexpr (WANT_GB) {
        double gd = c.g;
        T g3 = (T)(gd * gd * gd);
        T kp = (T)(gd * (gd + 2.0) / ((1.0 + gd) * (1.0 + gd)));
        T p[3] = {px[0].v[e], px[1].v[e], px[2].v[e]};
        T en = px[3].v[e];
        T sdot = b[0] * p[0] + b[1] * p[1] + b[2] * p[2];
        T ce = g3 * (en + sdot);
        T cq = kp * g3 * sdot + g3 * en;
        T cr = kap * sdot + g * en;
#pragma unroll
        for (int d = 0; d < 3; ++d)
          ob[d].v[e] = ge * (ce * b[d] + g * p[d]) + gdb * (cq * b[d] + kap * p[d]) + cr * gp[d];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) store_pack<T, V>(gx.c[k], i, ox[k]);
    if constexpr (WANT_GB) {
#pragma unroll
      for (int k = 0; k < 3; ++k) store_pack<T, V>(gb.c[k], i, ob[k]);
    }
    return 0;
  }
};

// ------------------------------------------------ general transformations

// Parameters per item of each kind: a 4x4 Lorentz matrix, a 3x3 rotation
// matrix, or an axis and an angle (all row-major columns).
template <int KIND>
struct TfParams {
  static constexpr int K = KIND == kTfLorentz ? 16 : (KIND == kTfRot3 ? 9 : 4);
  static constexpr int N = KIND == kTfLorentz ? 4 : 3;  // order of the matrix
};

template <typename T, int K>
struct ColsK {
  const T* c[K];
};
template <typename T, int K>
struct OutColsK {
  T* c[K];
};

// Rotation matrix of an axis a and an angle t by Rodrigues' formula,
// R = cos t I + sin t [u]x + (1 - cos t) u u^T with u = a/|a|; a zero axis
// gives the identity.
template <typename T>
__device__ __forceinline__ void axis_angle_matrix(T ax, T ay, T az, T t, T r[9]) {
  const T l2 = ax * ax + ay * ay + az * az;
  const bool axis = l2 > T(0);
  const T il = axis ? inv_sqrt(l2) : T(0);
  const T u0 = ax * il, u1 = ay * il, u2 = az * il;
  T sn, cs;
  sincos_t<false>(t, &sn, &cs);
  sn = axis ? sn : T(0);
  cs = axis ? cs : T(1);
  const T w = T(1) - cs;
  r[0] = cs + u0 * u0 * w;
  r[1] = u0 * u1 * w - u2 * sn;
  r[2] = u0 * u2 * w + u1 * sn;
  r[3] = u1 * u0 * w + u2 * sn;
  r[4] = cs + u1 * u1 * w;
  r[5] = u1 * u2 * w - u0 * sn;
  r[6] = u2 * u0 * w - u1 * sn;
  r[7] = u2 * u1 * w + u0 * sn;
  r[8] = cs + u2 * u2 * w;
}

// Fused multiply-add in the element type.
__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }

// Parameter packs: per item (STRIDE 1) or one value for all items (STRIDE 0).
template <typename T, int V, int STRIDE, int K>
__device__ __forceinline__ void load_params(const ColsK<T, K>& m, int64_t i, Pack<T, V> (&p)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if constexpr (STRIDE == 1) {
      p[k] = load_pack<T, V>(m.c[k], i);
    } else {
      const T v = m.c[k][0];
#pragma unroll
      for (int e = 0; e < V; ++e) p[k].v[e] = v;
    }
  }
}

// The N x N matrix of element e.
template <typename T, int KIND, int V, int K>
__device__ __forceinline__ void matrix_of(const Pack<T, V> (&p)[K], int e, T mat[TfParams<KIND>::N * TfParams<KIND>::N]) {
  if constexpr (KIND == kTfAxisAngle) {
    axis_angle_matrix<T>(p[0].v[e], p[1].v[e], p[2].v[e], p[3].v[e], mat);
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) mat[k] = p[k].v[e];
  }
}

// y = L x (Lorentz: all four components) or p' = R p, E' = E (rotations).
template <typename T, int KIND, int STRIDE>
struct TransformFwd {
  static constexpr bool kCounts = false;
  static constexpr int kBlock = kBlockStream;
  static constexpr int K = TfParams<KIND>::K, N = TfParams<KIND>::N;
  Cols4<T> x;
  ColsK<T, K> m;
  OutCols4<T> y;
  template <int V>
  __device__ __forceinline__ unsigned run(int64_t i) const {
    Pack<T, V> px[4], pm[K], out[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) px[k] = load_pack<T, V>(x.c[k], i);
    load_params<T, V, STRIDE, K>(m, i, pm);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      T mat[N * N];
      matrix_of<T, KIND, V, K>(pm, e, mat);
#pragma unroll
      for (int a = 0; a < N; ++a) {
        T acc = mat[N * a] * px[0].v[e];
#pragma unroll
        for (int c = 1; c < N; ++c) acc = fma_t(mat[N * a + c], px[c].v[e], acc);
        out[a].v[e] = acc;
      }
      if constexpr (N == 3) out[3].v[e] = px[3].v[e];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) store_pack<T, V>(y.c[k], i, out[k]);
    return 0;
  }
};

// Reverse mode: grad_x = M^T grad_y (E passes through a rotation); with
// WANT_GM the per-item matrix gradient grad_M[N a + c] = grad_y_a x_c.
template <typename T, int KIND, int STRIDE, bool WANT_GM>
struct TransformBwd {
  static constexpr bool kCounts = false;
  static constexpr int kBlock = kBlockStream;
  static constexpr int K = TfParams<KIND>::K, N = TfParams<KIND>::N;
  Cols4<T> x, gy;
  ColsK<T, K> m;
  OutCols4<T> gx;
  OutColsK<T, N * N> gm;
  template <int V>
  __device__ __forceinline__ unsigned run(int64_t i) const {
    Pack<T, V> pg[4], px[4], pm[K], ox[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      pg[k] = load_pack<T, V>(gy.c[k], i);
      if constexpr (WANT_GM) px[k] = load_pack<T, V>(x.c[k], i);
    }
    load_params<T, V, STRIDE, K>(m, i, pm);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      T mat[N * N];
      matrix_of<T, KIND, V, K>(pm, e, mat);
#pragma unroll
      for (int c = 0; c < N; ++c) {
        T acc = mat[c] * pg[0].v[e];
#pragma unroll
        for (int a = 1; a < N; ++a) acc = fma_t(mat[N * a + c], pg[a].v[e], acc);
        ox[c].v[e] = acc;
      }
      if constexpr (N == 3) ox[3].v[e] = pg[3].v[e];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) store_pack<T, V>(gx.c[k], i, ox[k]);
    if constexpr (WANT_GM) {
#pragma unroll
      for (int a = 0; a < N; ++a) {
#pragma unroll
        for (int c = 0; c < N; ++c) {
          Pack<T, V> o;
#pragma unroll
          for (int e = 0; e < V; ++e) o.v[e] = pg[a].v[e] * px[c].v[e];
          store_pack<T, V>(gm.c[N * a + c], i, o);
        }
      }
    }
    return 0;
  }
};

template <typename T>
Cols4<T> cols4(const void* const p[4]) {
  return {{(const T*)p[0], (const T*)p[1], (const T*)p[2], (const T*)p[3]}};
}
template <typename T>
Cols3<T> cols3(const void* const p[3]) {
  return {{(const T*)p[0], (const T*)p[1], (const T*)p[2]}};
}
template <typename T>
OutCols4<T> out4(void* const p[4]) {
  return {{(T*)p[0], (T*)p[1], (T*)p[2], (T*)p[3]}};
}
template <typename T>
OutCols3<T> out3(void* const p[3]) {
  if (!p) return {{nullptr, nullptr, nullptr}};
  return {{(T*)p[0], (T*)p[1], (T*)p[2]}};
}

template <int N>
bool all16(const void* const* p) {
  for (int k = 0; k < N; ++k)
    if (!aligned16(p[k])) return false;
  return true;
}

template <typename T>
hipError_t mass_typed(glv_coords co, glv_mode mode, int64_t n, const void* const a[4],
                      const void* const b[4], void* m, unsigned long long* fb, hipStream_t s) {
  bool al = all16<4>(a) && all16<4>(b) && aligned16(m);
  Cols4<T> ca = cols4<T>(a), cb = cols4<T>(b);
  if (mode == GLV_COMPENSATED) return dispatch_width<T>(MassComp<T>{ca, cb, (T*)m}, al, n, fb, s);
  switch (co) {
    case GLV_PXPYPZE:
      return dispatch_width<T>(MassPlain<T, GLV_PXPYPZE>{ca, cb, (T*)m}, al, n, nullptr, s);
    case GLV_PTETAPHIM:
      return dispatch_width<T>(MassPlain<T, GLV_PTETAPHIM>{ca, cb, (T*)m}, al, n, nullptr, s);
    case GLV_PXPYPZM:
      return dispatch_width<T>(MassPlain<T, GLV_PXPYPZM>{ca, cb, (T*)m}, al, n, nullptr, s);
    default:
      return dispatch_width<T>(MassPlain<T, GLV_PTETAPHIE>{ca, cb, (T*)m}, al, n, nullptr, s);
  }
}

template <typename Op>
hipError_t run_mass_hist(const Op& op, bool al, int64_t n, const HistSpec& h, unsigned long long* counts,
                         unsigned long long* fb, hipStream_t s) {
  using T = typename Op::Scalar;
  constexpr int V = Vec16<T>::N;
  const bool lds = h.nb + 2 <= kHistLdsSlots;
  const int64_t packs = al ? n / V : n;
  int64_t blocks = (packs + kFusedHistBlock - 1) / kFusedHistBlock;
  // the LDS path merges once per workgroup: 1024 workgroups (32 wavefronts
  // per CU) keep the streams busy without multiplying the merges
  const int64_t cap = lds ? 1024 : 65536;
  blocks = blocks < 1 ? 1 : (blocks > cap ? cap : blocks);
  const dim3 g((unsigned)blocks), b(kFusedHistBlock);
  if (al && lds)
    hipLaunchKernelGGL((k_mass_hist<Op, V, true>), g, b, 0, s, op, n, h, counts, fb);
  else if (al)
    hipLaunchKernelGGL((k_mass_hist<Op, V, false>), g, b, 0, s, op, n, h, counts, fb);
  else if (lds)
    hipLaunchKernelGGL((k_mass_hist<Op, 1, true>), g, b, 0, s, op, n, h, counts, fb);
  else
    hipLaunchKernelGGL((k_mass_hist<Op, 1, false>), g, b, 0, s, op, n, h, counts, fb);
  return hipGetLastError();
}

template <typename T>
hipError_t mass_hist_typed(glv_coords co, glv_mode mode, int64_t n, const void* const a[4], const void* const b[4],
                           const HistSpec& h, unsigned long long* counts, unsigned long long* fb, hipStream_t s) {
  const bool al = all16<4>(a) && all16<4>(b);
  Cols4<T> ca = cols4<T>(a), cb = cols4<T>(b);
  if (mode == GLV_COMPENSATED) return run_mass_hist(MassComp<T>{ca, cb, nullptr}, al, n, h, counts, fb, s);
  switch (co) {
    case GLV_PXPYPZE:
      return run_mass_hist(MassPlain<T, GLV_PXPYPZE>{ca, cb, nullptr}, al, n, h, counts, nullptr, s);
    case GLV_PTETAPHIM:
      return run_mass_hist(MassPlain<T, GLV_PTETAPHIM>{ca, cb, nullptr}, al, n, h, counts, nullptr, s);
    case GLV_PXPYPZM:
      return run_mass_hist(MassPlain<T, GLV_PXPYPZM>{ca, cb, nullptr}, al, n, h, counts, nullptr, s);
    default:
      return run_mass_hist(MassPlain<T, GLV_PTETAPHIE>{ca, cb, nullptr}, al, n, h, counts, nullptr, s);
  }
}

template <typename T>
hipError_t mass_bwd_typed(glv_coords co, int64_t n, const void* const a[4], const void* const b[4],
                          const void* gm, void* const ga[4], void* const gb[4], hipStream_t s) {
  bool al = all16<4>(a) && all16<4>(b) && aligned16(gm) && all16<4>((const void* const*)ga) &&
            all16<4>((const void* const*)gb);
  Cols4<T> ca = cols4<T>(a), cb = cols4<T>(b);
  OutCols4<T> oa = out4<T>(ga), ob = out4<T>(gb);
  const T* g = (const T*)gm;
  switch (co) {
    case GLV_PXPYPZE:
      return dispatch_width<T>(MassBwd<T, GLV_PXPYPZE>{ca, cb, g, oa, ob}, al, n, nullptr, s);
    case GLV_PTETAPHIM:
      return dispatch_width<T>(MassBwd<T, GLV_PTETAPHIM>{ca, cb, g, oa, ob}, al, n, nullptr, s);
    case GLV_PXPYPZM:
      return dispatch_width<T>(MassBwd<T, GLV_PXPYPZM>{ca, cb, g, oa, ob}, al, n, nullptr, s);
    default:
      return dispatch_width<T>(MassBwd<T, GLV_PTETAPHIE>{ca, cb, g, oa, ob}, al, n, nullptr, s);
  }
}

template <typename T>
hipError_t boost_typed(int64_t n, const void* const x[4], const void* const beta[3], int64_t bs,
                       void* const y[4], hipStream_t s) {
  bool al = all16<4>(x) && all16<4>((const void* const*)y) && (bs == 0 || all16<3>(beta));
  if (bs == 1) return dispatch_width<T>(BoostFwd<T, 1>{cols4<T>(x), cols3<T>(beta), out4<T>(y)}, al, n, nullptr, s);
  return dispatch_width<T>(BoostFwd<T, 0>{cols4<T>(x), cols3<T>(beta), out4<T>(y)}, al, n, nullptr, s);
}

template <typename T>
hipError_t boost_bwd_typed(int64_t n, const void* const x[4], const void* const beta[3], int64_t bs,
                           const void* const gy[4], void* const gx[4], void* const gb[3],
                           hipStream_t s) {
  bool want = gb != nullptr;
  bool al = all16<4>(gy) && all16<4>((const void* const*)gx) && (bs == 0 || all16<3>(beta)) &&
            (!want || (all16<4>(x) && all16<3>((const void* const*)gb)));
  Cols4<T> cx = want ? cols4<T>(x) : Cols4<T>{{nullptr, nullptr, nullptr, nullptr}};
  Cols3<T> cbeta = cols3<T>(beta);
  if (want) {
    // grad_beta is per item: beta_stride 1 only (checked by the caller)
    return dispatch_width<T>(BoostBwd<T, 1, true>{cx, cbeta, cols4<T>(gy), out4<T>(gx), out3<T>(gb)}, al, n,
                             nullptr, s);
  }
  if (bs == 1)
    return dispatch_width<T>(BoostBwd<T, 1, false>{cx, cbeta, cols4<T>(gy), out4<T>(gx), out3<T>(nullptr)}, al,
                             n, nullptr, s);
  return dispatch_width<T>(BoostBwd<T, 0, false>{cx, cbeta, cols4<T>(gy), out4<T>(gx), out3<T>(nullptr)}, al, n,
                           nullptr, s);
}

template <typename T, int K>
ColsK<T, K> colsk(const void* const* p) {
  ColsK<T, K> r;
#pragma unroll
  for (int k = 0; k < K; ++k) r.c[k] = p ? (const T*)p[k] : nullptr;
  return r;
}
template <typename T, int K>
OutColsK<T, K> outk(void* const* p) {
  OutColsK<T, K> r;
#pragma unroll
  for (int k = 0; k < K; ++k) r.c[k] = p ? (T*)p[k] : nullptr;
  return r;
}

template <typename T, int KIND>
hipError_t transform_typed(int64_t n, const void* const x[4], const void* const* m, int64_t ms, void* const y[4],
                           hipStream_t s) {
  constexpr int K = TfParams<KIND>::K;
  const bool al = all16<4>(x) && all16<4>((const void* const*)y) && (ms == 0 || all16<K>(m));
  const ColsK<T, K> cm = colsk<T, K>(m);
  if (ms == 1) return dispatch_width<T>(TransformFwd<T, KIND, 1>{cols4<T>(x), cm, out4<T>(y)}, al, n, nullptr, s);
  return dispatch_width<T>(TransformFwd<T, KIND, 0>{cols4<T>(x), cm, out4<T>(y)}, al, n, nullptr, s);
}

template <typename T, int KIND>
hipError_t transform_bwd_typed(int64_t n, const void* const x[4], const void* const* m, int64_t ms,
                               const void* const gy[4], void* const gx[4], void* const* gm, hipStream_t s) {
  constexpr int K = TfParams<KIND>::K, NN = TfParams<KIND>::N * TfParams<KIND>::N;
  const bool want = gm != nullptr;
  const bool al = all16<4>(gy) && all16<4>((const void* const*)gx) && (ms == 0 || all16<K>(m)) &&
                  (!want || (all16<4>(x) && all16<NN>((const void* const*)gm)));
  const Cols4<T> cx = want ? cols4<T>(x) : Cols4<T>{{nullptr, nullptr, nullptr, nullptr}};
  const ColsK<T, K> cm = colsk<T, K>(m);
  if constexpr (KIND != kTfAxisAngle) {
    if (want)  // per-item matrix gradients: stride 1 only (checked by the caller)
      return dispatch_width<T>(TransformBwd<T, KIND, 1, true>{cx, cols4<T>(gy), cm, out4<T>(gx), outk<T, NN>(gm)},
                               al, n, nullptr, s);
  }
  if (ms == 1)
    return dispatch_width<T>(TransformBwd<T, KIND, 1, false>{cx, cols4<T>(gy), cm, out4<T>(gx), outk<T, NN>(nullptr)},
                             al, n, nullptr, s);
  return dispatch_width<T>(TransformBwd<T, KIND, 0, false>{cx, cols4<T>(gy), cm, out4<T>(gx), outk<T, NN>(nullptr)},
                           al, n, nullptr, s);
}

template <typename T, int FROM>
hipError_t convert_to(glv_coords to, int64_t n, const void* const in[4], void* const out[4], hipStream_t s) {
  const bool al = all16<4>(in) && all16<4>((const void* const*)out);
  const Cols4<T> ci = cols4<T>(in);
  const OutCols4<T> co = out4<T>(out);
  switch (to) {
    case GLV_PXPYPZE:
      return dispatch_width<T>(Convert<T, FROM, GLV_PXPYPZE>{ci, co}, al, n, nullptr, s);
    case GLV_PTETAPHIM:
      return dispatch_width<T>(Convert<T, FROM, GLV_PTETAPHIM>{ci, co}, al, n, nullptr, s);
    case GLV_PXPYPZM:
      return dispatch_width<T>(Convert<T, FROM, GLV_PXPYPZM>{ci, co}, al, n, nullptr, s);
    default:
      return dispatch_width<T>(Convert<T, FROM, GLV_PTETAPHIE>{ci, co}, al, n, nullptr, s);
  }
}

template <typename T>
hipError_t convert_typed(glv_coords from, glv_coords to, int64_t n, const void* const in[4], void* const out[4],
                         hipStream_t s) {
  switch (from) {
    case GLV_PXPYPZE:
      return convert_to<T, GLV_PXPYPZE>(to, n, in, out, s);
    case GLV_PTETAPHIM:
      return convert_to<T, GLV_PTETAPHIM>(to, n, in, out, s);
    case GLV_PXPYPZM:
      return convert_to<T, GLV_PXPYPZM>(to, n, in, out, s);
    default:
      return convert_to<T, GLV_PTETAPHIE>(to, n, in, out, s);
  }
}

template <typename T, int FROM>
hipError_t convert_bwd_to(glv_coords to, int64_t n, const void* const in[4], const void* const gout[4],
                          void* const gin[4], hipStream_t s) {
  const bool al = all16<4>(in) && all16<4>(gout) && all16<4>((const void* const*)gin);
  const Cols4<T> ci = cols4<T>(in), cg = cols4<T>(gout);
  const OutCols4<T> co = out4<T>(gin);
  switch (to) {
    case GLV_PXPYPZE:
      return dispatch_width<T>(ConvertBwd<T, FROM, GLV_PXPYPZE>{ci, cg, co}, al, n, nullptr, s);
    case GLV_PTETAPHIM:
      return dispatch_width<T>(ConvertBwd<T, FROM, GLV_PTETAPHIM>{ci, cg, co}, al, n, nullptr, s);
    case GLV_PXPYPZM:
      return dispatch_width<T>(ConvertBwd<T, FROM, GLV_PXPYPZM>{ci, cg, co}, al, n, nullptr, s);
    default:
      return dispatch_width<T>(ConvertBwd<T, FROM, GLV_PTETAPHIE>{ci, cg, co}, al, n, nullptr, s);
  }
}

template <typename T>
hipError_t convert_bwd_typed(glv_coords from, glv_coords to, int64_t n, const void* const in[4],
                             const void* const gout[4], void* const gin[4], hipStream_t s) {
  switch (from) {
    case GLV_PXPYPZE:
      return convert_bwd_to<T, GLV_PXPYPZE>(to, n, in, gout, gin, s);
    case GLV_PTETAPHIM:
      return convert_bwd_to<T, GLV_PTETAPHIM>(to, n, in, gout, gin, s);
    case GLV_PXPYPZM:
      return convert_bwd_to<T, GLV_PXPYPZM>(to, n, in, gout, gin, s);
    default:
      return convert_bwd_to<T, GLV_PTETAPHIE>(to, n, in, gout, gin, s);
  }
}

}  // namespace

hipError_t launch_convert(glv_dtype dt, glv_coords from, glv_coords to, int64_t n, const void* const in[4],
                          void* const out[4], hipStream_t s) {
  if (dt == GLV_F64) return convert_typed<double>(from, to, n, in, out, s);
  return convert_typed<float>(from, to, n, in, out, s);
}

hipError_t launch_convert_bwd(glv_dtype dt, glv_coords from, glv_coords to, int64_t n, const void* const in[4],
                              const void* const gout[4], void* const gin[4], hipStream_t s) {
  if (dt == GLV_F64) return convert_bwd_typed<double>(from, to, n, in, gout, gin, s);
  return convert_bwd_typed<float>(from, to, n, in, gout, gin, s);
}

hipError_t launch_mass(glv_dtype dt, glv_coords co, glv_mode mode, int64_t n, const void* const a[4],
                       const void* const b[4], void* m, unsigned long long* fb, hipStream_t s) {
  if (dt == GLV_F64) return mass_typed<double>(co, mode, n, a, b, m, nullptr, s);
  return mass_typed<float>(co, mode, n, a, b, m, fb, s);
}

hipError_t launch_mass_histogram(glv_dtype dt, glv_coords co, glv_mode mode, int64_t n, const void* const a[4],
                                 const void* const b[4], double lo, double hi, int64_t n_bins,
                                 unsigned long long* counts, unsigned long long* fb, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const HistSpec h{lo, hi, (double)n_bins / (hi - lo), n_bins};
  if (dt == GLV_F64) return mass_hist_typed<double>(co, mode, n, a, b, h, counts, nullptr, s);
  return mass_hist_typed<float>(co, mode, n, a, b, h, counts, fb, s);
}

hipError_t launch_mass_comp_bwd(glv_dtype dt, int64_t n, const void* const a[4], const void* const b[4],
                                const void* gm, void* const ga[4], void* const gb[4], hipStream_t s) {
  const bool al = all16<4>(a) && all16<4>(b) && aligned16(gm) && all16<4>((const void* const*)ga) &&
                  all16<4>((const void* const*)gb);
  if (dt == GLV_F64)
    return dispatch_width<double>(MassCompBwd<double>{cols4<double>(a), cols4<double>(b), (const double*)gm,
                                                      out4<double>(ga), out4<double>(gb)},
                                  al, n, nullptr, s);
  return dispatch_width<float>(MassCompBwd<float>{cols4<float>(a), cols4<float>(b), (const float*)gm,
                                                  out4<float>(ga), out4<float>(gb)},
                               al, n, nullptr, s);
}

hipError_t launch_mass_bwd(glv_dtype dt, glv_coords co, int64_t n, const void* const a[4],
                           const void* const b[4], const void* gm, void* const ga[4],
                           void* const gb[4], hipStream_t s) {
  if (dt == GLV_F64) return mass_bwd_typed<double>(co, n, a, b, gm, ga, gb, s);
  return mass_bwd_typed<float>(co, n, a, b, gm, ga, gb, s);
}

hipError_t launch_boost(glv_dtype dt, int64_t n, const void* const x[4], const void* const beta[3],
                        int64_t bs, void* const y[4], hipStream_t s) {
  if (dt == GLV_F64) return boost_typed<double>(n, x, beta, bs, y, s);
  return boost_typed<float>(n, x, beta, bs, y, s);
}

hipError_t launch_boost_bwd(glv_dtype dt, int64_t n, const void* const x[4],
                            const void* const beta[3], int64_t bs, const void* const gy[4],
                            void* const gx[4], void* const gb[3], hipStream_t s) {
  if (dt == GLV_F64) return boost_bwd_typed<double>(n, x, beta, bs, gy, gx, gb, s);
  return boost_bwd_typed<float>(n, x, beta, bs, gy, gx, gb, s);
}

hipError_t launch_transform(glv_dtype dt, int kind, int64_t n, const void* const x[4], const void* const* m,
                            int64_t ms, void* const y[4], hipStream_t s) {
  const bool f64 = dt == GLV_F64;
  switch (kind) {
    case kTfLorentz:
      return f64 ? transform_typed<double, kTfLorentz>(n, x, m, ms, y, s)
                 : transform_typed<float, kTfLorentz>(n, x, m, ms, y, s);
    case kTfRot3:
      return f64 ? transform_typed<double, kTfRot3>(n, x, m, ms, y, s)
                 : transform_typed<float, kTfRot3>(n, x, m, ms, y, s);
    default:
      return f64 ? transform_typed<double, kTfAxisAngle>(n, x, m, ms, y, s)
                 : transform_typed<float, kTfAxisAngle>(n, x, m, ms, y, s);
  }
}

hipError_t launch_transform_bwd(glv_dtype dt, int kind, int64_t n, const void* const x[4], const void* const* m,
                                int64_t ms, const void* const gy[4], void* const gx[4], void* const* gm,
                                hipStream_t s) {
  const bool f64 = dt == GLV_F64;
  switch (kind) {
    case kTfLorentz:
      return f64 ? transform_bwd_typed<double, kTfLorentz>(n, x, m, ms, gy, gx, gm, s)
                 : transform_bwd_typed<float, kTfLorentz>(n, x, m, ms, gy, gx, gm, s);
    case kTfRot3:
      return f64 ? transform_bwd_typed<double, kTfRot3>(n, x, m, ms, gy, gx, gm, s)
                 : transform_bwd_typed<float, kTfRot3>(n, x, m, ms, gy, gx, gm, s);
    default:
      return f64 ? transform_bwd_typed<double, kTfAxisAngle>(n, x, m, ms, gy, gx, nullptr, s)
                 : transform_bwd_typed<float, kTfAxisAngle>(n, x, m, ms, gy, gx, nullptr, s);
  }
}

}  // namespace glv
