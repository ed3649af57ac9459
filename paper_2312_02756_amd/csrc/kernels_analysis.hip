// The analysis step after the mass (not in the paper; Sec. 6 places
// GenVector inside ROOT, which analyses such data): a histogram of masses,
// and per CSR event the pair whose mass lies closest to a target.
#include "glv_device.h"
#include "glv_launch.h"

namespace glv {
namespace {

constexpr int kHistBlock = 256;
// Counters (bins plus under- and overflow) a workgroup keeps in LDS: 32 KiB.
constexpr int kHistLdsSlots = 8192;
// Workgroups of the LDS path (two per CU): each merges its counters into the
// global ones once, so fewer, longer-lived workgroups mean fewer global atomics.
constexpr int64_t kHistGrid = 512;
constexpr int kBestBlock = 256;

struct HistSpec {
  double lo, hi, s;  // s = n_bins / (hi - lo), formed on the host
  int64_t nb;
};

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

// Per-workgroup counters in LDS, merged with one global atomic per non-empty
// slot.  Grid-stride over packs of V values (16-byte loads), then the tail.
template <typename T, int V>
__global__ __launch_bounds__(kHistBlock) void k_hist_lds(const T* __restrict__ v, int64_t n, HistSpec h,
                                                         unsigned long long* __restrict__ counts) {
  __shared__ unsigned int bins[kHistLdsSlots];
  const int nslot = (int)h.nb + 2;
  for (int b = threadIdx.x; b < nslot; b += kHistBlock) bins[b] = 0;
  __syncthreads();
  const int64_t nv = n / V;
  const int64_t tid = (int64_t)blockIdx.x * kHistBlock + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kHistBlock;
  for (int64_t i = tid; i < nv; i += stride) {
    const Pack<T, V> p = load_pack<T, V>(v, i);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const int64_t s = hist_slot((double)p.v[e], h);
      if (s >= 0) atomicAdd(&bins[s], 1u);
    }
  }
  if constexpr (V > 1) {
    const int64_t t = nv * V + tid;
    if (t < n) {
      const int64_t s = hist_slot((double)v[t], h);
      if (s >= 0) atomicAdd(&bins[s], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nslot; b += kHistBlock)
    if (bins[b]) atomicAdd(&counts[b], (unsigned long long)bins[b]);
}

// More slots than LDS holds: global atomics per value.
template <typename T>
__global__ __launch_bounds__(kHistBlock) void k_hist_global(const T* __restrict__ v, int64_t n, HistSpec h,
                                                            unsigned long long* __restrict__ counts) {
  const int64_t stride = (int64_t)gridDim.x * kHistBlock;
  for (int64_t i = (int64_t)blockIdx.x * kHistBlock + threadIdx.x; i < n; i += stride) {
    const int64_t s = hist_slot((double)v[i], h);
    if (s >= 0) atomicAdd(&counts[s], 1ull);
  }
}

template <typename T>
hipError_t hist_typed(int64_t n, const void* m, double lo, double hi, int64_t nb, unsigned long long* counts,
                      hipStream_t s) {
  const HistSpec h{lo, hi, (double)nb / (hi - lo), nb};
  const T* v = (const T*)m;
  if (nb + 2 <= kHistLdsSlots) {
    constexpr int V = Vec16<T>::N;
    const bool al = (reinterpret_cast<uintptr_t>(m) & 15) == 0;
    const int64_t packs = al ? n / V : n;
    int64_t blocks = (packs + kHistBlock - 1) / kHistBlock;
    blocks = blocks < 1 ? 1 : (blocks > kHistGrid ? kHistGrid : blocks);
    if (al)
      hipLaunchKernelGGL((k_hist_lds<T, V>), dim3((unsigned)blocks), dim3(kHistBlock), 0, s, v, n, h, counts);
    else
      hipLaunchKernelGGL((k_hist_lds<T, 1>), dim3((unsigned)blocks), dim3(kHistBlock), 0, s, v, n, h, counts);
  } else {
    int64_t blocks = (n + kHistBlock - 1) / kHistBlock;
    blocks = blocks < 1 ? 1 : (blocks > 65536 ? 65536 : blocks);
    hipLaunchKernelGGL((k_hist_global<T>), dim3((unsigned)blocks), dim3(kHistBlock), 0, s, v, n, h, counts);
  }
  return hipGetLastError();
}

// One lane per event: its pairs in rank order, the smallest |m - target| in
// binary64, the first rank among equal distances; NaN is never chosen.
template <typename T>
__global__ __launch_bounds__(kBestBlock) void k_best_pair(int64_t ne, const int64_t* __restrict__ po,
                                                          const T* __restrict__ pm, double target,
                                                          int64_t* __restrict__ rank, T* __restrict__ best_m) {
  const int64_t e = (int64_t)blockIdx.x * kBestBlock + threadIdx.x;
  if (e >= ne) return;
  const int64_t lo = po[e], hi = po[e + 1];
  int64_t r = -1;
  double best = 0.0;
  T bm = (T)__builtin_nan("");
  for (int64_t k = lo; k < hi; ++k) {
    const T m = pm[k];
    const double d = fabs((double)m - target);
    if (d != d) continue;
    if (r < 0 || d < best) {
      r = k - lo;
      best = d;
      bm = m;
    }
  }
  rank[e] = r;
  best_m[e] = bm;
}

}  // namespace

hipError_t launch_histogram(glv_dtype dt, int64_t n, const void* m, double lo, double hi, int64_t n_bins,
                            unsigned long long* counts, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (dt == GLV_F64) return hist_typed<double>(n, m, lo, hi, n_bins, counts, s);
  return hist_typed<float>(n, m, lo, hi, n_bins, counts, s);
}

hipError_t launch_best_pair(glv_dtype dt, int64_t n_events, const int64_t* pair_offsets, const void* pair_m,
                            double target, int64_t* rank, void* best_m, hipStream_t s) {
  if (n_events <= 0) return hipSuccess;
  const int64_t blocks = (n_events + kBestBlock - 1) / kBestBlock;
  if (dt == GLV_F64)
    hipLaunchKernelGGL((k_best_pair<double>), dim3((unsigned)blocks), dim3(kBestBlock), 0, s, n_events, pair_offsets,
                       (const double*)pair_m, target, rank, (double*)best_m);
  else
    hipLaunchKernelGGL((k_best_pair<float>), dim3((unsigned)blocks), dim3(kBestBlock), 0, s, n_events, pair_offsets,
                       (const float*)pair_m, target, rank, (float*)best_m);
  return hipGetLastError();
}

}  // namespace glv
