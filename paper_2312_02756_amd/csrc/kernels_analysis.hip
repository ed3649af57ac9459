// The analysis step after the mass (not in the paper; Sec. 6 places
// GenVector inside ROOT, which analyses such data): a histogram of masses,
// and per CSR event the pair whose mass lies closest to a target.
#include "glv_device.h"
#include "glv_launch.h"

namespace glv {
namespace {

constexpr int kHistBlock = 1024;
// Workgroups of the LDS path (one per CU, 16 wavefronts each): each merges
// its counters into the global ones once, so fewer, larger workgroups mean
// fewer global atomics on each bin.
constexpr int64_t kHistGrid = 256;
constexpr int kHistUnroll = 4;   // value packs in flight per thread
// Best pair: four lanes per event with eight pair loads in flight each (a
// wavefront covers 16 events and reads an average event in one step): 79 ->
// 70 us on 2^20 Poisson(8) events against eight lanes with four loads.
constexpr int kBestLanes = 4;    // lanes per event in the best-pair kernel
constexpr int kBestBlock = 256;  // 64 events per workgroup
constexpr int kBestUnroll = 8;   // pair loads in flight per lane

// Counts one value: the in-range bins by LDS atomics, the under- and
// overflow in the lane's registers.  Values outside [lo, hi) all land on two
// slots, whose atomics serialise within an instruction; where they are
// common (41 % overflow in the 2^26-pair stress masses over [0, 200) GeV)
// they dominated the kernel.
__device__ __forceinline__ void hist_count(double x, const HistSpec& h, unsigned* bins, unsigned* n_lo,
                                           unsigned* n_hi) {
  const int64_t s = hist_slot(x, h);
  if (s == 0)
    ++*n_lo;
  else if (s == h.nb + 1)
    ++*n_hi;
  else if (s > 0)
    atomicAdd(&bins[s], 1u);
}

// Per-workgroup counters in LDS, merged with one global atomic per non-empty
// slot.  Grid-stride over packs of V values (16-byte loads, kHistUnroll in
// flight per thread before their counts), then the rest and the tail.
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
  unsigned n_lo = 0, n_hi = 0;
  int64_t i = tid;
  for (; i + (kHistUnroll - 1) * stride < nv; i += kHistUnroll * stride) {
    Pack<T, V> p[kHistUnroll];
#pragma unroll
    for (int u = 0; u < kHistUnroll; ++u) p[u] = load_pack<T, V>(v, i + u * stride);
#pragma unroll
    for (int u = 0; u < kHistUnroll; ++u)
#pragma unroll
      for (int e = 0; e < V; ++e) hist_count((double)p[u].v[e], h, bins, &n_lo, &n_hi);
  }
  for (; i < nv; i += stride) {
    const Pack<T, V> p = load_pack<T, V>(v, i);
#pragma unroll
    for (int e = 0; e < V; ++e) hist_count((double)p.v[e], h, bins, &n_lo, &n_hi);
  }
  if constexpr (V > 1) {
    const int64_t t = nv * V + tid;
    if (t < n) hist_count((double)v[t], h, bins, &n_lo, &n_hi);
  }
  if (n_lo) atomicAdd(&bins[0], n_lo);
  if (n_hi) atomicAdd(&bins[nslot - 1], n_hi);
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

// kBestLanes lanes per event: each lane walks every kBestLanes-th pair of
// its event (a lane group reads consecutive pairs together) keeping the
// smallest (distance, rank); a butterfly over the group then takes the
// lexicographic minimum, so the lowest rank wins among equal distances; the
// mass travels with it, so no dependent read follows.
// The distance's bits order as unsigned integers (it is not negative);
// ~0 marks "none" (above every distance, +inf included), and NaN distances
// never enter.
template <typename T>
__global__ __launch_bounds__(kBestBlock) void k_best_pair(int64_t ne, const int64_t* __restrict__ po,
                                                          const T* __restrict__ pm, double target,
                                                          int64_t* __restrict__ rank, T* __restrict__ best_m) {
  const int64_t e = ((int64_t)blockIdx.x * kBestBlock + threadIdx.x) / kBestLanes;
  const int sub = threadIdx.x % kBestLanes;
  const bool live = e < ne;  // lanes past the last event still join the butterfly
  int64_t lo = 0, hi = 0;
  if (live) {
    lo = po[e];
    hi = po[e + 1];
  }
  unsigned long long bd = ~0ull;
  int64_t br = 0;
  T bm = T(0);
  // kBestUnroll loads in flight per lane before their comparisons; positions
  // past the event read as NaN and drop out like NaN masses
  for (int64_t k = lo + sub; k < hi; k += kBestUnroll * kBestLanes) {
    T m[kBestUnroll];
#pragma unroll
    for (int u = 0; u < kBestUnroll; ++u) {
      const int64_t kk = k + u * kBestLanes;
      m[u] = kk < hi ? pm[kk] : (T)__builtin_nan("");
    }
#pragma unroll
    for (int u = 0; u < kBestUnroll; ++u) {
      const double d = fabs((double)m[u] - target);
      const unsigned long long b = (unsigned long long)__double_as_longlong(d);
      if (d == d && b < bd) {  // a lane's ranks only grow, so a tie keeps its earlier rank
        bd = b;
        br = k + u * kBestLanes - lo;
        bm = m[u];
      }
    }
  }
#pragma unroll
  for (int off = kBestLanes / 2; off > 0; off >>= 1) {
    const unsigned long long od = __shfl_xor(bd, off, kBestLanes);
    const int64_t orr = __shfl_xor(br, off, kBestLanes);
    const T om = __shfl_xor(bm, off, kBestLanes);
    if (od < bd || (od == bd && orr < br)) {
      bd = od;
      br = orr;
      bm = om;
    }
  }
  if (live && sub == 0) {
    const bool found = bd != ~0ull;
    rank[e] = found ? br : -1;
    best_m[e] = found ? bm : (T)__builtin_nan("");
  }
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
  constexpr int64_t kEventsPerBlock = kBestBlock / kBestLanes;
  const int64_t blocks = (n_events + kEventsPerBlock - 1) / kEventsPerBlock;
  if (dt == GLV_F64)
    hipLaunchKernelGGL((k_best_pair<double>), dim3((unsigned)blocks), dim3(kBestBlock), 0, s, n_events, pair_offsets,
                       (const double*)pair_m, target, rank, (double*)best_m);
  else
    hipLaunchKernelGGL((k_best_pair<float>), dim3((unsigned)blocks), dim3(kBestBlock), 0, s, n_events, pair_offsets,
                       (const float*)pair_m, target, rank, (float*)best_m);
  return hipGetLastError();
}

}  // namespace glv
