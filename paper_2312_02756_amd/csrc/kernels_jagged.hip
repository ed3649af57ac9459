// Jagged (CSR) event kernels for gfx950: pair-offset scan, offset checks,
// and the one-launch per-event reduction -- each event's total 4-vector,
// its mass and the masses of all its particle pairs (the pair mass of
// GenVectorX Fig. 1 applied to every i < j inside an event) -- with its
// reverse mode.
//
// Work decomposition of the reduction.  A workgroup takes a tile of
// consecutive events.  Their particles are contiguous in the columns, so the
// workgroup streams them once (coalesced), converts each particle once and
// stages the results in LDS in event-aligned chunks of at most
// `lds_particles` particles.  Then
//   * one lane per event sums its particles in CSR order (totals, and the
//     event mass of the plain mode);
//   * the chunk's pairs -- contiguous in the output too -- are split into
//     equal contiguous slices, one per wavefront; lanes take consecutive pair
//     indices (two per lane and iteration: k and k + 64 in the plain mode,
//     k and k + 1 in the compensated mode), locate their event (binary
//     search once, then stepping forward over the staged per-event records),
//     turn the in-event rank into (i, j) through a table of co-lexicographic
//     pairs and store the pair mass (a wavefront's stores cover consecutive
//     addresses);
//   * in the compensated mode the event mass is
//     m^2 = sum_i M_i^2 + 2 sum_{i<j} K_ij (all terms >= 0); each wavefront
//     folds its lanes' K_ij by a segmented lane-move (DPP) scan keyed by
//     event and adds the segment sums to a per-(wavefront, event) LDS slot,
//     and the event lane adds the slots in wavefront order: the result
//     depends on the tiling only, never on timing.
// An event with more particles than fit in LDS is left to a second, small
// launch (k_event_reduce_big), where a whole workgroup takes it straight from
// global memory (correct for any size, slower); on collider-sized events that
// launch only reads the offsets.
#include "glv_device.h"
#include "glv_launch.h"

namespace glv {
namespace {

__device__ __forceinline__ int64_t npairs(int64_t c) { return c * (c - 1) / 2; }

// ------------------------------------------------------------ pair offsets

// Multi-workgroup exclusive scan of n_e (n_e - 1)/2 in three launches, with
// pair_offsets itself holding the per-tile totals between them (no scratch):
//   1. workgroup b sums the pair counts of its kScanTile events and writes the
//      total to pair_offsets[end_b], end_b = min((b + 1) kScanTile, ne);
//   2. one workgroup turns those totals into running totals in place and sets
//      pair_offsets[0] = 0;
//   3. workgroup b scans its own events from pair_offsets[b kScanTile] and
//      writes pair_offsets[e + 1] for its events except the last one, whose
//      value step 2 left in place -- so no entry one workgroup reads is
//      written by another.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanThreads * kScanPer;

// Exclusive prefix over the workgroup of one int64 per thread; *total gets
// the workgroup's sum.  ws holds one int64 per wavefront.
__device__ __forceinline__ int64_t block_excl_scan(int64_t x, int64_t* ws, int64_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int64_t v = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t y = __shfl_up(v, d);
    if (lane >= d) v += y;
  }
  if (lane == 63) ws[wid] = v;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int w = 0; w < nw; ++w) {
    if (w < wid) before += ws[w];
    all += ws[w];
  }
  __syncthreads();
  *total = all;
  return before + v - x;
}

__global__ __launch_bounds__(kScanThreads) void k_po_tile_totals(const int64_t* __restrict__ off,
                                                                 int64_t* __restrict__ po, int64_t ne) {
  __shared__ int64_t ws[kScanThreads / 64];
  const int64_t b0 = (int64_t)blockIdx.x * kScanTile;
  int64_t sum = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const int64_t e = b0 + j * kScanThreads + threadIdx.x;
    if (e < ne) sum += npairs(off[e + 1] - off[e]);
  }
  int64_t total;
  block_excl_scan(sum, ws, &total);
  if (threadIdx.x == 0) po[min(b0 + kScanTile, ne)] = total;
}

__global__ __launch_bounds__(1024) void k_po_scan_totals(int64_t* __restrict__ po, int64_t ne, int64_t ntiles) {
  __shared__ int64_t ws[1024 / 64];
  if (threadIdx.x == 0) po[0] = 0;
  int64_t carry = 0;
  for (int64_t base = 0; base < ntiles; base += 1024) {
    const int64_t b = base + threadIdx.x;
    const int64_t at = min((b + 1) * kScanTile, ne);
    const int64_t v = (b < ntiles) ? po[at] : 0;
    int64_t total;
    const int64_t ex = block_excl_scan(v, ws, &total);
    if (b < ntiles) po[at] = carry + ex + v;
    carry += total;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_po_tile_scan(const int64_t* __restrict__ off,
                                                               int64_t* __restrict__ po, int64_t ne) {
  __shared__ int64_t c[kScanTile];
  __shared__ int64_t ws[kScanThreads / 64];
  const int64_t b0 = (int64_t)blockIdx.x * kScanTile;
  const int64_t end = min(b0 + kScanTile, ne);
  const int64_t base = (blockIdx.x == 0) ? 0 : po[b0];
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const int idx = j * kScanThreads + threadIdx.x;
    const int64_t e = b0 + idx;
    c[idx] = (e < ne) ? npairs(off[e + 1] - off[e]) : 0;
  }
  __syncthreads();
  int64_t run = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) run += c[threadIdx.x * kScanPer + k];
  int64_t total;
  int64_t pre = base + block_excl_scan(run, ws, &total);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    pre += c[threadIdx.x * kScanPer + k];
    c[threadIdx.x * kScanPer + k] = pre;  // inclusive: pair_offsets[e + 1]
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const int idx = j * kScanThreads + threadIdx.x;
    const int64_t e = b0 + idx;
    if (e + 1 < end) po[e + 1] = c[idx];
  }
}

__global__ __launch_bounds__(256) void k_validate_offsets(const int64_t* __restrict__ off, int64_t ne,
                                                          int64_t np, long long* bad) {
  long long cnt = 0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e <= ne; e += stride) {
    int64_t v = off[e];
    if (e == 0 && v != 0) ++cnt;
    if (e == ne && v != np) ++cnt;
    if (e < ne && off[e + 1] < v) ++cnt;
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) cnt += __shfl_xor(cnt, d);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd((unsigned long long*)bad, (unsigned long long)cnt);
}

// --------------------------------------------------------------- helpers

// i of the pair with in-event rank r among n particles (lexicographic i < j):
// the largest i with R(i) = i (2n - i - 1)/2 <= r.
__device__ __forceinline__ int64_t row_start(int64_t i, int64_t n) { return i * (2 * n - i - 1) / 2; }

__device__ __forceinline__ void decode_pair(int64_t r, int64_t n, int64_t* pi, int64_t* pj) {
  double b = (double)(2 * n - 1);
  int64_t i = (int64_t)((b - sqrt(b * b - 8.0 * (double)r)) * 0.5);
  if (i < 0) i = 0;
  if (i > n - 2) i = n - 2;
  while (i > 0 && row_start(i, n) > r) --i;
  while (i < n - 2 && row_start(i + 1, n) <= r) ++i;
  *pi = i;
  *pj = i + 1 + (r - row_start(i, n));
}

// Decode for events staged in LDS (2 <= n <= 4096).  With b = 2n - 1 the
// row is the floor of the root x = (b - sqrt(b^2 - 8r))/2 of R(x) = r.  In
// FP32 b^2 - 8r (< 2^27, one rounding by the fused multiply-add) is off by at
// most 4 and is at least 9, so the hardware square root (1 ulp) puts the
// estimate within one row of the answer: one step down and one step up fix it.
// Products stay below 2^25, so 24-bit multiplies are exact.
__device__ __forceinline__ int row_start32(int i, int n) { return (int)(__umul24(i, 2 * n - i - 1) >> 1); }

__device__ __forceinline__ void decode_pair_small(int r, int n, int* pi, int* pj) {
  const float b = (float)(2 * n - 1);
  const float d = fmaf(b, b, -8.0f * (float)r);
  int i = (int)((b - __builtin_amdgcn_sqrtf(fmaxf(d, 0.0f))) * 0.5f);
  i = max(0, min(i, n - 2));
  if (row_start32(i, n) > r) --i;
  if (i < n - 2 && row_start32(i + 1, n) <= r) ++i;
  *pi = i;
  *pj = i + 1 + (r - row_start32(i, n));
}

// Pair of lexicographic rank r among n particles, through the mirrored pair
// (n-1-j, n-1-i): the mirror reverses the order, so its rank in
// co-lexicographic order (by the larger index, then the smaller) is
// P - 1 - r with P = n(n-1)/2, and co-lexicographic ranks do not depend on
// n.  One table of the kColexN(kColexN-1)/2 co-lexicographic pairs, built once
// per workgroup in LDS, therefore serves every event of at most kColexN
// particles; larger events take the square-root decode.
constexpr int kColexN = 32;
constexpr int kColexPairs = kColexN * (kColexN - 1) / 2;

// Entry r of the table: the pair (a, b), a < b, with b(b-1)/2 + a = r, as
// a | b << 8.
__device__ __forceinline__ unsigned short colex_entry(int r) {
  int b = (int)((1.0f + __builtin_amdgcn_sqrtf(1.0f + 8.0f * (float)r)) * 0.5f);
  while (b * (b - 1) / 2 > r) --b;
  while ((b + 1) * b / 2 <= r) ++b;
  return (unsigned short)((r - b * (b - 1) / 2) | (b << 8));
}

__device__ __forceinline__ void pair_of_rank(int r, int n, const unsigned short* colex, int* pi, int* pj) {
  if (n <= kColexN) {
    const unsigned t = colex[(int)(__umul24(n, n - 1) >> 1) - 1 - r];
    *pi = n - 1 - (int)(t >> 8);
    *pj = n - 1 - (int)(t & 0xffu);
  } else {
    decode_pair_small(r, n, pi, pj);
  }
}

// Per event of a chunk: first particle and first pair, relative to the chunk.
struct EvRec {
  int o;
  int p;
};

// Last event e in [lo, hi) with rec[e].p <= key (p non-decreasing).
__device__ __forceinline__ int search_rec(const EvRec* rec, int lo, int hi, int key) {
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (rec[mid].p <= key)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int search_le(const int64_t* a, int lo, int hi, int64_t key) {
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (a[mid] <= key)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Per-particle staged records in LDS, read with 16-byte LDS loads:
//   cart[t] = (px, py, pz, E)                       every mode
//   legA[t] = (pt, eta, phi, M), legB[t] = (mT, delta)   compensated mode
template <typename T>
struct V4 {
  typedef T type __attribute__((ext_vector_type(4)));
};
template <typename T>
struct V2 {
  typedef T type __attribute__((ext_vector_type(2)));
};

template <typename T, int MODE>
struct Stage {
  typename V4<T>::type* cart;
  typename V4<T>::type* legA;
  typename V2<T>::type* legB;
};

template <typename T, int COORDS, int MODE>
__device__ __forceinline__ void stage_particle(const Cols4<T>& p, int64_t gi, const Stage<T, MODE>& s,
                                               int slot) {
  T c0 = p.c[0][gi], c1 = p.c[1][gi], c2 = p.c[2][gi], c3 = p.c[3][gi];
  if constexpr (MODE == GLV_COMPENSATED) {  // (pt, eta, phi, M)
    T v[4];
    const LegC<T> L = comp_leg_cart<T>(c0, c1, c2, c3, v);
    s.cart[slot] = typename V4<T>::type{v[0], v[1], v[2], v[3]};
    s.legA[slot] = typename V4<T>::type{c0, c1, c2, c3};
    s.legB[slot] = typename V2<T>::type{L.mt, L.delta};
  } else {
    T v[4];
    to_cart<COORDS>(c0, c1, c2, c3, v);
    s.cart[slot] = typename V4<T>::type{v[0], v[1], v[2], v[3]};
  }
}

// acc += rec[lo] + rec[lo+1] + ... + rec[hi-1], component-wise and in index
// order (each component's additions stay sequential), two records read per
// LDS wait (four would cost the kernel its sixth wavefront per SIMD).
template <typename A, typename V>
__device__ __forceinline__ void sum_records(const V* rec, int lo, int hi, A acc[4]) {
  int t = lo;
  for (; t + 2 <= hi; t += 2) {
    const V r0 = rec[t], r1 = rec[t + 1];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += (A)r0[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += (A)r1[k];
  }
  for (; t < hi; ++t) {
    const V r = rec[t];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += (A)r[k];
  }
}

// Compensated leg terms of a staged particle; *mass receives M.
template <typename T, int MODE>
__device__ __forceinline__ LegC<T> staged_leg(const Stage<T, MODE>& s, int slot, T* mass) {
  const typename V4<T>::type a = s.legA[slot];
  const typename V2<T>::type b = s.legB[slot];
  LegC<T> L;
  L.pt = a[0];
  L.eta = a[1];
  L.phi = a[2];
  *mass = a[3];
  L.m2 = a[3] * a[3];
  L.mt = b[0];
  L.delta = b[1];
  return L;
}

// Compensated pair mass and K = E_i E_j - p_i.p_j (as double) from two legs,
// with the FP64 redo of an FP32 pair whose error bound is too large.
template <typename T>
__device__ __forceinline__ T comp_pair(const LegC<T>& a, const LegC<T>& b, T ma, T mb, double* kout,
                                       unsigned* fb) {
  T k;
  if constexpr (sizeof(T) == 4) {
    bool redo;
    T m2 = comp_pair_m2<T>(a, b, &k, &redo);
    if (redo) {
      LegC<double> da = comp_leg<double, true>(a.pt, a.eta, a.phi, ma);
      LegC<double> db = comp_leg<double, true>(b.pt, b.eta, b.phi, mb);
      double kd;
      double m2d = comp_pair_m2<double, true>(da, db, &kd, nullptr);
      *kout = kd;
      ++*fb;
      return (T)sqrt(m2d);
    }
    *kout = (double)k;
    return sqrt_budgeted(m2);
  } else {
    T m2 = comp_pair_m2<T>(a, b, &k, nullptr);
    *kout = (double)k;
    return d_sqrt(m2);
  }
}

// FP32 compensated pair with the redo left to k_event_reduce_big: *redo is
// set when the error bound asks for FP64.
__device__ __forceinline__ float comp_pair_fp32(const LegC<float>& a, const LegC<float>& b, double* kout,
                                                bool* redo) {
  float k;
  const float m2 = comp_pair_m2<float>(a, b, &k, redo);
  *kout = (double)k;
  return sqrt_budgeted(m2);
}

// Marks an event of the tiled FP32 compensated reduction that holds a pair
// needing the FP64 redo: written to the event's mass (or, without event
// masses, to its first pair mass) for k_event_reduce_big to find.  A quiet NaN
// with a payload that arithmetic does not produce; should an input NaN carry
// it, the event is merely recomputed.
constexpr unsigned kRedoMarkBits = 0x7fd2e6b1u;
__device__ __forceinline__ float redo_mark() { return __builtin_bit_cast(float, kRedoMarkBits); }
__device__ __forceinline__ bool is_redo_mark(float x) { return __builtin_bit_cast(unsigned, x) == kRedoMarkBits; }

// Cross-lane moves within a wavefront (GFX9 DPP controls): shift right by d
// lanes within each row of 16 lanes, lane 15 of each row to the next row,
// lane 31 to rows 2 and 3, and the whole wavefront left or right by one
// lane.  A lane
// whose source does not exist, or whose row is masked off, receives `old`.
constexpr int kDppRowShr = 0x110;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;

template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i32(int x, int old) {
  return __builtin_amdgcn_update_dpp(old, x, CTRL, ROWS, 0xf, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double x) {  // old = +0
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)dpp_i32<CTRL, ROWS>((int)(unsigned)b, 0);
  const unsigned hi = (unsigned)dpp_i32<CTRL, ROWS>((int)(unsigned)(b >> 32), 0);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_scan_step(double& x, int key) {
  const double y = dpp_f64<CTRL, ROWS>(x);
  const int ky = dpp_i32<CTRL, ROWS>(key, -1);  // -1: never a key
  x = (ky == key) ? x + y : x;
}

// Inclusive segmented sum over a full wavefront: keys do not decrease with the
// lane, and each lane receives the sum of x over the lanes at or below it with
// its key.  Sums within rows by shifts of 1, 2, 4 and 8, then the running row
// totals carried across rows (lane 15 into rows 1 and 3, lane 31 into rows 2
// and 3); a source with another key adds nothing (keys are monotone, so the
// lanes between agree too).  No LDS traffic; all 64 lanes must be active.
__device__ __forceinline__ double seg_scan_wave(double x, int key) {
  seg_scan_step<kDppRowShr + 1, 0xf>(x, key);
  seg_scan_step<kDppRowShr + 2, 0xf>(x, key);
  seg_scan_step<kDppRowShr + 4, 0xf>(x, key);
  seg_scan_step<kDppRowShr + 8, 0xf>(x, key);
  seg_scan_step<kDppRowBcast15, 0xa>(x, key);
  seg_scan_step<kDppRowBcast31, 0xc>(x, key);
  return x;
}

// Deterministic workgroup sum of one double per thread (fixed tree).
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < nw; ++w) r += red[w];
  __syncthreads();
  return r;
}

template <typename T>
__device__ __forceinline__ void store_out(T* p, int64_t i, T v) {
  __builtin_nontemporal_store(v, p + i);
}

// ---------------------------------------------------------------- forward

struct FwdOut {
  void* total[4];
  void* event_m;
  void* pair_m;
};

template <typename T, int COORDS, int MODE>
struct FwdArgs {
  Cols4<T> p;
  const int64_t* off;
  const int64_t* poff;
  T* total[4];
  T* event_m;
  T* pair_m;
  unsigned long long* fallback;
  int64_t ne;
  int epb;  // events per tile
  int cap;  // particles staged per chunk
};

// One event too large for LDS: the whole workgroup, from global memory.
template <typename T, int COORDS, int MODE>
__device__ void big_event(const FwdArgs<T, COORDS, MODE>& A, int64_t e, int64_t lo, int64_t hi, double* red,
                          unsigned* fb, bool totals = true) {
  const int64_t n = hi - lo;
  double acc[4] = {0, 0, 0, 0};
  double msum = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    if (totals) {
      T v[4];
      to_cart<COORDS>(A.p.c[0][i], A.p.c[1][i], A.p.c[2][i], A.p.c[3][i], v);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] += (double)v[k];
    }
    if constexpr (MODE == GLV_COMPENSATED) msum += (double)A.p.c[3][i] * (double)A.p.c[3][i];
  }
  T tot[4] = {0, 0, 0, 0};
  if (totals) {
#pragma unroll
    for (int k = 0; k < 4; ++k) tot[k] = (T)block_sum(acc[k], red);
  }
  if constexpr (MODE == GLV_COMPENSATED) msum = block_sum(msum, red);
  double ksum = 0.0;
  const bool want_k = (MODE == GLV_COMPENSATED) && A.event_m;
  if (A.pair_m || want_k) {
    const int64_t q = npairs(n);
    const int64_t base = A.poff ? A.poff[e] : 0;
    for (int64_t r = threadIdx.x; r < q; r += blockDim.x) {
      int64_t i, j;
      decode_pair(r, n, &i, &j);
      i += lo;
      j += lo;
      T m;
      if constexpr (MODE == GLV_COMPENSATED) {
        T va[4], vb[4];  // the conversions are not needed here
        LegC<T> a = comp_leg_cart<T>(A.p.c[0][i], A.p.c[1][i], A.p.c[2][i], A.p.c[3][i], va);
        LegC<T> b = comp_leg_cart<T>(A.p.c[0][j], A.p.c[1][j], A.p.c[2][j], A.p.c[3][j], vb);
        double kd;
        m = comp_pair<T>(a, b, A.p.c[3][i], A.p.c[3][j], &kd, fb);
        ksum += kd;
      } else {
        T va[4], vb[4], w[4];
        to_cart<COORDS>(A.p.c[0][i], A.p.c[1][i], A.p.c[2][i], A.p.c[3][i], va);
        to_cart<COORDS>(A.p.c[0][j], A.p.c[1][j], A.p.c[2][j], A.p.c[3][j], vb);
        add4<T>(va, vb, w);
        m = mass_of(w);
      }
      if (A.pair_m) store_out(A.pair_m, base + r, m);
    }
    if (want_k) ksum = block_sum(ksum, red);
  }
  if (threadIdx.x == 0) {
    if (totals && A.total[0]) {
#pragma unroll
      for (int k = 0; k < 4; ++k) A.total[k][e] = tot[k];
    }
    if (A.event_m) {
      if constexpr (MODE == GLV_COMPENSATED)
        A.event_m[e] = (T)sqrt(msum + 2.0 * ksum);
      else
        A.event_m[e] = mass_of(tot);
    }
  }
  __syncthreads();
}

template <typename T, int COORDS, int MODE>
__global__ __launch_bounds__(kMaxBlock) void k_event_reduce(FwdArgs<T, COORDS, MODE> A) {
  extern __shared__ __align__(32) unsigned char lds[];
  const int epb = A.epb, cap = A.cap;
  const int nwaves = blockDim.x >> 6;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // LDS (each record array holds cap records of a size that is a multiple of
  // the next one's alignment, so all stay aligned for any cap):
  //   cart[cap] (4 T), legA[cap] (4 T), legB[cap] (2 T)   staged records
  //   s_off[epb+1], s_poff[epb+1]   int64, the tile's offsets
  //   red[16], acc[nwaves*epb]      double
  //   ch[epb+1]                     EvRec, offsets relative to the chunk
  //   colex[kColexPairs]            uint16, the pair table
  //   s_redo[epb]                   int, FP32 compensated only
  Stage<T, MODE> st;
  st.cart = reinterpret_cast<typename V4<T>::type*>(lds);
  unsigned char* after = lds + (size_t)cap * 4 * sizeof(T);
  if constexpr (MODE == GLV_COMPENSATED) {
    st.legA = reinterpret_cast<typename V4<T>::type*>(after);
    st.legB = reinterpret_cast<typename V2<T>::type*>(after + (size_t)cap * 4 * sizeof(T));
    after += (size_t)cap * 6 * sizeof(T);
  }
  int64_t* s_off = reinterpret_cast<int64_t*>(after);
  int64_t* s_poff = s_off + (epb + 1);
  double* red = reinterpret_cast<double*>(s_poff + (epb + 1));
  double* acc = red + 16;
  EvRec* ch = reinterpret_cast<EvRec*>(acc + ((MODE == GLV_COMPENSATED) ? nwaves * epb : 0));
  unsigned short* colex = reinterpret_cast<unsigned short*>(ch + (epb + 1));
  // FP32 compensated: events of the chunk with a pair needing the FP64 redo
  int* s_redo = reinterpret_cast<int*>(colex + ((kColexPairs + 1) & ~1));
  constexpr bool kDefer = (MODE == GLV_COMPENSATED) && (sizeof(T) == 4);
  // a wave's share of a chunk's pairs is a shift: nwaves is a power of two
  const int lg_waves = __builtin_ctz(nwaves);
  const int wid_s = __builtin_amdgcn_readfirstlane(wid);

  const bool want_pairs = A.pair_m != nullptr;
  const bool want_k = (MODE == GLV_COMPENSATED) && A.event_m != nullptr;
  unsigned fb = 0;
  const int64_t ntiles = (A.ne + epb - 1) / epb;

  if constexpr (MODE == GLV_COMPENSATED) {
    for (int i = threadIdx.x; i < nwaves * epb; i += blockDim.x) acc[i] = 0.0;
  }
  if (want_pairs || want_k) {
    for (int r = threadIdx.x; r < kColexPairs; r += blockDim.x) colex[r] = colex_entry(r);
  }

  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t e0 = tile * epb;
    const int nev = (int)min((int64_t)epb, A.ne - e0);
    for (int i = threadIdx.x; i <= nev; i += blockDim.x) {
      s_off[i] = A.off[e0 + i];
      if (want_pairs || want_k) s_poff[i] = A.poff[e0 + i];
    }
    __syncthreads();
    int ca = 0;
    while (ca < nev) {
      if (s_off[ca + 1] - s_off[ca] > cap) {  // k_event_reduce_big's event
        ++ca;
        continue;
      }
      // largest cb with s_off[cb] - s_off[ca] <= cap (cb > ca)
      const int cb = search_le(s_off, ca + 1, nev + 1, s_off[ca] + cap);
      const int nch = cb - ca;
      const int64_t pbase = s_off[ca];
      const int64_t q0 = (want_pairs || want_k) ? s_poff[ca] : 0;
      const int np = (int)(s_off[cb] - pbase);
      // chunk-relative offsets, so the pair loop works in 32-bit integers
      for (int t = threadIdx.x; t <= nch; t += blockDim.x)
        ch[t] = EvRec{(int)(s_off[ca + t] - pbase), (want_pairs || want_k) ? (int)(s_poff[ca + t] - q0) : 0};
      if constexpr (kDefer) {
        for (int t = threadIdx.x; t < nch; t += blockDim.x) s_redo[t] = 0;
      }
      for (int t = threadIdx.x; t < np; t += blockDim.x) stage_particle<T, COORDS, MODE>(A.p, pbase + t, st, t);
      __syncthreads();

      // one lane per event: totals in CSR order, plain event mass
      double msum = 0.0;
      const int my = (int)threadIdx.x;  // event ca + my of the tile
      if (my < nch) {
        const int lo = ch[my].o, hi = ch[my + 1].o;
        T tot[4];
        if constexpr (MODE == GLV_COMPENSATED) {
          // totals and sum of M^2 in one pass, two particles per LDS wait
          double d[4] = {0, 0, 0, 0};
          int t = lo;
          for (; t + 2 <= hi; t += 2) {
            const typename V4<T>::type r0 = st.cart[t], r1 = st.cart[t + 1];
            const double m0 = (double)st.legA[t][3], m1 = (double)st.legA[t + 1][3];
#pragma unroll
            for (int k = 0; k < 4; ++k) d[k] = (d[k] + (double)r0[k]) + (double)r1[k];
            msum = (msum + m0 * m0) + m1 * m1;
          }
          if (t < hi) {
            const typename V4<T>::type r0 = st.cart[t];
            const double m0 = (double)st.legA[t][3];
#pragma unroll
            for (int k = 0; k < 4; ++k) d[k] += (double)r0[k];
            msum += m0 * m0;
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) tot[k] = (T)d[k];
        } else if constexpr (sizeof(T) == 4) {
          double d[4] = {0, 0, 0, 0};
          sum_records(st.cart, lo, hi, d);
#pragma unroll
          for (int k = 0; k < 4; ++k) tot[k] = (T)d[k];
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) tot[k] = T(0);
          sum_records(st.cart, lo, hi, tot);
        }
        const int64_t e = e0 + ca + my;
        if (A.total[0]) {
#pragma unroll
          for (int k = 0; k < 4; ++k) store_out(A.total[k], e, tot[k]);
        }
        if constexpr (MODE != GLV_COMPENSATED) {
          if (A.event_m) store_out(A.event_m, e, mass_of(tot));
        }
      }

      // pairs: one contiguous slice of the chunk's pairs per wavefront
      if (want_pairs || want_k) {
        const int q = __builtin_amdgcn_readfirstlane(ch[nch].p);  // < 2^22: cap <= 2048
        const int lo = (q * wid_s) >> lg_waves, hi = (q * (wid_s + 1)) >> lg_waves;
        // A lane's pair index grows by 64 per iteration, so its event is found
        // once by binary search and afterwards by stepping forward (a few
        // events at most per iteration on collider-sized events).
        int ev = 0;
        EvRec cur{0, 0}, nxt{0, 0};
        bool located = false;
        if constexpr (MODE != GLV_COMPENSATED) {
          // two pairs per lane and iteration, k and k + 64: their LDS reads and
          // mass evaluations overlap (the second's event is stepped to from the
          // first's)
          for (int it = lo; it < hi; it += 128) {
            const int k0 = it + lane, k1 = k0 + 64;
            if (k0 < hi) {
              if (!located) {
                ev = search_rec(ch, 0, nch, k0);
                cur = ch[ev];
                nxt = ch[ev + 1];
                located = true;
              }
              while (nxt.p <= k0) {
                cur = nxt;
                nxt = ch[++ev + 1];
              }
              int i, j;
              pair_of_rank(k0 - cur.p, nxt.o - cur.o, colex, &i, &j);
              const int si0 = cur.o + i, sj0 = cur.o + j;
              const bool two = k1 < hi;
              int si1 = si0, sj1 = sj0;
              if (two) {
                while (nxt.p <= k1) {
                  cur = nxt;
                  nxt = ch[++ev + 1];
                }
                pair_of_rank(k1 - cur.p, nxt.o - cur.o, colex, &i, &j);
                si1 = cur.o + i;
                sj1 = cur.o + j;
              }
              const typename V4<T>::type a0 = st.cart[si0], b0 = st.cart[sj0];
              const typename V4<T>::type a1 = st.cart[si1], b1 = st.cart[sj1];
              T w0[4], w1[4];
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                w0[c] = a0[c] + b0[c];
                w1[c] = a1[c] + b1[c];
              }
              const T m0 = mass_of(w0), m1 = mass_of(w1);
              store_out(A.pair_m, q0 + k0, m0);
              if (two) store_out(A.pair_m, q0 + k1, m1);
            }
          }
        } else {
          // compensated: two consecutive pairs per lane and iteration,
          // k0 = it + 2 lane and k1 = k0 + 1, usually of one event, so that
          // the K scan runs once per 128 pairs.  A lane whose k1 opens another
          // event holds a head (k0, the last pair of its event) and a tail
          // (k1); tails are scanned by event, a head takes the previous
          // lane's scanned tail when that lane's tail has its event.
          auto pair_at = [&](int si, int sj, int e, double* kd) -> T {
            T ma, mb;
            const LegC<T> la = staged_leg<T, MODE>(st, si, &ma), lb = staged_leg<T, MODE>(st, sj, &mb);
            if constexpr (kDefer) {
              bool redo;
              const T m = comp_pair_fp32(la, lb, kd, &redo);
              if (redo) s_redo[e] = 1;
              return m;
            } else {
              return comp_pair<T>(la, lb, ma, mb, kd, &fb);
            }
          };
          // a lane's two masses go out as one store: the slots start where the
          // global pair index q0 + k is even (lane 0 of the first iteration
          // may then hold only the slice's first pair)
          const int sh = (int)((q0 + lo) & 1);
          for (int it = lo - sh; it < hi; it += 128) {
            int k0 = it + 2 * lane;
            bool v0 = k0 >= lo && k0 < hi, v1 = k0 + 1 < hi;
            if (!v0 && v1) {
              k0 += 1;
              v0 = true;
              v1 = false;
            }
            const int k1 = k0 + 1;
            double kd0 = 0.0, kd1 = 0.0;
            int ev0 = 0x7fffffff, ev1 = 0x7fffffff;  // past the slice: never an event
            if (v0) {
              if (!located) {
                ev = search_rec(ch, 0, nch, k0);
                cur = ch[ev];
                nxt = ch[ev + 1];
                located = true;
              }
              while (nxt.p <= k0) {
                cur = nxt;
                nxt = ch[++ev + 1];
              }
              int i, j;
              pair_of_rank(k0 - cur.p, nxt.o - cur.o, colex, &i, &j);
              ev0 = ev;
              const T m0 = pair_at(cur.o + i, cur.o + j, ev, &kd0);
              T m1 = T(0);
              if (v1) {
                if (nxt.p <= k1) {  // k0 closed its event: k1 is (0, 1) of the next with pairs
                  do {
                    cur = nxt;
                    nxt = ch[++ev + 1];
                  } while (nxt.p <= k1);
                  i = 0;
                  j = 1;
                } else if (++j == nxt.o - cur.o) {  // lexicographic successor
                  ++i;
                  j = i + 1;
                }
                ev1 = ev;
                m1 = pair_at(cur.o + i, cur.o + j, ev, &kd1);
              }
              if (want_pairs) {
                T* out = A.pair_m + q0 + k0;
                if (v1 && (reinterpret_cast<uintptr_t>(out) & (2 * sizeof(T) - 1)) == 0) {
                  __builtin_nontemporal_store(typename V2<T>::type{m0, m1},
                                              reinterpret_cast<typename V2<T>::type*>(out));
                } else {
                  __builtin_nontemporal_store(m0, out);
                  if (v1) __builtin_nontemporal_store(m1, out + 1);
                }
              }
            }
            if (want_k) {
              const bool split = v1 && ev1 != ev0;
              const int tkey = v1 ? ev1 : ev0;  // keys ascend with the lane
              const double ts = seg_scan_wave(split ? kd1 : kd0 + kd1, tkey);
              const double pts = dpp_f64<kDppWaveShr1, 0xf>(ts);        // lane 0: 0
              const int pkey = dpp_i32<kDppWaveShr1, 0xf>(tkey, -1);     // lane 0: -1
              const int nfirst = dpp_i32<kDppWaveShl1, 0xf>(ev0, -1);    // lane 63: -1
              if (split) acc[wid * epb + ev0] += (pkey == ev0 ? pts : 0.0) + kd0;
              if (v0 && nfirst != tkey) acc[wid * epb + tkey] += ts;
            }
          }
        }
      }
      __syncthreads();
      if constexpr (MODE == GLV_COMPENSATED) {
        if (want_k && my < nch) {
          double ks = 0.0;
          for (int w = 0; w < nwaves; ++w) {
            ks += acc[w * epb + my];
            acc[w * epb + my] = 0.0;
          }
          T em = (T)sqrt(msum + 2.0 * ks);
          if constexpr (kDefer) {
            if (s_redo[my]) em = redo_mark();
          }
          store_out(A.event_m, e0 + ca + my, em);
        }
      }
      if constexpr (kDefer) {  // without event masses the mark goes to the event's first pair mass
        if (!A.event_m && want_pairs && my < nch && s_redo[my]) store_out(A.pair_m, q0 + ch[my].p, redo_mark());
      }
      __syncthreads();
      ca = cb;
    }
  }
  if constexpr (MODE == GLV_COMPENSATED && sizeof(T) == 4) {
    if (A.fallback) {
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) fb += __shfl_xor(fb, d);
      if (lane == 0 && fb) atomicAdd(A.fallback, (unsigned long long)fb);
    }
  }
}

// Events of more than cap particles, which k_event_reduce leaves out: the
// workgroup scans the offsets for them and takes each one whole, from global
// memory.  A separate launch, so that this rare path does not set the main
// kernel's register budget; on collider-sized events it only reads the offsets.
// In the FP32 compensated mode the same scan finds the events k_event_reduce
// marked for the FP64 redo (a mark in the event mass, or in the first pair
// mass without event masses) and recomputes their pair masses and event mass
// with the redo, counting the redone pairs; their totals stay as computed.
constexpr int kBigBlock = 256;

template <typename T, int COORDS, int MODE>
__global__ __launch_bounds__(kBigBlock) void k_event_reduce_big(FwdArgs<T, COORDS, MODE> A) {
  constexpr bool kDefer = (MODE == GLV_COMPENSATED) && (sizeof(T) == 4);
  __shared__ double red[16];
  __shared__ int64_t list[kBigBlock];  // event << 1 | (1: redo only)
  __shared__ int count;
  unsigned fb = 0;
  for (int64_t base = (int64_t)blockIdx.x * kBigBlock; base < A.ne; base += (int64_t)gridDim.x * kBigBlock) {
    const int64_t e = base + threadIdx.x;
    bool big = false, redo = false;
    if (e < A.ne) {
      const int64_t n = A.off[e + 1] - A.off[e];
      big = n > A.cap;
      if constexpr (kDefer) {
        if (!big && n >= 2) {
          if (A.event_m)
            redo = is_redo_mark(A.event_m[e]);
          else if (A.pair_m)
            redo = is_redo_mark(A.pair_m[A.poff[e]]);
        }
      }
    }
    if (!__syncthreads_or(big || redo)) continue;
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
    if (big || redo) list[atomicAdd(&count, 1)] = (e << 1) | (redo ? 1 : 0);
    __syncthreads();
    const int nbig = count;
    for (int b = 0; b < nbig; ++b) {
      const int64_t eb = list[b] >> 1;
      big_event<T, COORDS, MODE>(A, eb, A.off[eb], A.off[eb + 1], red, &fb, (list[b] & 1) == 0);
    }
    __syncthreads();
  }
  if constexpr (MODE == GLV_COMPENSATED && sizeof(T) == 4) {
    if (A.fallback) {
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) fb += __shfl_xor(fb, d);
      if ((threadIdx.x & 63) == 0 && fb) atomicAdd(A.fallback, (unsigned long long)fb);
    }
  }
}

// --------------------------------------------------------------- backward

template <typename T, int COORDS>
struct BwdArgs {
  Cols4<T> p;
  const int64_t* off;
  const int64_t* poff;
  const T* gt[4];
  const T* gem;
  const T* gpair;
  T* gp[4];
  int64_t ne;
  int epb;
  int cap;
};

// Cartesian gradient of particle i from its partners (global memory path).
template <typename T, int COORDS>
__device__ __forceinline__ void partner_sum_global(const BwdArgs<T, COORDS>& A, int64_t lo, int64_t n,
                                                   int64_t pbase, int64_t ai, const T vi[4], T u[4]) {
  for (int64_t bj = 0; bj < n; ++bj) {
    if (bj == ai) continue;
    const int64_t r = ai < bj ? ai : bj, c = ai < bj ? bj : ai;
    const T g = A.gpair[pbase + row_start(r, n) + (c - r - 1)];
    T vj[4], w[4], uw[4];
    const int64_t j = lo + bj;
    to_cart<COORDS>(A.p.c[0][j], A.p.c[1][j], A.p.c[2][j], A.p.c[3][j], vj);
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = vi[k] + vj[k];
    dmass<T>(w, g, uw);
#pragma unroll
    for (int k = 0; k < 4; ++k) u[k] += uw[k];
  }
}

template <typename T, int COORDS>
__device__ void big_event_bwd(const BwdArgs<T, COORDS>& A, int64_t e, int64_t lo, int64_t hi, double* red) {
  const int64_t n = hi - lo;
  // total 4-vector for the event-mass term
  double acc[4] = {0, 0, 0, 0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    T v[4];
    to_cart<COORDS>(A.p.c[0][i], A.p.c[1][i], A.p.c[2][i], A.p.c[3][i], v);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += (double)v[k];
  }
  T tot[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) tot[k] = (T)block_sum(acc[k], red);
  T ut[4] = {0, 0, 0, 0};
  if (A.gem) dmass<T>(tot, A.gem[e], ut);
  if (A.gt[0]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) ut[k] += A.gt[k][e];
  }
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    T c0 = A.p.c[0][i], c3 = A.p.c[3][i];
    LegJ<T> L = to_cart_j<COORDS, T>(c0, A.p.c[1][i], A.p.c[2][i], c3);
    T u[4] = {ut[0], ut[1], ut[2], ut[3]};
    if (A.gpair) partner_sum_global<T, COORDS>(A, lo, n, A.poff[e], i - lo, L.v, u);
    T g[4];
    chain_coords<COORDS, T>(L, c0, c3, u, g);
#pragma unroll
    for (int k = 0; k < 4; ++k) store_out(A.gp[k], i, g[k]);
  }
  __syncthreads();
}

// Pairs staged per chunk of the backward: at most this many per particle of
// the chunk capacity (a chunk also ends where its pairs would exceed it).
constexpr int kBwdPairsPerParticle = 4;

__device__ __forceinline__ int64_t bwd_pair_cap(int cap) { return (int64_t)kBwdPairsPerParticle * cap; }

// An event the tiled backward leaves to k_event_reduce_bwd_big.
__device__ __forceinline__ bool bwd_big(int64_t n, int cap, bool pairs) {
  return n > cap || (pairs && npairs(n) > bwd_pair_cap(cap));
}

// LDS-staged backward.  A chunk holds at most one particle per thread (cap <=
// block; the launch clamps the staging capacity to the workgroup) and, when
// pair gradients are given, kBwdPairsPerParticle * cap pairs:
//   * thread t converts particle t of the chunk once, keeps its Cartesian
//     vector and Jacobian pieces (cos phi, sin phi, sinh eta, cosh eta) in
//     registers and stages the vector in LDS for its partners; the chunk's
//     pair gradients -- contiguous in grad_pair -- are copied to LDS, each
//     thread issuing all of its loads before its stores; one lane per event
//     records its particles' event (from the offsets: all one phase);
//   * pair phase: each pair's gradient g_ij becomes c_ij = g_ij / |m_ij| in
//     place, computed once, by one of its two legs: particle a of an event of
//     n takes the partners a + 1, ..., a + d cyclically, d = (n - 1) / 2
//     rounded down, plus a + n/2 when n is even and a < n/2 -- every pair
//     once, about n/2 per particle, whatever the particle's place;
//   * in the same phase one lane per event (spread over the wavefronts; its
//     g_total and g_m were loaded with the chunk) sums the event's vectors V
//     in CSR order and stages g_total + g_m dm(V)/dV, the upstream every
//     particle of the event receives from the event outputs;
//   * thread t then walks its event's particles in CSR order and adds the
//     pair terms c_ij (v_i + v_j) = c_ij v_i + c_ij v_j of its partners
//     (dm(w)/dw = (-P, E) / |m|, the same 4-vector for both legs of a pair),
//     walking the pair indices incrementally, then the event's upstream, and
//     applies its own conversion Jacobian.
template <typename T, int COORDS>
__global__ __launch_bounds__(kMaxBlock) void k_event_reduce_bwd(BwdArgs<T, COORDS> A) {
  extern __shared__ __align__(32) unsigned char lds[];
  using R4 = typename V4<T>::type;
  // event totals of FP32 data are summed in FP64
  using Acc = typename std::conditional<sizeof(T) == 4, double, T>::type;
  const int epb = A.epb, cap = A.cap;  // cap <= blockDim.x
  const bool pairs = A.gpair != nullptr;
  const bool want_v = A.gem != nullptr;
  const int qcap = pairs ? (int)bwd_pair_cap(cap) : 0;
  const int tid = (int)threadIdx.x;
  const bool want_u = want_v || A.gt[0] != nullptr;
  // LDS: cart[cap], s_ut[epb] (R4), s_g[qcap + 2] (T; qcap is even, one
  //      slot of slack), s_gm[epb rounded up to even] (T), s_off[epb+1],
  //      s_poff[epb+1] (int64), ch[epb+1] (EvRec), ev_of[cap] (uint16)
  R4* cart = reinterpret_cast<R4*>(lds);
  R4* s_ut = cart + cap;
  T* s_g = reinterpret_cast<T*>(s_ut + epb);
  T* s_gm = s_g + qcap + 2;
  int64_t* s_off = reinterpret_cast<int64_t*>(s_gm + ((epb + 1) & ~1));
  int64_t* s_poff = s_off + (epb + 1);
  EvRec* ch = reinterpret_cast<EvRec*>(s_poff + (epb + 1));
  unsigned short* ev_of = reinterpret_cast<unsigned short*>(ch + (epb + 1));
  // event lanes: event t of a chunk belongs to thread (t % nw) * 64 + t / nw,
  // spread over the workgroup's nw wavefronts (the block is a power of two
  // >= 64 and a chunk has at most epb <= block events); tev is the inverse
  const int nw = (int)blockDim.x >> 6;
  const int tev = (tid & 63) * nw + (tid >> 6);
  const int64_t ntiles = (A.ne + epb - 1) / epb;

  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t e0 = tile * epb;
    const int nev = (int)min((int64_t)epb, A.ne - e0);
    for (int i = tid; i <= nev; i += blockDim.x) {
      s_off[i] = A.off[e0 + i];
      if (pairs) s_poff[i] = A.poff[e0 + i];
    }
    __syncthreads();
    int ca = 0;
    while (ca < nev) {
      if (bwd_big(s_off[ca + 1] - s_off[ca], cap, pairs)) {  // k_event_reduce_bwd_big's event
        ++ca;
        continue;
      }
      // largest cb with at most cap particles (and qcap pairs) from ca
      int cb = search_le(s_off, ca + 1, nev + 1, s_off[ca] + cap);
      if (pairs) cb = min(cb, search_le(s_poff, ca + 1, nev + 1, s_poff[ca] + qcap));
      const int nch = cb - ca;
      const int64_t pbase = s_off[ca];
      const int64_t q0 = pairs ? s_poff[ca] : 0;
      const int np = (int)(s_off[cb] - pbase);
      const int nq = pairs ? (int)(s_poff[cb] - q0) : 0;
      const bool mine = tid < np;
      const int64_t gi = pbase + tid;
      // loads first: own particle, up to kBwdPairsPerParticle pair gradients
      T c[4] = {0, 0, 0, 0};
      if (mine) {
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] = A.p.c[k][gi];
      }
      T gv[kBwdPairsPerParticle];
#pragma unroll
      for (int r = 0; r < kBwdPairsPerParticle; ++r) {
        const int idx = tid + r * (int)blockDim.x;
        gv[r] = (idx < nq) ? A.gpair[q0 + idx] : T(0);
      }
      // the event lane's upstreams (g_total, g_m), staged with the rest
      const bool evl = want_u && tev < nch;
      T gtv[4] = {0, 0, 0, 0}, gmv = 0;
      if (evl) {
        const int64_t e = e0 + ca + tev;
        if (A.gt[0]) {
#pragma unroll
          for (int k = 0; k < 4; ++k) gtv[k] = A.gt[k][e];
        }
        if (want_v) gmv = A.gem[e];
      }
      for (int t = tid; t <= nch; t += blockDim.x)
        ch[t] = EvRec{(int)(s_off[ca + t] - pbase), pairs ? (int)(s_poff[ca + t] - q0) : 0};
      for (int t = tid; t < nch; t += blockDim.x) {
        const int lo = (int)(s_off[ca + t] - pbase), hi = (int)(s_off[ca + t + 1] - pbase);
        for (int i = lo; i < hi; ++i) ev_of[i] = (unsigned short)t;
      }
#pragma unroll
      for (int r = 0; r < kBwdPairsPerParticle; ++r) {
        const int idx = tid + r * (int)blockDim.x;
        if (idx < nq) s_g[idx] = gv[r];
      }
      if (evl) {
        s_ut[tev] = R4{gtv[0], gtv[1], gtv[2], gtv[3]};
        s_gm[tev] = gmv;
      }
      LegJ<T> L = to_cart_j<COORDS, T, true>(c[0], c[1], c[2], c[3]);
      if (mine) cart[tid] = R4{L.v[0], L.v[1], L.v[2], L.v[3]};
      __syncthreads();

      // one lane per event: the upstream every particle's 4-vector receives
      // from the event outputs, g_total + g_m dm(V)/dV, with V summed in CSR
      // order
      if (evl && want_v) {
        const int lo = ch[tev].o, hi = ch[tev + 1].o;
        Acc vt[4] = {0, 0, 0, 0};
        int i = lo;
        for (; i + 1 < hi; i += 2) {  // both reads first
          const R4 v0 = cart[i], v1 = cart[i + 1];
#pragma unroll
          for (int k = 0; k < 4; ++k) vt[k] = (vt[k] + (Acc)v0[k]) + (Acc)v1[k];
        }
        if (i < hi) {
          const R4 v0 = cart[i];
#pragma unroll
          for (int k = 0; k < 4; ++k) vt[k] += (Acc)v0[k];
        }
        T tot[4], ud[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) tot[k] = (T)vt[k];
        dmass<T>(tot, s_gm[tev], ud);
        const R4 gt4 = s_ut[tev];
        s_ut[tev] = R4{ud[0] + gt4[0], ud[1] + gt4[1], ud[2] + gt4[2], ud[3] + gt4[3]};
      }

      // Pair ranks inside an event: pair (b, a), b < a, sits at
      // R(b) + a - b - 1, which grows by n - b - 2 with b; pair (a, b), b > a,
      // at R(a) + b - a - 1, consecutive from R(a) = a (2n - a - 1) / 2.
      int ev = 0, n = 0, ai = 0;
      EvRec rc{0, 0};
      if (mine) {
        ev = ev_of[tid];
        rc = ch[ev];
        n = ch[ev + 1].o - rc.o;
        ai = tid - rc.o;
      }
      const int qrow = rc.p + (int)(__umul24(ai, 2 * n - ai - 1) >> 1);
      if (pairs) {
        if (mine) {
          const int cnt = ((n - 1) >> 1) + ((n & 1) == 0 && 2 * ai < n ? 1 : 0);
          int qlo = rc.p + ai - 1, qhi = qrow;
          for (int t = 0, b = ai + 1; t < cnt; ++t, ++b) {
            const bool wrap = b >= n;
            const int bb = wrap ? b - n : b;
            const int q = wrap ? qlo : qhi;
            const T g = s_g[q];
            const R4 vj = cart[rc.o + bb];
            T w[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) w[k] = L.v[k] + vj[k];
            s_g[q] = pair_coef<T>(w, g);
            if (wrap)
              qlo += n - bb - 2;
            else
              ++qhi;
          }
        }
      }
      if (pairs || want_u) __syncthreads();  // s_g and s_ut complete

      if (mine) {
        T u[4] = {0, 0, 0, 0};
        if (want_u) {
          const R4 ut = s_ut[ev];
#pragma unroll
          for (int k = 0; k < 4; ++k) u[k] = ut[k];
        }
        if (pairs && n > 1) {
          // partners in ascending order: S = sum of c_ab v_b, C = sum of c_ab
          T S[4] = {0, 0, 0, 0}, C = 0;
          int qlo = rc.p + ai - 1, qhi = qrow;
          for (int bj = 0; bj < n; ++bj) {
            // branch-free: at bj == ai the slot read (at most nq, the slack
            // slot) is replaced by 0, which adds exact zeros
            const bool below = bj < ai;
            const T cs = s_g[below ? qlo : qhi];
            const R4 vj = cart[rc.o + bj];
            const T cab = (bj == ai) ? T(0) : cs;
#pragma unroll
            for (int k = 0; k < 4; ++k) S[k] += cab * vj[k];
            C += cab;
            qlo += below ? n - bj - 2 : 0;
            qhi += bj > ai ? 1 : 0;
          }
          // sum of c_ab (v_a + v_b) = C v_a + S, with dm/dw = (-P, E) / |m|
#pragma unroll
          for (int k = 0; k < 3; ++k) u[k] -= C * L.v[k] + S[k];
          u[3] += C * L.v[3] + S[3];
        }
        T g[4];
        chain_coords<COORDS, T>(L, c[0], c[3], u, g);
#pragma unroll
        for (int k = 0; k < 4; ++k) store_out(A.gp[k], gi, g[k]);
      }
      __syncthreads();
      ca = cb;
    }
  }
}

// Backward of the events k_event_reduce_bwd leaves out (more than cap
// particles), as k_event_reduce_big does for the forward.
template <typename T, int COORDS>
__global__ __launch_bounds__(kBigBlock) void k_event_reduce_bwd_big(BwdArgs<T, COORDS> A) {
  __shared__ double red[16];
  __shared__ int64_t list[kBigBlock];
  __shared__ int count;
  for (int64_t base = (int64_t)blockIdx.x * kBigBlock; base < A.ne; base += (int64_t)gridDim.x * kBigBlock) {
    const int64_t e = base + threadIdx.x;
    const bool big = e < A.ne && bwd_big(A.off[e + 1] - A.off[e], A.cap, A.gpair != nullptr);
    if (!__syncthreads_or(big)) continue;
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
    if (big) list[atomicAdd(&count, 1)] = e;
    __syncthreads();
    const int nbig = count;
    for (int b = 0; b < nbig; ++b) {
      const int64_t eb = list[b];
      big_event_bwd<T, COORDS>(A, eb, A.off[eb], A.off[eb + 1], red);
    }
    __syncthreads();
  }
}

int big_grid(int64_t ne) {
  return (int)std::min<int64_t>(std::max<int64_t>(1, (ne + kBigBlock - 1) / kBigBlock), 2048);
}

// The backward stages at most one particle per thread.
int bwd_cap(const Tiling& t) { return std::min(t.lds_particles, t.block); }

int grid_for(int64_t ne, int epb) {
  int64_t tiles = (ne + epb - 1) / epb;
  if (tiles < 1) tiles = 1;
  if (tiles > 0x7fffffff) tiles = 0x7fffffff;
  return (int)tiles;
}

template <typename T, int COORDS, int MODE>
hipError_t fwd_typed(int64_t ne, const int64_t* off, const int64_t* poff, const void* const p[4],
                     void* const total[4], void* em, void* pm, unsigned long long* fb, const Tiling& t,
                     size_t lds, hipStream_t s) {
  FwdArgs<T, COORDS, MODE> A;
  for (int k = 0; k < 4; ++k) {
    A.p.c[k] = (const T*)p[k];
    A.total[k] = total ? (T*)total[k] : nullptr;
  }
  A.off = off;
  A.poff = poff;
  A.event_m = (T*)em;
  A.pair_m = (T*)pm;
  A.fallback = fb;
  A.ne = ne;
  A.epb = t.events_per_tile;
  A.cap = t.lds_particles;
  hipLaunchKernelGGL((k_event_reduce<T, COORDS, MODE>), dim3(grid_for(ne, t.events_per_tile)), dim3(t.block),
                     lds, s, A);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((k_event_reduce_big<T, COORDS, MODE>), dim3(big_grid(ne)), dim3(kBigBlock), 0, s, A);
  return hipGetLastError();
}

template <typename T, int COORDS>
hipError_t bwd_typed(int64_t ne, const int64_t* off, const int64_t* poff, const void* const p[4],
                     const void* const gt[4], const void* gem, const void* gpair, void* const gp[4],
                     const Tiling& t, size_t lds, hipStream_t s) {
  BwdArgs<T, COORDS> A;
  for (int k = 0; k < 4; ++k) {
    A.p.c[k] = (const T*)p[k];
    A.gt[k] = gt ? (const T*)gt[k] : nullptr;
    A.gp[k] = (T*)gp[k];
  }
  A.off = off;
  A.poff = poff;
  A.gem = (const T*)gem;
  A.gpair = (const T*)gpair;
  A.ne = ne;
  A.epb = t.events_per_tile;
  A.cap = bwd_cap(t);
  hipLaunchKernelGGL((k_event_reduce_bwd<T, COORDS>), dim3(grid_for(ne, t.events_per_tile)), dim3(t.block), lds,
                     s, A);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((k_event_reduce_bwd_big<T, COORDS>), dim3(big_grid(ne)), dim3(kBigBlock), 0, s, A);
  return hipGetLastError();
}

template <typename T>
hipError_t fwd_dt(glv_coords co, glv_mode mode, int64_t ne, const int64_t* off, const int64_t* poff,
                  const void* const p[4], void* const total[4], void* em, void* pm, unsigned long long* fb,
                  const Tiling& t, size_t lds, hipStream_t s) {
  if (mode == GLV_COMPENSATED)
    return fwd_typed<T, GLV_PTETAPHIM, GLV_COMPENSATED>(ne, off, poff, p, total, em, pm, fb, t, lds, s);
  switch (co) {
    case GLV_PXPYPZE:
      return fwd_typed<T, GLV_PXPYPZE, GLV_PLAIN>(ne, off, poff, p, total, em, pm, nullptr, t, lds, s);
    case GLV_PTETAPHIM:
      return fwd_typed<T, GLV_PTETAPHIM, GLV_PLAIN>(ne, off, poff, p, total, em, pm, nullptr, t, lds, s);
    case GLV_PXPYPZM:
      return fwd_typed<T, GLV_PXPYPZM, GLV_PLAIN>(ne, off, poff, p, total, em, pm, nullptr, t, lds, s);
    default:
      return fwd_typed<T, GLV_PTETAPHIE, GLV_PLAIN>(ne, off, poff, p, total, em, pm, nullptr, t, lds, s);
  }
}

template <typename T>
hipError_t bwd_dt(glv_coords co, int64_t ne, const int64_t* off, const int64_t* poff, const void* const p[4],
                  const void* const gt[4], const void* gem, const void* gpair, void* const gp[4],
                  const Tiling& t, size_t lds, hipStream_t s) {
  switch (co) {
    case GLV_PXPYPZE:
      return bwd_typed<T, GLV_PXPYPZE>(ne, off, poff, p, gt, gem, gpair, gp, t, lds, s);
    case GLV_PTETAPHIM:
      return bwd_typed<T, GLV_PTETAPHIM>(ne, off, poff, p, gt, gem, gpair, gp, t, lds, s);
    case GLV_PXPYPZM:
      return bwd_typed<T, GLV_PXPYPZM>(ne, off, poff, p, gt, gem, gpair, gp, t, lds, s);
    default:
      return bwd_typed<T, GLV_PTETAPHIE>(ne, off, poff, p, gt, gem, gpair, gp, t, lds, s);
  }
}

}  // namespace

size_t event_reduce_lds_bytes(glv_dtype dt, glv_mode mode, const Tiling& t) {
  size_t tsz = (dt == GLV_F64) ? 8 : 4;
  size_t cols = (mode == GLV_COMPENSATED) ? 10 : 4;
  size_t nwaves = (size_t)t.block / 64;
  size_t acc = (mode == GLV_COMPENSATED) ? nwaves * (size_t)t.events_per_tile * 8 : 0;
  size_t redo = (mode == GLV_COMPENSATED && dt == GLV_F32) ? (size_t)t.events_per_tile * sizeof(int) : 0;
  return 2 * ((size_t)t.events_per_tile + 1) * 8 + 16 * 8 + acc + ((size_t)t.events_per_tile + 1) * sizeof(EvRec) +
         ((kColexPairs + 1) & ~1) * sizeof(unsigned short) + redo + cols * (size_t)t.lds_particles * tsz;
}

size_t event_reduce_bwd_lds_bytes(glv_dtype dt, const Tiling& t) {
  // the pair-gradient area is sized for pair gradients given; it is the
  // bound the launch must satisfy either way
  const size_t tsz = (dt == GLV_F64) ? 8 : 4;
  const size_t cap = (size_t)bwd_cap(t), epb = (size_t)t.events_per_tile;
  const size_t qcap = (size_t)kBwdPairsPerParticle * cap;
  return 4 * (cap + epb) * tsz + (qcap + 2) * tsz + ((epb + 1) & ~(size_t)1) * tsz + 2 * (epb + 1) * 8 +
         (epb + 1) * sizeof(EvRec) + cap * sizeof(unsigned short);
}

hipError_t launch_pair_offsets(int64_t ne, const int64_t* off, int64_t* po, hipStream_t s) {
  const int64_t ntiles = (ne + kScanTile - 1) / kScanTile;
  if (ntiles == 0) {  // no events: pair_offsets = {0}
    hipLaunchKernelGGL(k_po_scan_totals, dim3(1), dim3(1024), 0, s, po, ne, (int64_t)0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_po_tile_totals, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, off, po, ne);
  hipLaunchKernelGGL(k_po_scan_totals, dim3(1), dim3(1024), 0, s, po, ne, ntiles);
  hipLaunchKernelGGL(k_po_tile_scan, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, off, po, ne);
  return hipGetLastError();
}

hipError_t launch_validate_offsets(int64_t ne, const int64_t* off, int64_t np, long long* bad, hipStream_t s) {
  int64_t blocks = (ne + 1 + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_validate_offsets, dim3((unsigned)blocks), dim3(256), 0, s, off, ne, np, bad);
  return hipGetLastError();
}

hipError_t launch_event_reduce(glv_dtype dt, glv_coords co, glv_mode mode, int64_t ne, const int64_t* off,
                               const int64_t* poff, const void* const p[4], void* const total[4], void* em,
                               void* pm, unsigned long long* fb, const Tiling& t, hipStream_t s) {
  size_t lds = event_reduce_lds_bytes(dt, mode, t);
  if (dt == GLV_F64) return fwd_dt<double>(co, mode, ne, off, poff, p, total, em, pm, nullptr, t, lds, s);
  return fwd_dt<float>(co, mode, ne, off, poff, p, total, em, pm, fb, t, lds, s);
}

hipError_t launch_event_reduce_bwd(glv_dtype dt, glv_coords co, int64_t ne, const int64_t* off,
                                   const int64_t* poff, const void* const p[4], const void* const gt[4],
                                   const void* gem, const void* gpair, void* const gp[4], const Tiling& t,
                                   hipStream_t s) {
  size_t lds = event_reduce_bwd_lds_bytes(dt, t);
  if (dt == GLV_F64) return bwd_dt<double>(co, ne, off, poff, p, gt, gem, gpair, gp, t, lds, s);
  return bwd_dt<float>(co, ne, off, poff, p, gt, gem, gpair, gp, t, lds, s);
}

}  // namespace glv
