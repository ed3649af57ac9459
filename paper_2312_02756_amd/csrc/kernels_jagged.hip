// Jagged (CSR) event kernels for gfx950: pair-offset scan, offset checks,
// and the one-launch per-event reduction -- each event's total 4-vector,
// its mass and the masses of all its particle pairs (the pair mass of
// GenVectorX Fig. 1 applied to every i < j inside an event) -- with its
// reverse mode.
//
// Work decomposition of the reduction.  Each wavefront takes its own tile of
// consecutive events and walks it in event-aligned chunks of at most
// `lds_particles` particles, staging each particle once, converted, in its
// own slice of LDS (no workgroup barrier: the wavefronts of a workgroup never
// share data).  Four lanes per event sum its particles, one residue class of
// the particle index modulo 4 each, combined in a fixed order; the
// chunk's pairs -- contiguous in the output too -- are dealt out as equal
// contiguous runs, one per lane, each lane stepping its run in lexicographic
// order across event boundaries, so every lane has the same work whatever the
// event sizes.  In the compensated mode each lane also sums K_ij over its run
// per event, and the partial sums of an event that spans runs are combined
// across lanes by a segmented scan keyed by event: deterministic for a
// tiling, never dependent on timing.  The same kernel can choose, per event,
// the pair whose mass lies closest to a target (a candidate per run and
// event, combined by the same scheme under a total order) instead of storing
// pair masses.
// The reverse mode stages one particle per thread of a workgroup (below).
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

// Per event of a chunk: first particle and first pair, relative to the chunk.
struct EvRec {
  int o;
  int p;
};

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
//   leg[2t] = (pt, eta, phi, M), leg[2t+1] = (mT, delta, mT - pt, M^2)
//                                                    compensated mode
template <typename T>
struct V4 {
  typedef T type __attribute__((ext_vector_type(4)));
};

// The total of an event's records rec[lo..hi) is ((P0 + P1) + (P2 + P3)), P_r
// the sum from zero, component-wise and in index order, of the records
// lo + r, lo + r + 4, ...  Forward and reverse mode both give each event a
// quad of lanes, one residue each, and combine the quad's sums in this order
// (lane ^ 1, then lane ^ 2), so that their totals agree bit for bit.
// residue_sum adds P_r to acc (two records read per LDS wait); with a
// non-null `legs` (compensated mode) it also adds the residue's sum of M^2
// (the mass is the fourth component of leg[2t]) to *m2.
template <typename V>
__device__ __forceinline__ void residue_sum(const V* rec, int lo, int hi, int r, double acc[4],
                                            const V* legs = nullptr, double* m2 = nullptr) {
  int t = lo + r;
  for (; t + 4 < hi; t += 8) {
    const V r0 = rec[t], r1 = rec[t + 4];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = (acc[k] + (double)r0[k]) + (double)r1[k];
    if (legs) {
      const double m0 = (double)legs[2 * t][3], m1 = (double)legs[2 * t + 8][3];
      *m2 = (*m2 + m0 * m0) + m1 * m1;
    }
  }
  if (t < hi) {
    const V r0 = rec[t];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += (double)r0[k];
    if (legs) {
      const double m0 = (double)legs[2 * t][3];
      *m2 += m0 * m0;
    }
  }
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
// lane 31 to rows 2 and 3, and the whole wavefront right by one lane.  A lane
// whose source does not exist, or whose row is masked off, receives `old`.
constexpr int kDppRowShr = 0x110;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;
constexpr int kDppWaveShr1 = 0x138;
// Within each quad of lanes: lane ^ 1 and lane ^ 2 (quad_perm [1,0,3,2] and
// [2,3,0,1]).
constexpr int kDppQuadXor1 = 0xb1;
constexpr int kDppQuadXor2 = 0x4e;

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

// A best-pair candidate (distance, in-event rank (-1: none), mass) and the
// strict order that picks it: any candidate over none, then the smaller
// distance, then the lower rank.  A total order, so that any grouping of a
// minimum gives the same candidate.
template <typename T>
__device__ __forceinline__ bool cand_better(double d, int r, double od, int orr) {
  return r >= 0 && (orr < 0 || d < od || (d == od && r < orr));
}

template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ T dpp_t(T x) {  // old = +0
  if constexpr (sizeof(T) == 8)
    return dpp_f64<CTRL, ROWS>(x);
  else
    return __builtin_bit_cast(T, dpp_i32<CTRL, ROWS>(__builtin_bit_cast(int, x), 0));
}

template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ void best_scan_step(double& d, int& r, T& m, int key) {
  const double yd = dpp_f64<CTRL, ROWS>(d);
  const int yr = dpp_i32<CTRL, ROWS>(r, -1);
  const T ym = dpp_t<CTRL, ROWS, T>(m);
  const int ky = dpp_i32<CTRL, ROWS>(key, -1);
  const bool take = ky == key && cand_better<T>(yd, yr, d, r);
  d = take ? yd : d;
  r = take ? yr : r;
  m = take ? ym : m;
}

// Inclusive segmented minimum of candidates over a full wavefront, the network
// of seg_scan_wave.
template <typename T>
__device__ __forceinline__ void best_scan_wave(double& d, int& r, T& m, int key) {
  best_scan_step<kDppRowShr + 1, 0xf, T>(d, r, m, key);
  best_scan_step<kDppRowShr + 2, 0xf, T>(d, r, m, key);
  best_scan_step<kDppRowShr + 4, 0xf, T>(d, r, m, key);
  best_scan_step<kDppRowShr + 8, 0xf, T>(d, r, m, key);
  best_scan_step<kDppRowBcast15, 0xa, T>(d, r, m, key);
  best_scan_step<kDppRowBcast31, 0xc, T>(d, r, m, key);
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
  int64_t* best_rank;  // per-event best pair (fused selection), or NULL
  T* best_m;
  double target;
  unsigned long long* fallback;
  int64_t ne;
  int epb;         // events per wavefront tile
  int cap;         // particles staged per chunk (per wavefront)
  int qcap;        // pairs evaluated per round (per wavefront)
  int wave_bytes;  // LDS bytes per wavefront
};

// Lexicographic minimum of (distance bits, rank) over the workgroup, the mass
// travelling with it; every thread receives the result.  `red` holds 48
// bytes per wavefront, for at most four wavefronts (the 256-thread workgroups
// of k_event_reduce_big; it is the 16-double scratch of block_sum, reused).
template <typename T>
__device__ __forceinline__ void block_best(unsigned long long* bd, int64_t* br, T* bm, double* red) {
  auto take = [&](unsigned long long od, int64_t orr, T om) {
    if (od < *bd || (od == *bd && orr < *br)) {
      *bd = od;
      *br = orr;
      *bm = om;
    }
  };
#pragma unroll
  for (int d = 32; d > 0; d >>= 1)
    take(__shfl_xor(*bd, d), __shfl_xor(*br, d), __shfl_xor(*bm, d));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  unsigned long long* sd = reinterpret_cast<unsigned long long*>(red);
  int64_t* sr = reinterpret_cast<int64_t*>(sd + 4);
  double* sm = reinterpret_cast<double*>(sr + 4);
  __syncthreads();
  if (lane == 0) {
    sd[wid] = *bd;
    sr[wid] = *br;
    sm[wid] = (double)*bm;
  }
  __syncthreads();
  for (int w = 0; w < nw; ++w) take(sd[w], sr[w], (T)sm[w]);
  __syncthreads();
}

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
  const bool want_best = A.best_rank != nullptr;
  unsigned long long bd = ~0ull;  // this thread's best: distance bits, rank, mass
  int64_t br = -1;
  T bmass = T(0);
  if (A.pair_m || want_k || want_best) {
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
      if (want_best) {  // a thread's ranks only grow: a tie keeps the earlier one
        const double d = fabs((double)m - A.target);
        const unsigned long long b = (unsigned long long)__double_as_longlong(d);
        if (d == d && b < bd) {
          bd = b;
          br = r;
          bmass = m;
        }
      }
    }
    if (want_k) ksum = block_sum(ksum, red);
    if (want_best) block_best<T>(&bd, &br, &bmass, red);
  }
  if (threadIdx.x == 0) {
    if (want_best) {
      A.best_rank[e] = bd != ~0ull ? br : -1;
      A.best_m[e] = bd != ~0ull ? bmass : (T)__builtin_nan("");
    }
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

// Orders the LDS accesses of the lanes of one wavefront.  The waves of a
// workgroup work independently, so the forward reduction needs no workgroup
// barrier: LDS operations of one wavefront are performed in program order, and
// the fences keep the compiler from moving LDS accesses across this point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The value of x held by lane `lane` (uniform), for a 64-bit x.
__device__ __forceinline__ int64_t readlane64(int64_t x, int lane) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(uint64_t)x, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)((uint64_t)x >> 32), lane);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Last c in [lo, hi) with a[c] <= key (a non-decreasing, a[lo] <= key).
__device__ __forceinline__ int search_le32(const int* a, int lo, int hi, int key) {
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] <= key)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// LDS of one wavefront of the forward reduction (cap particles, qcap pairs):
//   cart[cap]  (px, py, pz, E)             staged Cartesian records
//   leg[2 cap] (pt, eta, phi, M), (mT, delta, mT - pt, M^2) per particle,
//              adjacent (one address for both reads)   compensated mode
//   pm[qcap]   FP64: pair masses of a round (stored from here, coalesced)
//   kev[epb+1] K of each of the chunk's events with pairs in a round
//              (compensated event mass)
//   bm[epb+1], br[epb+1]  best pair of each of the chunk's events with
//              pairs in a round: mass and in-event rank (-1: none)
//              (fused best-pair selection)
//   eo, en, ep [epb + 1] int               the chunk's events with pairs:
//              first particle, size, first pair (chunk-relative), then a
//              sentinel (np, 0, nq)
template <typename T, int MODE>
struct WaveLds {
  typename V4<T>::type* cart;
  typename V4<T>::type* leg;
  T* pm;
  double* kev;
  T* bm;
  int* br;
  int* eo;
  int* en;
  int* ep;
};

template <typename T, int MODE, bool BEST>
__host__ __device__ __forceinline__ size_t wave_lds_bytes(int cap, int qcap, int epb) {
  size_t b = (size_t)cap * 4 * sizeof(T);
  if (MODE == GLV_COMPENSATED) b += (size_t)cap * 8 * sizeof(T) + (size_t)(epb + 1) * sizeof(double);
  if (BEST)
    b += (size_t)(epb + 1) * (sizeof(T) + sizeof(int));  // each event's best of a round
  else if (sizeof(T) == 8)
    b += (size_t)qcap * sizeof(T);  // staged pair masses
  b += 3 * (size_t)(epb + 1) * sizeof(int);
  return (b + 31) & ~(size_t)31;
}

template <typename T, int MODE, bool BEST>
__device__ __forceinline__ WaveLds<T, MODE> carve_wave_lds(unsigned char* p, int cap, int qcap, int epb) {
  WaveLds<T, MODE> w;
  w.cart = reinterpret_cast<typename V4<T>::type*>(p);
  p += (size_t)cap * 4 * sizeof(T);
  if constexpr (MODE == GLV_COMPENSATED) {
    w.leg = reinterpret_cast<typename V4<T>::type*>(p);
    p += (size_t)cap * 8 * sizeof(T);
    w.kev = reinterpret_cast<double*>(p);
    p += (size_t)(epb + 1) * sizeof(double);
  } else {
    w.leg = nullptr;
    w.kev = nullptr;
  }
  w.pm = reinterpret_cast<T*>(p);
  w.bm = reinterpret_cast<T*>(p);
  if (BEST) {
    p += (size_t)(epb + 1) * sizeof(T);
    w.br = reinterpret_cast<int*>(p);
    p += (size_t)(epb + 1) * sizeof(int);
  } else {
    w.br = nullptr;
    if (sizeof(T) == 8) p += (size_t)qcap * sizeof(T);
  }
  w.eo = reinterpret_cast<int*>(p);
  w.en = w.eo + (epb + 1);
  w.ep = w.en + (epb + 1);
  return w;
}

// Particles of a chunk held in registers between their load and their
// staging: lane t of the wavefront keeps particles t, t + 64, ...; FP64 keeps
// one per lane (64 particles), FP32 two (128).  Particles of larger chunks
// past these are loaded when staged.
template <typename T>
struct Prefetch {
  static constexpr int kSlots = sizeof(T) == 8 ? 1 : 2;
  T v[kSlots][4];
};

template <typename T>
__device__ __forceinline__ void prefetch_chunk(const Cols4<T>& p, int64_t base, int np, int lane, Prefetch<T>* r) {
#pragma unroll
  for (int s = 0; s < Prefetch<T>::kSlots; ++s) {
    const int t = lane + 64 * s;
    if (t < np) {
#pragma unroll
      for (int k = 0; k < 4; ++k) r->v[s][k] = __builtin_nontemporal_load(p.c[k] + base + t);
    }
  }
}

// Converts one particle and writes its staged records (slot t).
template <typename T, int COORDS, int MODE>
__device__ __forceinline__ void stage_one(const WaveLds<T, MODE>& W, int t, T c0, T c1, T c2, T c3) {
  using R4 = typename V4<T>::type;
  T v[4];
  if constexpr (MODE == GLV_COMPENSATED) {  // (pt, eta, phi, M)
    const LegC<T> L = comp_leg_cart<T>(c0, c1, c2, c3, v);
    W.leg[2 * t] = R4{c0, c1, c2, c3};
    W.leg[2 * t + 1] = R4{L.mt, L.delta, L.dmt, L.m2};
  } else {
    to_cart<COORDS, T, true>(c0, c1, c2, c3, v);
  }
  W.cart[t] = R4{v[0], v[1], v[2], v[3]};
}

// Compensated leg terms of a staged particle, from its two leg records at q;
// *mass receives M.
template <typename T>
__device__ __forceinline__ LegC<T> staged_leg(const typename V4<T>::type* q, T* mass) {
  const typename V4<T>::type a = q[0];
  const typename V4<T>::type b = q[1];
  LegC<T> L;
  L.pt = a[0];
  L.eta = a[1];
  L.phi = a[2];
  *mass = a[3];
  L.mt = b[0];
  L.delta = b[1];
  L.dmt = b[2];
  L.m2 = b[3];
  return L;
}

// The chunk of a wavefront's tile that starts at the first event at or after
// `from` small enough to stage (n <= cap): [*ca, *cb), the longest run of
// consecutive events whose particles fit in cap slots and whose pairs number
// at most pcap (the first event always belongs to it).  *ca = nev: none left.
__device__ __forceinline__ void next_chunk(int from, int nev, uint64_t valid, bool mine, int64_t olo, int64_t ohi,
                                           int cap, int64_t plo, int64_t phi, int64_t pcap, int* ca, int* cb) {
  const uint64_t after = from >= 64 ? 0ull : (valid & (~0ull << from));
  const uint64_t small = __ballot(mine && (ohi - olo) <= (int64_t)cap) & after;
  const int a = small ? (int)__builtin_ctzll(small) : nev;
  int b = a;
  if (a < nev) {
    const int64_t base = readlane64(olo, a), pbase = readlane64(plo, a);
    const uint64_t ge = valid & (~0ull << a);
    const uint64_t fits = __ballot(mine && (ohi - base <= (int64_t)cap) && (phi - pbase <= pcap)) & ge;
    // the first event always opens the chunk (its pairs then take several rounds)
    const uint64_t stop = ge & ~fits & ~(1ull << a);
    b = stop ? (int)__builtin_ctzll(stop) : nev;
  }
  *ca = a;
  *cb = b;
}

// Wavefronts per SIMD the compiler must leave room for (its register budget):
// five for the FP32 compensated reduction and the plain best pair, which
// otherwise take 107 and 101 VGPRs and four wavefronts (a few bytes then
// spill; on 2^20 events FP32 compensated 233 -> 218 us, fused best pair
// 205 -> 198 us); none for the FP64 compensated mode and the compensated best
// pair, which would spill more (the FP32 one measured 257 -> 292 us); the
// plain reductions fit six anyway.
template <typename T, int MODE, bool BEST>
constexpr int fwd_waves() {
  return (MODE == GLV_COMPENSATED && (sizeof(T) == 8 || BEST)) ? 1 : 5;
}

// The forward reduction.  Each wavefront of a workgroup independently takes a
// tile of epb consecutive events (one per lane for their offsets) and walks it
// in chunks of consecutive events holding at most cap particles; the next
// chunk's particles are loaded into registers while the current one is
// reduced, so that their latency hides behind its arithmetic:
//   1. stage: the chunk's particles are converted once and written to the
//      wave's LDS;
//   2. totals: four lanes per event, each summing one residue class of the
//      particle index modulo 4 in index order, combined as
//      ((P0 + P1) + (P2 + P3)) (the plain event mass from that total; in the
//      compensated mode also the sum of M^2);
//   3. pairs, in rounds: lane L takes the contiguous pairs [L m, (L + 1) m)
//      of the round, locates the first by a binary search over the chunk's
//      events with pairs and the square-root decode of its rank, then steps
//      to the lexicographic successor -- every lane the same number of pairs
//      whatever the event sizes, and a handful of integer operations per
//      step.  FP64 masses go to the wave's LDS, in rounds of 64 m pairs with m
//      odd (which spreads one LDS store instruction's lanes over distinct
//      banks), and from there to pair_m with coalesced stores; FP32 masses
//      (two lanes of a store instruction per 64-byte segment at m = 8) are
//      stored by their lane, in one round (plain mode) or rounds of qcap
//      (compensated mode and best pair, whose chunks hold at most one round
//      of pairs unless a single event has more).  In the compensated mode
//      each lane also sums K = E_i E_j - p_i.p_j of its pairs per event: an
//      event inside one run takes the lane's sum, an event spanning runs the
//      scan of their tails (keyed by event over the lanes) plus the head of
//      the run where it ends; the event's lane adds its K per round:
//      deterministic for a tiling.
// Events with more than cap particles are left to k_event_reduce_big.  In
// the FP32 compensated mode a pair whose error bound asks for FP64 makes its
// K a NaN; the event's lane then writes a marker -- a quiet NaN with a fixed
// payload -- into the event mass (or, without event masses, into the event's
// first pair mass), and k_event_reduce_big recomputes the event.
template <typename T, int COORDS, int MODE, bool BEST>
__global__ __launch_bounds__(kMaxBlock, (fwd_waves<T, MODE, BEST>())) void k_event_reduce(FwdArgs<T, COORDS, MODE> A) {
  extern __shared__ __align__(32) unsigned char lds[];
  constexpr bool kComp = MODE == GLV_COMPENSATED;
  constexpr bool kDefer = kComp && (sizeof(T) == 4);
  constexpr int kSlots = Prefetch<T>::kSlots;
  constexpr bool kStageMasses = sizeof(T) == 8 && !BEST;
  using R4 = typename V4<T>::type;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nwaves = blockDim.x >> 6;
  const int epb = A.epb, cap = A.cap, qcap = A.qcap;
  const WaveLds<T, MODE> W = carve_wave_lds<T, MODE, BEST>(lds + (size_t)wid * A.wave_bytes, cap, qcap, epb);

  const int64_t e0 = ((int64_t)blockIdx.x * nwaves + wid) * epb;
  if (e0 >= A.ne) return;  // the whole wavefront: no workgroup barrier follows
  const int nev = (int)min((int64_t)epb, A.ne - e0);
  const bool want_pairs = !BEST && A.pair_m != nullptr;
  // FP32 compensated: K is summed whenever pairs are evaluated (a NaN sum marks the redo)
  const bool want_k = kComp && (A.event_m != nullptr || (kDefer && (want_pairs || BEST)));
  const bool need_po = want_pairs || want_k || BEST;
  const bool want_sums = A.total[0] != nullptr || A.event_m != nullptr;

  // this lane's event of the tile
  const bool mine = lane < nev;
  int64_t olo = 0, ohi = 0, plo = 0, phi = 0;
  if (mine) {
    olo = A.off[e0 + lane];
    ohi = A.off[e0 + lane + 1];
    if (need_po) {
      plo = A.poff[e0 + lane];
      phi = A.poff[e0 + lane + 1];
    }
  }
  const uint64_t valid = (nev >= 64) ? ~0ull : ((1ull << nev) - 1);
  // where the rounds hold per-pair partials (compensated, best pair), a chunk
  // takes at most one round of pairs, so that no round runs nearly empty
  // (FP32 compensated 252 -> 241 us, best pair 254 -> 225 us on 2^20
  // Poisson(8) events); an event with more pairs alone takes several rounds
  const int64_t pcap = (kComp || BEST) && need_po ? (int64_t)qcap : ((int64_t)1 << 62);
  unsigned fb = 0;

  int ca, cb;
  next_chunk(0, nev, valid, mine, olo, ohi, cap, plo, phi, pcap, &ca, &cb);
  Prefetch<T> pre;
  if (ca < nev) {
    const int64_t b0 = readlane64(olo, ca);
    prefetch_chunk(A.p, b0, (int)(readlane64(ohi, cb - 1) - b0), lane, &pre);
  }
  while (ca < nev) {
    const int64_t base = readlane64(olo, ca);
    const int np = (int)(readlane64(ohi, cb - 1) - base);
    const int64_t q0 = need_po ? readlane64(plo, ca) : 0;
    const int nq = need_po ? (int)(readlane64(phi, cb - 1) - q0) : 0;
    const bool in_chunk = lane >= ca && lane < cb;
    const int lo_rel = (int)(olo - base), n_e = (int)(ohi - olo);

    // the chunk's events with pairs, compacted, then the sentinel
    const bool has_pairs = in_chunk && n_e >= 2;
    const uint64_t hp = __ballot(has_pairs);
    const int ncp = __builtin_popcountll(hp);
    const int my_c = __builtin_popcountll(hp & ((1ull << lane) - 1));  // this event among those with pairs
    if (need_po) {
      if (has_pairs) {
        const int c = my_c;
        W.eo[c] = lo_rel;
        W.en[c] = n_e;
        W.ep[c] = (int)(plo - q0);
      }
      if (lane == 0) {
        W.eo[ncp] = np;
        W.en[ncp] = 0;
        W.ep[ncp] = nq;
      }
    }

    // 1. stage the chunk's particles: those held in registers, then any
    //    beyond them straight from memory
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      const int t = lane + 64 * s;
      if (t < np) stage_one<T, COORDS, MODE>(W, t, pre.v[s][0], pre.v[s][1], pre.v[s][2], pre.v[s][3]);
    }
    for (int t = lane + 64 * kSlots; t < np; t += 64) {
      const int64_t gi = base + t;
      stage_one<T, COORDS, MODE>(W, t, A.p.c[0][gi], A.p.c[1][gi], A.p.c[2][gi], A.p.c[3][gi]);
    }
    wave_sync();

    // the next chunk's particles into registers, in flight from here on
    int na, nb;
    next_chunk(cb, nev, valid, mine, olo, ohi, cap, plo, phi, pcap, &na, &nb);
    if (na < nev) {
      const int64_t b1 = readlane64(olo, na);
      prefetch_chunk(A.p, b1, (int)(readlane64(ohi, nb - 1) - b1), lane, &pre);
    }

    // 2. totals: four lanes per event, one residue sum each (residue_sum),
    //    combined across the lane quad in the fixed order, 16 events per
    //    pass; the plain event mass from the total; in the compensated mode
    //    also the sum of M^2, handed to the event's lane
    double msum = 0.0;
    if (want_sums) {
      const int nk = cb - ca;  // events in the chunk
      const int rr = lane & 3;
      const R4* legs = nullptr;
      if constexpr (kComp) legs = W.leg;
      for (int c0 = 0; c0 < nk; c0 += 16) {
        const int c = c0 + (lane >> 2);
        const bool act = c < nk;
        const int src = min(ca + c, 63);
        const int glo = __shfl(lo_rel, src), gn = __shfl(n_e, src);
        const int lo = act ? glo : 0, hi = act ? glo + gn : 0;
        double tot[4] = {0, 0, 0, 0}, ms = 0.0;
        residue_sum(W.cart, lo, hi, rr, tot, legs, &ms);
        // (P0 + P1) + (P2 + P3): partner lane ^ 1, then lane ^ 2, of the quad
#pragma unroll
        for (int k = 0; k < 4; ++k) tot[k] = tot[k] + dpp_f64<kDppQuadXor1, 0xf>(tot[k]);
#pragma unroll
        for (int k = 0; k < 4; ++k) tot[k] = tot[k] + dpp_f64<kDppQuadXor2, 0xf>(tot[k]);
        if constexpr (kComp) {
          ms = ms + dpp_f64<kDppQuadXor1, 0xf>(ms);
          ms = ms + dpp_f64<kDppQuadXor2, 0xf>(ms);
        }
        if (act && rr == 0) {
          const int64_t e = e0 + ca + c;
          T tt[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) tt[k] = (T)tot[k];
          if (A.total[0]) {
#pragma unroll
            for (int k = 0; k < 4; ++k) store_out(A.total[k], e, tt[k]);
          }
          if constexpr (!kComp) {
            if (A.event_m) store_out(A.event_m, e, mass_of(tt));
          }
        }
        if constexpr (kComp) {
          // the event lanes of this pass take their quad's sum of M^2
          const int q = lane - ca - c0;
          const double mq = __shfl(ms, min(max(q, 0), 15) << 2);
          if (q >= 0 && q < 16 && in_chunk) msum = mq;
        }
      }
    }

    // 3. pairs, in rounds
    double ks = 0.0;  // the event lane's sum of K (compensated)
    double ebd = 0.0;  // the event lane's best pair (ebr < 0: none yet)
    int ebr = -1;
    T ebm = T(0);
    if (need_po) {
      // the records the pair loop reads per particle: the compensated legs
      // (two records each) or the Cartesian vectors
      constexpr int kStride = kComp ? 2 : 1;
      const R4* const recs = kComp ? W.leg : W.cart;
      const int rcap = kStageMasses ? 64 * (((qcap >> 6) - 1) | 1) : ((kComp || BEST) ? qcap : 0x3fffffff);
      T* const pout = want_pairs ? A.pair_m + q0 : nullptr;
      for (int r0 = 0; r0 < nq; r0 += rcap) {
        const int qn = min(rcap, nq - r0);
        // pairs per lane, odd where the masses pass through LDS
        const int m = kStageMasses ? (((qn + 63) >> 6) | 1) : ((qn + 63) >> 6);
        int k = r0 + lane * m;
        const int kend = min(k + m, r0 + qn);
        // the run's K partials of events it shares with other runs: the head
        // (the end of an event begun before the run) and the tail (the start
        // of an event that goes on after it); events wholly inside the run go
        // to kev directly
        double head = 0.0, tail = 0.0;
        double hd = 0.0, td = 0.0;  // best pair: the head's and the tail's candidates
        int hr = -1, tr = -1;
        T hm = T(0), tm = T(0);
        bool has_head = false, has_tail = false, first_seg = true, began_before = false;
        int head_c = 0, cur_c = ncp;  // cur_c: the run's current event (after a closing pair: the next)
        const bool ran = k < kend;
        if (k < kend) {
          int c = search_le32(W.ep, 0, ncp, k);
          const int o = W.eo[c], n = W.en[c];
          int i, j;
          decode_pair_small(k - W.ep[c], n, &i, &j);
          int cn = c + 1;
          int on = W.eo[cn], nn = W.en[cn];  // the next event with pairs (or the sentinel)
          // the staged records of the pair's two particles and the end of
          // their event, stepped directly (kStride records per particle)
          const R4* qa = recs + kStride * (o + i);
          const R4* qb = recs + kStride * (o + j);
          const R4* qe = recs + kStride * (o + n);
          double kacc = 0.0;
          int rk = k - W.ep[c];  // in-event rank of pair k
          cur_c = c;
          began_before = rk > 0;
          double bdist = 0.0;    // the run's best so far (brk < 0: none)
          int brk = -1;
          T bmass = T(0);
          for (; k < kend; ++k) {
            T mk;
            if constexpr (kComp) {
              T ma, mb;
              const LegC<T> la = staged_leg<T>(qa, &ma), lb = staged_leg<T>(qb, &mb);
              double kd;
              if constexpr (kDefer) {
                bool redo;
                float kf;
                mk = sqrt_budgeted(comp_pair_m2<float>(la, lb, &kf, &redo));
                kd = (double)(redo ? __builtin_nanf("") : kf);
              } else {
                mk = comp_pair<T>(la, lb, ma, mb, &kd, &fb);
              }
              kacc += kd;
            } else {
              const R4 ra = *qa, b = *qb;
              T w[4];
#pragma unroll
              for (int q = 0; q < 4; ++q) w[q] = ra[q] + b[q];
              mk = mass_of(w);
            }
            if constexpr (BEST) {
              // ranks grow along the run, so a tie keeps the earlier pair
              const double d = fabs((double)mk - A.target);
              if (d == d && (brk < 0 || d < bdist)) {
                bdist = d;
                brk = rk;
                bmass = mk;
              }
              ++rk;
            } else if constexpr (kStageMasses) {
              W.pm[k - r0] = mk;
            } else if (want_pairs) {
              pout[k] = mk;
            }
            // lexicographic successor within the chunk
            const int seg_c = cur_c;  // pair k's event
            bool fin = false;
            qb += kStride;
            if (qb == qe) {  // the row's last partner: the next row
              qa += kStride;
              if (qa + kStride == qe) {  // the event's last pair: the next event
                fin = true;
                qa = recs + kStride * on;
                qe = qa + kStride * nn;
                cur_c = cn;
                cn = min(cn + 1, ncp);
                on = W.eo[cn];
                nn = W.en[cn];
              }
              qb = qa + kStride;
            }
            if (fin || k + 1 == kend) {  // the run's partials at its last pair of the event
              // the head ends an event begun in an earlier run, the tail starts
              // one that goes on in the next run; an event wholly inside the
              // run goes to its slot directly
              const bool is_head = fin && first_seg && began_before;
              if constexpr (kComp) {
                if (is_head)
                  head = kacc;
                else if (fin)
                  W.kev[seg_c] = kacc;
                else
                  tail = kacc;
                kacc = 0.0;
              }
              if constexpr (BEST) {
                if (is_head) {
                  hd = bdist;
                  hr = brk;
                  hm = bmass;
                } else if (fin) {
                  W.bm[seg_c] = bmass;
                  W.br[seg_c] = brk;
                } else {
                  td = bdist;
                  tr = brk;
                  tm = bmass;
                }
                brk = -1;
                rk = 0;
              }
              if (is_head) {
                has_head = true;
                head_c = seg_c;
              }
              has_tail = !fin;
              first_seg = false;
            }
          }
        }
        // Each shared event's K (best pair): the tails of the runs it spans,
        // combined by a segmented scan keyed by event, then with the head of
        // the run where it ends; an event that goes on into the next round
        // takes the scan at the round's last run.  Keys grow with the lane: 2e
        // for a tail on event e, 2e + 1 for a run whose last event e closed in
        // it (cur_c is then e + 1), past every event for a run without pairs.
        const int key = has_tail ? 2 * cur_c : (ran ? 2 * cur_c - 1 : 2 * ncp + 1);
        if constexpr (BEST) {
          double sd = has_tail ? td : 0.0;
          int sr = has_tail ? tr : -1;
          T sm = has_tail ? tm : T(0);
          best_scan_wave<T>(sd, sr, sm, key);
          const double pd = dpp_f64<kDppWaveShr1, 0xf>(sd);
          const int pr = dpp_i32<kDppWaveShr1, 0xf>(sr, -1);
          const T pmv = dpp_t<kDppWaveShr1, 0xf, T>(sm);
          const int pk = dpp_i32<kDppWaveShr1, 0xf>(key, -1);
          if (has_head) {
            // the earlier runs' best, unless the head's is strictly better
            const bool from_prev = pk == 2 * head_c;
            double bd = from_prev ? pd : 0.0;
            int brr = from_prev ? pr : -1;
            T bmv = from_prev ? pmv : T(0);
            if (cand_better<T>(hd, hr, bd, brr)) {
              brr = hr;
              bmv = hm;
            }
            W.bm[head_c] = bmv;
            W.br[head_c] = brr;
          }
          if (has_tail && kend == r0 + qn) {
            W.bm[cur_c] = sm;
            W.br[cur_c] = sr;
          }
        }
        if constexpr (kComp) {
          if (want_k) {
            const double sc = seg_scan_wave(has_tail ? tail : 0.0, key);
            const double sp = dpp_f64<kDppWaveShr1, 0xf>(sc);
            const int kp = dpp_i32<kDppWaveShr1, 0xf>(key, -1);
            if (has_head) W.kev[head_c] = (kp == 2 * head_c ? sp : 0.0) + head;
            if (has_tail && kend == r0 + qn) W.kev[cur_c] = sc;
          }
        }
        wave_sync();
        if (kStageMasses && want_pairs) {
          T* out = A.pair_m + q0 + r0;
          for (int t = lane; t < qn; t += 64) store_out(out, t, W.pm[t]);
        }
        if constexpr (kComp) {
          if (want_k && in_chunk && n_e >= 2) {
            const int plo_rel = (int)(plo - q0), phi_rel = (int)(phi - q0);
            if (max(plo_rel, r0) < min(phi_rel, r0 + qn)) ks += W.kev[my_c];  // pairs in this round
          }
        }
        if constexpr (BEST) {
          if (in_chunk && n_e >= 2) {
            const int plo_rel = (int)(plo - q0), phi_rel = (int)(phi - q0);
            if (max(plo_rel, r0) < min(phi_rel, r0 + qn)) {  // pairs in this round (in rank order)
              const int r = W.br[my_c];
              if (r >= 0) {
                const T bmv = W.bm[my_c];
                const double d = fabs((double)bmv - A.target);
                if (ebr < 0 || d < ebd) {
                  ebd = d;
                  ebr = r;
                  ebm = bmv;
                }
              }
            }
          }
        }
        wave_sync();
      }
    }
    bool marked = false;  // FP32 compensated: a pair of the event asked for the FP64 redo
    if constexpr (kComp) {
      if (want_k && in_chunk) {
        marked = kDefer && (ks != ks) && n_e >= 2;
        if (A.event_m) {
          T em = (T)sqrt(msum + 2.0 * ks);
          if constexpr (kDefer) {
            if (marked) em = redo_mark();
          }
          store_out(A.event_m, e0 + lane, em);
        } else if (!BEST) {
          if constexpr (kDefer) {
            // without event masses the mark goes to the event's first pair
            // mass, after this wavefront's own stores of the chunk's masses
            if (__ballot(marked)) {
              // every earlier store of the wavefront completes first
              __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
              if (marked) A.pair_m[plo] = redo_mark();
            }
          }
        }
      }
    }
    if constexpr (BEST) {
      // without event masses a redo mark goes to the event's best mass
      if (in_chunk) {
        const bool mark_here = marked && A.event_m == nullptr;
        A.best_rank[e0 + lane] = ebr;
        store_out(A.best_m, e0 + lane, mark_here ? redo_mark() : (ebr >= 0 ? ebm : (T)__builtin_nan("")));
      }
    }
    wave_sync();
    ca = na;
    cb = nb;
  }
  if constexpr (kComp && sizeof(T) == 4) {
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
// Events each thread of the second launch sizes per pass (kBigScan coalesced
// slices of kBigBlock events): all their offsets are read at once, so the
// scan of 2^20 events takes one or two memory latencies per workgroup with a
// grid that fits the GPU (it took several rounds at one event per thread;
// four slices measured 1-2 % faster in the calls than eight or sixteen).
constexpr int kBigScan = 4;

// Sizes of events base + k kBigBlock + threadIdx.x, k < kBigScan, or -1 past
// the last event.
__device__ __forceinline__ void scan_sizes(const int64_t* off, int64_t ne, int64_t base, int64_t n[kBigScan]) {
  int64_t lo[kBigScan], hi[kBigScan];
#pragma unroll
  for (int k = 0; k < kBigScan; ++k) {
    const int64_t e = base + k * kBigBlock + threadIdx.x;
    lo[k] = 0;
    hi[k] = -1;
    if (e < ne) {
      lo[k] = off[e];
      hi[k] = off[e + 1];
    }
  }
#pragma unroll
  for (int k = 0; k < kBigScan; ++k) n[k] = hi[k] - lo[k];
}

template <typename T, int COORDS, int MODE>
__global__ __launch_bounds__(kBigBlock) void k_event_reduce_big(FwdArgs<T, COORDS, MODE> A) {
  constexpr bool kDefer = (MODE == GLV_COMPENSATED) && (sizeof(T) == 4);
  __shared__ double red[16];
  __shared__ int64_t list[kBigBlock];  // event << 1 | (1: redo only)
  __shared__ int count;
  unsigned fb = 0;
  const int64_t step = (int64_t)gridDim.x * kBigBlock * kBigScan;
  for (int64_t base = (int64_t)blockIdx.x * kBigBlock * kBigScan; base < A.ne; base += step) {
    // kBigScan coalesced slices of kBigBlock events, all offsets in flight at once
    int64_t n[kBigScan];
    scan_sizes(A.off, A.ne, base, n);
    unsigned bigm = 0, redom = 0;  // bit k: event k of this thread
#pragma unroll
    for (int k = 0; k < kBigScan; ++k) {
      if (n[k] > A.cap) bigm |= 1u << k;
      if constexpr (kDefer) {
        const int64_t e = base + k * kBigBlock + threadIdx.x;
        bool redo = false;
        if (n[k] >= 2 && n[k] <= A.cap) {
          if (A.event_m)
            redo = is_redo_mark(A.event_m[e]);
          else if (A.best_m)
            redo = is_redo_mark(A.best_m[e]);
          else if (A.pair_m)
            redo = is_redo_mark(A.pair_m[A.poff[e]]);
        }
        if (redo) redom |= 1u << k;
      }
    }
#pragma unroll 1
    for (int k = 0; k < kBigScan; ++k) {
      const int64_t e = base + k * kBigBlock + threadIdx.x;
      const bool big = (bigm >> k) & 1u, redo = (redom >> k) & 1u;
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
  const T* tot[4];  // the forward's event totals, or null: recomputed
  T* gp[4];
  int64_t ne;
  int epb;         // events per wavefront tile
  int cap;         // particles staged per chunk (per wavefront)
  int qcap;        // pair upstreams staged per chunk (per wavefront)
  int wave_bytes;  // LDS bytes per wavefront
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
  // total 4-vector for the event-mass term: the forward's, or summed here
  T ut[4] = {0, 0, 0, 0};
  if (A.gem) {
    T tot[4];
    if (A.tot[0]) {
#pragma unroll
      for (int k = 0; k < 4; ++k) tot[k] = A.tot[k][e];
    } else {
      double acc[4] = {0, 0, 0, 0};
      for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        T v[4];
        to_cart<COORDS>(A.p.c[0][i], A.p.c[1][i], A.p.c[2][i], A.p.c[3][i], v);
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += (double)v[k];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) tot[k] = (T)block_sum(acc[k], red);
    }
    dmass<T>(tot, A.gem[e], ut);
  }
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

// An event the tiled backward leaves to k_event_reduce_bwd_big: more than
// cap particles or, with pair upstreams, more than qcap pairs.
__device__ __forceinline__ bool bwd_big(int64_t n, int cap, int qcap, bool pairs) {
  return n > cap || (pairs && npairs(n) > (int64_t)qcap);
}

// LDS-staged backward.  A workgroup takes tiles of epb consecutive events and
// walks each in chunks of consecutive events with at most cap particles (one
// per thread: cap <= block) and, when pair upstreams are given, at most qcap
// pairs:
//   * thread t converts particle t of the chunk once, keeps its Cartesian
//     vector and Jacobian pieces (cos phi, sin phi, sinh eta, cosh eta) in
//     registers and stages the vector in LDS for its partners; the chunk's
//     pair upstreams -- contiguous in grad_pair -- are copied to LDS, two
//     loads in flight per thread; one lane per event records its particles'
//     event;
//   * pair phase: each pair's upstream g_ij becomes c_ij = g_ij / |m_ij| in
//     place, computed once, by one of its two legs: particle a of an event of
//     n takes the partners a + 1, ..., a + d cyclically, d = (n - 1) / 2
//     rounded down, plus a + n/2 when n is even and a < n/2 -- every pair
//     once, about n/2 per particle, whatever the particle's place;
//   * in the same phase a quad of threads per event sums the event's vectors
//     V as the forward does (or the event's lane, which loaded its g_total
//     and g_m with the chunk, takes V from the forward's totals), and
//     g_total + g_m dm(V)/dV, the upstream every particle of the event
//     receives from the event outputs, is staged;
//   * thread t sums the pair terms c_ij (v_i + v_j) = c_ij v_i + c_ij v_j
//     (dm(w)/dw = (-P, E) / |m|, the same 4-vector for both legs of a pair)
//     of its own pairs while evaluating them, then walks the partners that
//     evaluated its other pairs (b = a - d cyclically, stepping the pair
//     indices incrementally), adds the event's upstream and applies its own
//     conversion Jacobian.
// Every sum has a fixed order and no atomics are needed.  Six wavefronts per
// SIMD (what the LDS of the default tiling allows): the compiler keeps the
// registers within that (a few bytes spilled in FP64), 318 -> 309 us on 2^20
// events against its own choice of five.
template <typename T, int COORDS>
__global__ __launch_bounds__(kMaxBlock, 6) void k_event_reduce_bwd(BwdArgs<T, COORDS> A) {
  extern __shared__ __align__(32) unsigned char lds[];
  using R4 = typename V4<T>::type;
  const int epb = A.epb, cap = A.cap;  // cap <= blockDim.x
  const bool pairs = A.gpair != nullptr;
  const bool want_v = A.gem != nullptr;
  const int qcap = pairs ? A.qcap : 0;
  const int tid = (int)threadIdx.x;
  const bool want_u = want_v || A.gt[0] != nullptr;
  // LDS: cart[cap], s_ut[epb] (R4), s_g[qcap + 2] (T; qcap is even, one
  //      slot of slack), s_gm[epb rounded up to even] (T), s_off[epb+1],
  //      s_poff[epb+1] (int64), ch[epb+1] (EvRec), ev_of[cap] (uint16)
  R4* cart = reinterpret_cast<R4*>(lds);
  R4* s_ut = cart + cap;
  T* s_g = reinterpret_cast<T*>(s_ut + epb);
  T* s_gm = s_g + A.qcap + 2;
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
      if (bwd_big(s_off[ca + 1] - s_off[ca], cap, qcap, pairs)) {  // k_event_reduce_bwd_big's event
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
      // loads first: own particle, the first pair upstreams
      T c[4] = {0, 0, 0, 0};
      if (mine) {
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] = A.p.c[k][gi];
      }
      // pair upstreams per thread in flight (two: 317 against 325 us for four
      // on 2^20 events, whose registers cost occupancy)
      constexpr int kG = 2;
      T gv[kG];
#pragma unroll
      for (int r = 0; r < kG; ++r) {
        const int idx = tid + r * (int)blockDim.x;
        gv[r] = (idx < nq) ? A.gpair[q0 + idx] : T(0);
      }
      // the event lane's upstreams (g_total, g_m), staged with the rest
      const bool evl = want_u && tev < nch;
      const bool given_v = want_v && A.tot[0] != nullptr;  // the forward's totals: no sum here
      T gtv[4] = {0, 0, 0, 0}, gmv = 0, tv[4] = {0, 0, 0, 0};
      if (evl) {
        const int64_t e = e0 + ca + tev;
        if (A.gt[0]) {
#pragma unroll
          for (int k = 0; k < 4; ++k) gtv[k] = A.gt[k][e];
        }
        if (want_v) gmv = A.gem[e];
        if (given_v) {
#pragma unroll
          for (int k = 0; k < 4; ++k) tv[k] = A.tot[k][e];
        }
      }
      for (int t = tid; t <= nch; t += blockDim.x)
        ch[t] = EvRec{(int)(s_off[ca + t] - pbase), pairs ? (int)(s_poff[ca + t] - q0) : 0};
      for (int t = tid; t < nch; t += blockDim.x) {
        const int lo = (int)(s_off[ca + t] - pbase), hi = (int)(s_off[ca + t + 1] - pbase);
        for (int i = lo; i < hi; ++i) ev_of[i] = (unsigned short)t;
      }
#pragma unroll
      for (int r = 0; r < kG; ++r) {
        const int idx = tid + r * (int)blockDim.x;
        if (idx < nq) s_g[idx] = gv[r];
      }
      // upstreams past the first kG per thread (pairs_per_round > kG block)
      for (int base = kG * (int)blockDim.x; base < nq; base += kG * (int)blockDim.x) {
#pragma unroll
        for (int r = 0; r < kG; ++r) {
          const int idx = base + tid + r * (int)blockDim.x;
          gv[r] = (idx < nq) ? A.gpair[q0 + idx] : T(0);
        }
#pragma unroll
        for (int r = 0; r < kG; ++r) {
          const int idx = base + tid + r * (int)blockDim.x;
          if (idx < nq) s_g[idx] = gv[r];
        }
      }
      if (evl) {
        if (given_v) {  // g_total + g_m dm(V)/dV at once, from the forward's V
          T ud[4];
          dmass<T>(tv, gmv, ud);
          s_ut[tev] = R4{ud[0] + gtv[0], ud[1] + gtv[1], ud[2] + gtv[2], ud[3] + gtv[3]};
        } else {
          s_ut[tev] = R4{gtv[0], gtv[1], gtv[2], gtv[3]};
        }
        s_gm[tev] = gmv;
      }
      LegJ<T> L = to_cart_j<COORDS, T, true>(c[0], c[1], c[2], c[3]);
      if (mine) cart[tid] = R4{L.v[0], L.v[1], L.v[2], L.v[3]};
      __syncthreads();

      // four lanes per event (events spread over the wavefronts like the
      // event lanes): the upstream every particle's 4-vector receives from
      // the event outputs, g_total + g_m dm(V)/dV, with V summed as the
      // forward sums it (the same residue sums, combined in the same order)
      if (want_v && !given_v) {
        const int rr = tid & 3;
        const int qe = ((tid & 63) >> 2) * nw + (tid >> 6);
        for (int c0 = 0; c0 < nch; c0 += (int)blockDim.x >> 2) {
          const int c = c0 + qe;
          const bool act = c < nch;
          int lo = 0, hi = 0;
          if (act) {
            lo = ch[c].o;
            hi = ch[c + 1].o;
          }
          double vt[4] = {0, 0, 0, 0};
          residue_sum(cart, lo, hi, rr, vt);
#pragma unroll
          for (int k = 0; k < 4; ++k) vt[k] = vt[k] + dpp_f64<kDppQuadXor1, 0xf>(vt[k]);
#pragma unroll
          for (int k = 0; k < 4; ++k) vt[k] = vt[k] + dpp_f64<kDppQuadXor2, 0xf>(vt[k]);
          if (act && rr == 0) {
            T tot[4], ud[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) tot[k] = (T)vt[k];
            dmass<T>(tot, s_gm[c], ud);
            const R4 gt4 = s_ut[c];
            s_ut[c] = R4{ud[0] + gt4[0], ud[1] + gt4[1], ud[2] + gt4[2], ud[3] + gt4[3]};
          }
        }
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
      // S = sum of c_ab v_b and C = sum of c_ab over the partners b: the
      // thread's own pairs as it evaluates them, then (after the barrier) the
      // pairs its partners evaluated -- an order fixed by the event alone
      T S[4] = {0, 0, 0, 0}, C = 0;
      const int cnt = ((n - 1) >> 1) + ((n & 1) == 0 && 2 * ai < n ? 1 : 0);
      if (pairs) {
        if (mine) {
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
            const T cf = pair_coef<T>(w, g);
            s_g[q] = cf;
#pragma unroll
            for (int k = 0; k < 4; ++k) S[k] += cf * vj[k];
            C += cf;
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
          // the pairs evaluated by the partners b = a - d (cyclically),
          // d = 1, ..., n - 1 - cnt: pair (b, a) at R(b) + a - b - 1 while
          // b < a (R(b - 1) = R(b) - (n - b)), pair (a, b) at R(a) + b - a - 1
          // once b wraps to n - 1, n - 2, ...
          const int inc = n - 1 - cnt;
          int b = ai - 1, qlo = qrow - (n - ai), qhi = qrow + n - 2 - ai;
          for (int t = 0; t < inc; ++t) {
            const bool below = b >= 0;
            const int bb = below ? b : b + n;
            const T cs = s_g[below ? qlo : qhi];
            const R4 vj = cart[rc.o + bb];
#pragma unroll
            for (int k = 0; k < 4; ++k) S[k] += cs * vj[k];
            C += cs;
            if (below)
              qlo -= n - b - 1;
            else
              --qhi;
            --b;
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
  const int64_t step = (int64_t)gridDim.x * kBigBlock * kBigScan;
  for (int64_t base = (int64_t)blockIdx.x * kBigBlock * kBigScan; base < A.ne; base += step) {
    int64_t n[kBigScan];
    scan_sizes(A.off, A.ne, base, n);
    unsigned bigm = 0;  // bit k: event k of this thread
#pragma unroll
    for (int k = 0; k < kBigScan; ++k)
      if (n[k] >= 0 && bwd_big(n[k], A.cap, A.qcap, A.gpair != nullptr)) bigm |= 1u << k;
#pragma unroll 1
    for (int k = 0; k < kBigScan; ++k) {
      const int64_t e = base + k * kBigBlock + threadIdx.x;
      const bool big = (bigm >> k) & 1u;
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
}

int big_grid(int64_t ne) {
  constexpr int64_t per = (int64_t)kBigBlock * kBigScan;
  return (int)std::min<int64_t>(std::max<int64_t>(1, (ne + per - 1) / per), 2048);
}


int grid_for(int64_t ne, int epb) {
  int64_t tiles = (ne + epb - 1) / epb;
  if (tiles < 1) tiles = 1;
  if (tiles > 0x7fffffff) tiles = 0x7fffffff;
  return (int)tiles;
}

template <typename T, int COORDS, int MODE>
hipError_t fwd_typed(int64_t ne, const int64_t* off, const int64_t* poff, const void* const p[4],
                     void* const total[4], void* em, void* pm, const BestOut* best, unsigned long long* fb,
                     const Tiling& t, size_t lds, hipStream_t s) {
  FwdArgs<T, COORDS, MODE> A;
  A.best_rank = best ? best->rank : nullptr;
  A.best_m = best ? (T*)best->mass : nullptr;
  A.target = best ? best->target : 0.0;
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
  A.qcap = t.pairs_per_round;
  const int waves = t.block / 64;
  const int64_t tiles = (ne + t.events_per_tile - 1) / t.events_per_tile;
  if (best) {
    A.wave_bytes = (int)wave_lds_bytes<T, MODE, true>(t.lds_particles, t.pairs_per_round, t.events_per_tile);
    hipLaunchKernelGGL((k_event_reduce<T, COORDS, MODE, true>), dim3(grid_for(tiles, waves)), dim3(t.block), lds, s,
                       A);
  } else {
    A.wave_bytes = (int)wave_lds_bytes<T, MODE, false>(t.lds_particles, t.pairs_per_round, t.events_per_tile);
    hipLaunchKernelGGL((k_event_reduce<T, COORDS, MODE, false>), dim3(grid_for(tiles, waves)), dim3(t.block), lds, s,
                       A);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((k_event_reduce_big<T, COORDS, MODE>), dim3(big_grid(ne)), dim3(kBigBlock), 0, s, A);
  return hipGetLastError();
}

// The backward stages at most one particle per thread.
int bwd_cap(const Tiling& t) { return std::min(t.lds_particles, t.block); }

template <typename T, int COORDS>
hipError_t bwd_typed(int64_t ne, const int64_t* off, const int64_t* poff, const void* const p[4],
                     const void* const gt[4], const void* gem, const void* gpair, void* const gp[4],
                     const void* const tot[4], const Tiling& t, size_t lds, hipStream_t s) {
  BwdArgs<T, COORDS> A;
  for (int k = 0; k < 4; ++k) {
    A.p.c[k] = (const T*)p[k];
    A.gt[k] = gt ? (const T*)gt[k] : nullptr;
    A.tot[k] = tot ? (const T*)tot[k] : nullptr;
    A.gp[k] = (T*)gp[k];
  }
  A.off = off;
  A.poff = poff;
  A.gem = (const T*)gem;
  A.gpair = (const T*)gpair;
  A.ne = ne;
  A.epb = t.events_per_tile;
  A.cap = bwd_cap(t);
  A.qcap = t.pairs_per_round;
  A.wave_bytes = 0;
  hipLaunchKernelGGL((k_event_reduce_bwd<T, COORDS>), dim3(grid_for(ne, t.events_per_tile)), dim3(t.block), lds,
                     s, A);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((k_event_reduce_bwd_big<T, COORDS>), dim3(big_grid(ne)), dim3(kBigBlock), 0, s, A);
  return hipGetLastError();
}

template <typename T>
hipError_t fwd_dt(glv_coords co, glv_mode mode, int64_t ne, const int64_t* off, const int64_t* poff,
                  const void* const p[4], void* const total[4], void* em, void* pm, const BestOut* b,
                  unsigned long long* fb, const Tiling& t, size_t lds, hipStream_t s) {
  if (mode == GLV_COMPENSATED)
    return fwd_typed<T, GLV_PTETAPHIM, GLV_COMPENSATED>(ne, off, poff, p, total, em, pm, b, fb, t, lds, s);
  switch (co) {
    case GLV_PXPYPZE:
      return fwd_typed<T, GLV_PXPYPZE, GLV_PLAIN>(ne, off, poff, p, total, em, pm, b, nullptr, t, lds, s);
    case GLV_PTETAPHIM:
      return fwd_typed<T, GLV_PTETAPHIM, GLV_PLAIN>(ne, off, poff, p, total, em, pm, b, nullptr, t, lds, s);
    case GLV_PXPYPZM:
      return fwd_typed<T, GLV_PXPYPZM, GLV_PLAIN>(ne, off, poff, p, total, em, pm, b, nullptr, t, lds, s);
    default:
      return fwd_typed<T, GLV_PTETAPHIE, GLV_PLAIN>(ne, off, poff, p, total, em, pm, b, nullptr, t, lds, s);
  }
}

template <typename T>
hipError_t bwd_dt(glv_coords co, int64_t ne, const int64_t* off, const int64_t* poff, const void* const p[4],
                  const void* const gt[4], const void* gem, const void* gpair, void* const gp[4],
                  const void* const tot[4], const Tiling& t, size_t lds, hipStream_t s) {
  switch (co) {
    case GLV_PXPYPZE:
      return bwd_typed<T, GLV_PXPYPZE>(ne, off, poff, p, gt, gem, gpair, gp, tot, t, lds, s);
    case GLV_PTETAPHIM:
      return bwd_typed<T, GLV_PTETAPHIM>(ne, off, poff, p, gt, gem, gpair, gp, tot, t, lds, s);
    case GLV_PXPYPZM:
      return bwd_typed<T, GLV_PXPYPZM>(ne, off, poff, p, gt, gem, gpair, gp, tot, t, lds, s);
    default:
      return bwd_typed<T, GLV_PTETAPHIE>(ne, off, poff, p, gt, gem, gpair, gp, tot, t, lds, s);
  }
}

template <bool BEST>
size_t fwd_wave_bytes(glv_dtype dt, glv_mode mode, int cap, int qcap, int epb) {
  if (dt == GLV_F64)
    return mode == GLV_COMPENSATED ? wave_lds_bytes<double, GLV_COMPENSATED, BEST>(cap, qcap, epb)
                                   : wave_lds_bytes<double, GLV_PLAIN, BEST>(cap, qcap, epb);
  return mode == GLV_COMPENSATED ? wave_lds_bytes<float, GLV_COMPENSATED, BEST>(cap, qcap, epb)
                                 : wave_lds_bytes<float, GLV_PLAIN, BEST>(cap, qcap, epb);
}

}  // namespace

size_t event_reduce_lds_bytes(glv_dtype dt, glv_mode mode, const Tiling& t, bool best) {
  const size_t waves = (size_t)t.block / 64;
  const int cap = t.lds_particles, qcap = t.pairs_per_round, epb = t.events_per_tile;
  return waves * (best ? fwd_wave_bytes<true>(dt, mode, cap, qcap, epb)
                       : fwd_wave_bytes<false>(dt, mode, cap, qcap, epb));
}

size_t event_reduce_bwd_lds_bytes(glv_dtype dt, const Tiling& t) {
  const size_t tsz = (dt == GLV_F64) ? 8 : 4;
  const size_t cap = (size_t)bwd_cap(t), epb = (size_t)t.events_per_tile, qcap = (size_t)t.pairs_per_round;
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
                               void* pm, unsigned long long* fb, const Tiling& t, hipStream_t s,
                               const BestOut* best) {
  size_t lds = event_reduce_lds_bytes(dt, mode, t, best != nullptr);
  if (dt == GLV_F64) return fwd_dt<double>(co, mode, ne, off, poff, p, total, em, pm, best, nullptr, t, lds, s);
  return fwd_dt<float>(co, mode, ne, off, poff, p, total, em, pm, best, fb, t, lds, s);
}

hipError_t launch_event_reduce_bwd(glv_dtype dt, glv_coords co, int64_t ne, const int64_t* off,
                                   const int64_t* poff, const void* const p[4], const void* const gt[4],
                                   const void* gem, const void* gpair, void* const gp[4], const Tiling& t,
                                   hipStream_t s, const void* const tot[4]) {
  size_t lds = event_reduce_bwd_lds_bytes(dt, t);
  if (dt == GLV_F64) return bwd_dt<double>(co, ne, off, poff, p, gt, gem, gpair, gp, tot, t, lds, s);
  return bwd_dt<float>(co, ne, off, poff, p, gt, gem, gpair, gp, tot, t, lds, s);
}

}  // namespace glv
