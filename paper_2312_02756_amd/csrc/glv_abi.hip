// C ABI of the library (declared in include/glv.h): argument validation on
// the host, dispatch to the gfx950 launchers, the per-process tiling choice
// of the jagged reduction and its autotuner.
//
// Validation never touches device memory and runs before any HIP call, so
// every error path can be exercised on a machine without a GPU.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "glv.h"
#include "glv_autotune.h"
#include "glv_launch.h"

namespace {

thread_local int g_last_hip = 0;

glv_status hip_status(hipError_t e) {
  if (e == hipSuccess) return GLV_OK;
  g_last_hip = (int)e;
  return GLV_EHIP;
}

bool dtype_ok(glv_dtype d) { return d == GLV_F32 || d == GLV_F64; }
bool coords_ok(glv_coords c) {
  return c == GLV_PXPYPZE || c == GLV_PTETAPHIM || c == GLV_PTETAPHIE || c == GLV_PXPYPZM;
}
size_t elem(glv_dtype d) { return d == GLV_F64 ? 8 : 4; }

glv_status mode_ok(glv_mode m, glv_coords c) {
  if (m == GLV_PLAIN) return GLV_OK;
  if (m == GLV_COMPENSATED) return c == GLV_PTETAPHIM ? GLV_OK : GLV_EINVAL_MODE;
  return GLV_EINVAL_MODE;
}

// Byte ranges for overlap checks.
struct Range {
  uintptr_t lo, hi;  // [lo, hi)
};
Range rng(const void* p, int64_t n, size_t es) {
  uintptr_t a = reinterpret_cast<uintptr_t>(p);
  return {a, a + (uintptr_t)n * es};
}
bool overlap(const Range& a, const Range& b) { return a.lo < b.hi && b.lo < a.hi; }

bool any_overlap(const std::vector<Range>& outs, const std::vector<Range>& ins) {
  for (size_t i = 0; i < outs.size(); ++i) {
    for (size_t j = i + 1; j < outs.size(); ++j)
      if (overlap(outs[i], outs[j])) return true;
    for (const Range& r : ins)
      if (overlap(outs[i], r)) return true;
  }
  return false;
}

template <int N>
bool nonnull(const void* const* p) {
  if (!p) return false;
  for (int k = 0; k < N; ++k)
    if (!p[k]) return false;
  return true;
}

// ----------------------------------------------------------- tiling state

struct TileKey {
  int device, dtype, coords, mode;
  bool operator<(const TileKey& o) const {
    return std::tie(device, dtype, coords, mode) < std::tie(o.device, o.dtype, o.coords, o.mode);
  }
};
std::mutex g_tile_mu;
std::map<TileKey, glv::Tiling> g_tiles;  // autotuned choices
constexpr int kBwdKey = -1;              // TileKey::mode of the backward's choice

void remember_tiling(glv_dtype dt, glv_coords co, int mode_key, const glv::Tiling& t) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tiles[{dev, (int)dt, (int)co, mode_key}] = t;
}

void write_tiling(const glv::Tiling& t, glv_tiling* out) {
  out->block = t.block;
  out->events_per_tile = t.events_per_tile;
  out->lds_particles = t.lds_particles;
  out->pairs_per_round = t.pairs_per_round;
}

// Times every candidate on `s` (one warm-up launch, then the best of three)
// and sets *chosen to the fastest; `launch(t)` enqueues one launch.
template <typename Launch>
hipError_t pick_fastest(const std::vector<glv::Tiling>& cands, hipStream_t s, Launch launch, glv::Tiling* chosen) {
  hipEvent_t e0, e1;
  hipError_t err = hipEventCreate(&e0);
  if (err != hipSuccess) return err;
  err = hipEventCreate(&e1);
  if (err != hipSuccess) {
    (void)hipEventDestroy(e0);
    return err;
  }
  float best_ms = 1e30f;
  for (const glv::Tiling& t : cands) {
    err = launch(t);
    if (err != hipSuccess) break;
    float tmin = 1e30f;
    for (int rep = 0; rep < 3 && err == hipSuccess; ++rep) {
      err = hipEventRecord(e0, s);
      if (err == hipSuccess) err = launch(t);
      if (err == hipSuccess) err = hipEventRecord(e1, s);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err == hipSuccess) tmin = std::min(tmin, ms);
    }
    if (err != hipSuccess) break;
    if (tmin < best_ms) {
      best_ms = tmin;
      *chosen = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return err;
}

// Forward: independent wavefronts, each taking tiles of 32 events, staging up
// to 128 particles and evaluating 512 pairs (8 per lane) per round -- 1024 in
// the FP32 compensated mode, whose chunks hold at most one round and whose
// rounds cost no LDS (2 % faster on 2^20 Poisson(8) events); four per
// workgroup, or two for the FP64 compensated mode, whose wavefront stages
// 18.8 KB (four would pass the 64 KiB workgroup limit).
glv::Tiling default_tiling(glv_dtype dt, glv_mode mode) {
  glv::Tiling t;
  t.block = (dt == GLV_F64 && mode == GLV_COMPENSATED) ? 128 : 256;
  t.events_per_tile = 32;
  t.lds_particles = 128;
  t.pairs_per_round = (dt == GLV_F32 && mode == GLV_COMPENSATED) ? 1024 : 512;
  return t;
}

// Fused best-pair selection: one wavefront per workgroup, tiles of 64
// events, 128 staged particles and rounds of 1024 pairs (its own choice: the
// selection keeps one candidate per event in LDS, so larger rounds cost no
// LDS; on 2^20 Poisson(8) events the smallest workgroups measured fastest,
// and 1024-pair rounds 3 % faster than 512).
glv::Tiling default_tiling_best() {
  glv::Tiling t;
  t.block = 64;
  t.events_per_tile = 64;
  t.lds_particles = 128;
  t.pairs_per_round = 1024;
  return t;
}

// Backward: 128-thread workgroups taking tiles of 64 events, staging one
// particle per thread and 512 pair upstreams.
glv::Tiling default_tiling_bwd(glv_dtype dt) {
  (void)dt;
  glv::Tiling t;
  t.block = 128;
  t.events_per_tile = 64;
  t.lds_particles = 128;
  t.pairs_per_round = 512;
  return t;
}

constexpr size_t kMaxLds = 64 * 1024;

bool block_ok(int b) { return (b == 64 || b == 128 || b == 256 || b == 512) && b <= glv::kMaxBlock; }

// Every field inside its allowed set and the workgroup's LDS within kMaxLds.
bool tiling_valid(glv_dtype dt, glv_mode mode, bool bwd, const glv::Tiling& t, bool best = false) {
  if (!block_ok(t.block)) return false;
  if (t.events_per_tile < 1 || t.events_per_tile > 64) return false;
  if (t.lds_particles < 64 || t.lds_particles > 4096) return false;
  if (t.pairs_per_round < 64 || t.pairs_per_round > 4096 || t.pairs_per_round % 64 != 0) return false;
  const size_t lds = bwd ? glv::event_reduce_bwd_lds_bytes(dt, t) : glv::event_reduce_lds_bytes(dt, mode, t, best);
  return lds <= kMaxLds;
}

// Resolve a user tiling (fields 0 = current choice) and validate it.
glv_status resolve_tiling(glv_dtype dt, glv_coords co, glv_mode mode, const glv_tiling* user, bool bwd,
                          glv::Tiling* out, bool best = false) {
  glv::Tiling base = bwd ? default_tiling_bwd(dt) : best ? default_tiling_best() : default_tiling(dt, mode);
  if (!best) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    std::lock_guard<std::mutex> lk(g_tile_mu);
    auto it = g_tiles.find({dev, (int)dt, (int)co, bwd ? kBwdKey : (int)mode});
    if (it != g_tiles.end()) base = it->second;
  }
  if (user) {
    if (user->block) base.block = user->block;
    if (user->events_per_tile) base.events_per_tile = user->events_per_tile;
    if (user->lds_particles) base.lds_particles = user->lds_particles;
    if (user->pairs_per_round) base.pairs_per_round = user->pairs_per_round;
  }
  if (!tiling_valid(dt, mode, bwd, base, best)) return GLV_EINVAL_TILING;
  *out = base;
  return GLV_OK;
}

glv_status check_event_args(glv_dtype dt, glv_coords co, glv_mode mode, int64_t ne, const int64_t* off,
                            const void* const p[4]) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (!coords_ok(co)) return GLV_EINVAL_COORDS;
  glv_status ms = mode_ok(mode, co);
  if (ms != GLV_OK) return ms;
  if (ne < 0) return GLV_EINVAL_SIZE;
  if (ne == 0) return GLV_OK;  // nothing is read or written
  if (!off) return GLV_EINVAL_OFFSETS;
  if (!nonnull<4>(p)) return GLV_EINVAL_NULL;
  return GLV_OK;
}

glv_status validate_event_reduce(glv_dtype dt, glv_coords co, glv_mode mode, int64_t ne, const int64_t* off,
                                 const int64_t* poff, const void* const p[4], void* const total[4], void* em,
                                 void* pm) {
  glv_status st = check_event_args(dt, co, mode, ne, off, p);
  if (st != GLV_OK || ne == 0) return st;
  if (total && !nonnull<4>((const void* const*)total)) return GLV_EINVAL_NULL;
  if ((pm || (mode == GLV_COMPENSATED && em)) && !poff) return GLV_EINVAL_OFFSETS;
  // outputs must not overlap each other or the offsets (their lengths are
  // known on the host: n_events; pair and particle counts are not, so only
  // the start addresses of those are compared)
  std::vector<Range> outs, ins;
  size_t es = elem(dt);
  if (total)
    for (int k = 0; k < 4; ++k) outs.push_back(rng(total[k], ne, es));
  if (em) outs.push_back(rng(em, ne, es));
  ins.push_back(rng(off, ne + 1, 8));
  if (poff) ins.push_back(rng(poff, ne + 1, 8));
  if (any_overlap(outs, ins)) return GLV_EINVAL_ALIAS;
  for (int k = 0; k < 4; ++k) {
    for (const Range& r : outs)
      if (reinterpret_cast<uintptr_t>(p[k]) >= r.lo && reinterpret_cast<uintptr_t>(p[k]) < r.hi)
        return GLV_EINVAL_ALIAS;
    if (pm == p[k]) return GLV_EINVAL_ALIAS;
  }
  if (pm) {
    uintptr_t a = reinterpret_cast<uintptr_t>(pm);
    for (const Range& r : outs)
      if (a >= r.lo && a < r.hi) return GLV_EINVAL_ALIAS;
    for (const Range& r : ins)
      if (a >= r.lo && a < r.hi) return GLV_EINVAL_ALIAS;
  }
  return GLV_OK;
}

}  // namespace

namespace {

// Arguments of a forward transformation x[4] -> y[4] with K parameter
// columns m (n values each at stride 1, one value at stride 0).  y may be x
// itself, column for column.
template <int K>
glv_status transform_args(glv_dtype dt, int64_t n, const void* const x[4], const void* const* m, int64_t ms,
                          void* const y[4]) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (n < 0) return GLV_EINVAL_SIZE;
  if (ms != 0 && ms != 1) return GLV_EINVAL_STRIDE;
  if (n == 0) return GLV_OK;
  if (!nonnull<4>(x) || !nonnull<K>(m) || !nonnull<4>((const void* const*)y)) return GLV_EINVAL_NULL;
  const size_t es = elem(dt);
  bool inplace = true;
  for (int k = 0; k < 4; ++k) inplace = inplace && (y[k] == x[k]);
  std::vector<Range> outs, ins;
  for (int k = 0; k < 4; ++k) outs.push_back(rng(y[k], n, es));
  for (int k = 0; k < K; ++k) ins.push_back(rng(m[k], ms ? n : 1, es));
  if (!inplace)
    for (int k = 0; k < 4; ++k) ins.push_back(rng(x[k], n, es));
  if (any_overlap(outs, ins)) return GLV_EINVAL_ALIAS;
  if (inplace)
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j)
        if (overlap(rng(x[i], n, es), rng(x[j], n, es))) return GLV_EINVAL_ALIAS;
  return GLV_OK;
}

// Arguments of a reverse mode: grad_y[4] -> grad_x[4], and with gm (NN
// columns, stride 1 only) the per-item parameter gradient, which needs x.
// No output overlaps an input or another output.
template <int K, int NN>
glv_status transform_bwd_args(glv_dtype dt, int64_t n, const void* const x[4], const void* const* m, int64_t ms,
                              const void* const gy[4], void* const gx[4], void* const* gm) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (n < 0) return GLV_EINVAL_SIZE;
  if (ms != 0 && ms != 1) return GLV_EINVAL_STRIDE;
  if (gm && ms != 1) return GLV_EINVAL_STRIDE;
  if (n == 0) return GLV_OK;
  if (!nonnull<K>(m) || !nonnull<4>(gy) || !nonnull<4>((const void* const*)gx)) return GLV_EINVAL_NULL;
  if (gm && (!nonnull<NN>((const void* const*)gm) || !nonnull<4>(x))) return GLV_EINVAL_NULL;
  const size_t es = elem(dt);
  std::vector<Range> outs, ins;
  for (int k = 0; k < 4; ++k) {
    outs.push_back(rng(gx[k], n, es));
    ins.push_back(rng(gy[k], n, es));
    if (gm) ins.push_back(rng(x[k], n, es));
  }
  for (int k = 0; k < K; ++k) ins.push_back(rng(m[k], ms ? n : 1, es));
  if (gm)
    for (int k = 0; k < NN; ++k) outs.push_back(rng(gm[k], n, es));
  if (any_overlap(outs, ins)) return GLV_EINVAL_ALIAS;
  return GLV_OK;
}

}  // namespace


namespace {

// ------------------------------------------------------------- autotuning

// The persistent cache: the file named by GLV_AUTOTUNE_CACHE, if set.
const char* cache_path() {
  const char* p = getenv("GLV_AUTOTUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

enum class CacheFile { kUsable, kMissing, kCorrupt };

// Reads the cache file; a corrupt file (or one holding a tiling that is not
// valid here) is reported on stderr once per call and then ignored, and
// never rewritten.
CacheFile read_cache(const char* path, glv_dtype dt, glv_mode mode, bool bwd, glv::tune::Entries* entries) {
  std::string why;
  const glv::tune::FileState fs = glv::tune::load(path, entries, &why);
  if (fs == glv::tune::FileState::kMissing) return CacheFile::kMissing;
  if (fs == glv::tune::FileState::kCorrupt) {
    fprintf(stderr, "glv: autotune cache %s is corrupt (%s); ignoring it\n", path, why.c_str());
    entries->clear();
    return CacheFile::kCorrupt;
  }
  (void)dt;
  (void)mode;
  (void)bwd;
  for (const auto& e : *entries) {
    // the key names dtype and direction; check the tiling against them
    const bool e_bwd = e.first.find("|bwd|") != std::string::npos;
    const glv_dtype e_dt = e.first.find("|f64|") != std::string::npos ? GLV_F64 : GLV_F32;
    const glv_mode e_mode = e.first.find("|fwd-compensated|") != std::string::npos ? GLV_COMPENSATED : GLV_PLAIN;
    if (!tiling_valid(e_dt, e_mode, e_bwd, e.second)) {
      fprintf(stderr, "glv: autotune cache %s is corrupt (invalid tiling for %s); ignoring it\n", path,
              e.first.c_str());
      entries->clear();
      return CacheFile::kCorrupt;
    }
  }
  return CacheFile::kUsable;
}

// Cache key of a dataset for this device, dtype, coordinate system and
// direction (the forward's mode included).
glv_status dataset_key(glv_dtype dt, glv_coords co, glv_mode mode, bool bwd, int64_t ne, const int64_t* off,
                       hipStream_t s, std::string* key) {
  std::string sig;
  if (ne > 0) {
    const hipError_t e = glv::tune::signature(ne, off, s, &sig);
    if (e != hipSuccess) return hip_status(e);
  } else {
    sig = glv::tune::signature_of_sizes(0, nullptr, 0);
  }
  const char* what = bwd ? "bwd" : (mode == GLV_COMPENSATED ? "fwd-compensated" : "fwd-plain");
  *key = glv::tune::make_key(dt, co, what, sig);
  return GLV_OK;
}

// The autotuners' common part: the dataset's key; its tiling from this
// process's earlier choices or the cache file, else the fastest candidate
// (timed on the caller's data, `launch` enqueueing one launch; the outputs
// end up holding that tiling's result), added to the cache file.
template <typename Launch>
glv_status autotune_common(glv_dtype dt, glv_coords co, glv_mode mode, bool bwd, int64_t ne, const int64_t* off,
                           const std::vector<glv::Tiling>& cands, const glv::Tiling& dflt, bool work, Launch launch,
                           glv_tiling* best, hipStream_t s) {
  std::string key;
  glv_status st = dataset_key(dt, co, mode, bwd, ne, off, s, &key);
  if (st != GLV_OK) return st;
  glv::Tiling chosen = dflt;
  bool hit = glv::tune::lookup_process(key, &chosen);
  const char* path = cache_path();
  glv::tune::Entries entries;
  CacheFile cf = CacheFile::kMissing;
  if (!hit && path) {
    cf = read_cache(path, dt, mode, bwd, &entries);
    for (const auto& e : entries) {
      if (e.first == key) {
        chosen = e.second;
        hit = true;
      }
    }
  }
  if (work) {
    hipError_t err = hipSuccess;
    if (!hit) err = pick_fastest(cands, s, launch, &chosen);
    if (err == hipSuccess) err = launch(chosen);  // the outputs hold the chosen tiling's result
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err != hipSuccess) return hip_status(err);
  }
  if (!hit && work && path && cf != CacheFile::kCorrupt) {
    entries.push_back({key, chosen});
    if (!glv::tune::save(path, entries))
      fprintf(stderr, "glv: could not write the autotune cache %s\n", path);
  }
  if (hit || work) glv::tune::remember_process(key, chosen);
  remember_tiling(dt, co, bwd ? kBwdKey : (int)mode, chosen);
  if (best) write_tiling(chosen, best);
  return GLV_OK;
}

}  // namespace

extern "C" {

int glv_abi_version(void) { return GLV_ABI_VERSION; }

int glv_last_hip_error(void) { return g_last_hip; }

const char* glv_status_str(glv_status s) {
  switch (s) {
    case GLV_OK: return "ok";
    case GLV_EINVAL_NULL: return "a required pointer is NULL";
    case GLV_EINVAL_SIZE: return "negative element or event count";
    case GLV_EINVAL_DTYPE: return "unknown dtype";
    case GLV_EINVAL_COORDS: return "unknown coordinate system";
    case GLV_EINVAL_MODE: return "mode unknown or not available for these coordinates";
    case GLV_EINVAL_ALIAS: return "an output overlaps an input or another output";
    case GLV_EINVAL_STRIDE: return "beta_stride must be 0 or 1 (1 when grad_beta is requested)";
    case GLV_EINVAL_OFFSETS: return "offsets or pair_offsets missing";
    case GLV_EINVAL_TILING: return "tiling field outside its allowed set";
    case GLV_EHIP: return "HIP error";
  }
  return "unknown status";
}

glv_status glv_invariant_mass(glv_dtype dt, glv_coords co, glv_mode mode, int64_t n, const void* const a[4],
                              const void* const b[4], void* m, unsigned long long* fallback, void* stream) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (!coords_ok(co)) return GLV_EINVAL_COORDS;
  glv_status ms = mode_ok(mode, co);
  if (ms != GLV_OK) return ms;
  if (n < 0) return GLV_EINVAL_SIZE;
  if (n == 0) return GLV_OK;
  if (!nonnull<4>(a) || !nonnull<4>(b) || !m) return GLV_EINVAL_NULL;
  size_t es = elem(dt);
  std::vector<Range> ins;
  for (int k = 0; k < 4; ++k) {
    ins.push_back(rng(a[k], n, es));
    ins.push_back(rng(b[k], n, es));
  }
  if (fallback) ins.push_back(rng(fallback, 1, 8));
  if (any_overlap({rng(m, n, es)}, ins)) return GLV_EINVAL_ALIAS;
  return hip_status(glv::launch_mass(dt, co, mode, n, a, b, m, fallback, (hipStream_t)stream));
}

namespace {

// Arguments of a pair-mass reverse mode (validated before any launch).
glv_status mass_bwd_args(glv_dtype dt, int64_t n, const void* const a[4], const void* const b[4], const void* gm,
                         void* const ga[4], void* const gb[4]) {
  if (!nonnull<4>(a) || !nonnull<4>(b) || !gm || !nonnull<4>((const void* const*)ga) ||
      !nonnull<4>((const void* const*)gb))
    return GLV_EINVAL_NULL;
  size_t es = elem(dt);
  std::vector<Range> ins, outs;
  for (int k = 0; k < 4; ++k) {
    ins.push_back(rng(a[k], n, es));
    ins.push_back(rng(b[k], n, es));
    outs.push_back(rng(ga[k], n, es));
    outs.push_back(rng(gb[k], n, es));
  }
  ins.push_back(rng(gm, n, es));
  return any_overlap(outs, ins) ? GLV_EINVAL_ALIAS : GLV_OK;
}

}  // namespace

glv_status glv_invariant_mass_comp_bwd(glv_dtype dt, int64_t n, const void* const a[4], const void* const b[4],
                                       const void* gm, void* const ga[4], void* const gb[4], void* stream) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (n < 0) return GLV_EINVAL_SIZE;
  if (n == 0) return GLV_OK;
  const glv_status st = mass_bwd_args(dt, n, a, b, gm, ga, gb);
  if (st != GLV_OK) return st;
  return hip_status(glv::launch_mass_comp_bwd(dt, n, a, b, gm, ga, gb, (hipStream_t)stream));
}

glv_status glv_invariant_mass_bwd(glv_dtype dt, glv_coords co, int64_t n, const void* const a[4],
                                  const void* const b[4], const void* gm, void* const ga[4], void* const gb[4],
                                  void* stream) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (!coords_ok(co)) return GLV_EINVAL_COORDS;
  if (n < 0) return GLV_EINVAL_SIZE;
  if (n == 0) return GLV_OK;
  const glv_status st = mass_bwd_args(dt, n, a, b, gm, ga, gb);
  if (st != GLV_OK) return st;
  return hip_status(glv::launch_mass_bwd(dt, co, n, a, b, gm, ga, gb, (hipStream_t)stream));
}

glv_status glv_boost(glv_dtype dt, int64_t n, const void* const x[4], const void* const beta[3],
                     int64_t beta_stride, void* const y[4], void* stream) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (n < 0) return GLV_EINVAL_SIZE;
  if (beta_stride != 0 && beta_stride != 1) return GLV_EINVAL_STRIDE;
  if (n == 0) return GLV_OK;
  if (!nonnull<4>(x) || !nonnull<3>(beta) || !nonnull<4>((const void* const*)y)) return GLV_EINVAL_NULL;
  size_t es = elem(dt);
  bool inplace = true;
  for (int k = 0; k < 4; ++k) inplace = inplace && (y[k] == x[k]);
  std::vector<Range> outs, ins;
  for (int k = 0; k < 4; ++k) outs.push_back(rng(y[k], n, es));
  for (int k = 0; k < 3; ++k) ins.push_back(rng(beta[k], beta_stride ? n : 1, es));
  if (!inplace)
    for (int k = 0; k < 4; ++k) ins.push_back(rng(x[k], n, es));
  if (any_overlap(outs, ins)) return GLV_EINVAL_ALIAS;
  if (inplace) {
    // in place is column for column; the x columns must still be disjoint
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j)
        if (overlap(rng(x[i], n, es), rng(x[j], n, es))) return GLV_EINVAL_ALIAS;
  }
  return hip_status(glv::launch_boost(dt, n, x, beta, beta_stride, y, (hipStream_t)stream));
}

glv_status glv_convert(glv_dtype dt, glv_coords from, glv_coords to, int64_t n, const void* const in[4],
                       void* const out[4], void* stream) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (!coords_ok(from) || !coords_ok(to)) return GLV_EINVAL_COORDS;
  if (n < 0) return GLV_EINVAL_SIZE;
  if (n == 0) return GLV_OK;
  if (!nonnull<4>(in) || !nonnull<4>((const void* const*)out)) return GLV_EINVAL_NULL;
  size_t es = elem(dt);
  bool inplace = true;
  for (int k = 0; k < 4; ++k) inplace = inplace && (out[k] == in[k]);
  std::vector<Range> outs, ins;
  for (int k = 0; k < 4; ++k) {
    outs.push_back(rng(out[k], n, es));
    if (!inplace) ins.push_back(rng(in[k], n, es));
  }
  if (any_overlap(outs, ins)) return GLV_EINVAL_ALIAS;  // in place: column for column, columns disjoint
  return hip_status(glv::launch_convert(dt, from, to, n, in, out, (hipStream_t)stream));
}

glv_status glv_convert_bwd(glv_dtype dt, glv_coords from, glv_coords to, int64_t n, const void* const in[4],
                           const void* const grad_out[4], void* const grad_in[4], void* stream) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (!coords_ok(from) || !coords_ok(to)) return GLV_EINVAL_COORDS;
  if (n < 0) return GLV_EINVAL_SIZE;
  if (n == 0) return GLV_OK;
  if (!nonnull<4>(in) || !nonnull<4>(grad_out) || !nonnull<4>((const void* const*)grad_in))
    return GLV_EINVAL_NULL;
  size_t es = elem(dt);
  bool inplace = true;  // grad_in over grad_out, column for column
  for (int k = 0; k < 4; ++k) inplace = inplace && (grad_in[k] == grad_out[k]);
  std::vector<Range> outs, ins;
  for (int k = 0; k < 4; ++k) {
    outs.push_back(rng(grad_in[k], n, es));
    ins.push_back(rng(in[k], n, es));
    if (!inplace) ins.push_back(rng(grad_out[k], n, es));
  }
  if (any_overlap(outs, ins)) return GLV_EINVAL_ALIAS;
  return hip_status(glv::launch_convert_bwd(dt, from, to, n, in, grad_out, grad_in, (hipStream_t)stream));
}

glv_status glv_boost_bwd(glv_dtype dt, int64_t n, const void* const x[4], const void* const beta[3],
                         int64_t beta_stride, const void* const gy[4], void* const gx[4], void* const gbeta[3],
                         void* stream) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (n < 0) return GLV_EINVAL_SIZE;
  if (beta_stride != 0 && beta_stride != 1) return GLV_EINVAL_STRIDE;
  if (gbeta && beta_stride != 1) return GLV_EINVAL_STRIDE;
  if (n == 0) return GLV_OK;
  if (!nonnull<3>(beta) || !nonnull<4>(gy) || !nonnull<4>((const void* const*)gx)) return GLV_EINVAL_NULL;
  if (gbeta && (!nonnull<3>((const void* const*)gbeta) || !nonnull<4>(x))) return GLV_EINVAL_NULL;
  size_t es = elem(dt);
  std::vector<Range> outs, ins;
  for (int k = 0; k < 4; ++k) {
    outs.push_back(rng(gx[k], n, es));
    ins.push_back(rng(gy[k], n, es));
    if (gbeta) ins.push_back(rng(x[k], n, es));
  }
  for (int k = 0; k < 3; ++k) {
    ins.push_back(rng(beta[k], beta_stride ? n : 1, es));
    if (gbeta) outs.push_back(rng(gbeta[k], n, es));
  }
  if (any_overlap(outs, ins)) return GLV_EINVAL_ALIAS;
  return hip_status(glv::launch_boost_bwd(dt, n, x, beta, beta_stride, gy, gx, gbeta, (hipStream_t)stream));
}

// ---------------------------------------------- general transformations

glv_status glv_lorentz_transform(glv_dtype dt, int64_t n, const void* const x[4], const void* const L[16],
                                 int64_t L_stride, void* const y[4], void* stream) {
  const glv_status st = transform_args<16>(dt, n, x, L, L_stride, y);
  if (st != GLV_OK || n == 0) return st;
  return hip_status(glv::launch_transform(dt, glv::kTfLorentz, n, x, L, L_stride, y, (hipStream_t)stream));
}

glv_status glv_lorentz_transform_bwd(glv_dtype dt, int64_t n, const void* const x[4], const void* const L[16],
                                     int64_t L_stride, const void* const grad_y[4], void* const grad_x[4],
                                     void* const grad_L[16], void* stream) {
  const glv_status st = transform_bwd_args<16, 16>(dt, n, x, L, L_stride, grad_y, grad_x, grad_L);
  if (st != GLV_OK || n == 0) return st;
  return hip_status(glv::launch_transform_bwd(dt, glv::kTfLorentz, n, x, L, L_stride, grad_y, grad_x, grad_L,
                                              (hipStream_t)stream));
}

glv_status glv_rotate(glv_dtype dt, int64_t n, const void* const x[4], const void* const R[9], int64_t R_stride,
                      void* const y[4], void* stream) {
  const glv_status st = transform_args<9>(dt, n, x, R, R_stride, y);
  if (st != GLV_OK || n == 0) return st;
  return hip_status(glv::launch_transform(dt, glv::kTfRot3, n, x, R, R_stride, y, (hipStream_t)stream));
}

glv_status glv_rotate_bwd(glv_dtype dt, int64_t n, const void* const x[4], const void* const R[9],
                          int64_t R_stride, const void* const grad_y[4], void* const grad_x[4],
                          void* const grad_R[9], void* stream) {
  const glv_status st = transform_bwd_args<9, 9>(dt, n, x, R, R_stride, grad_y, grad_x, grad_R);
  if (st != GLV_OK || n == 0) return st;
  return hip_status(glv::launch_transform_bwd(dt, glv::kTfRot3, n, x, R, R_stride, grad_y, grad_x, grad_R,
                                              (hipStream_t)stream));
}

glv_status glv_rotate_axis_angle(glv_dtype dt, int64_t n, const void* const x[4], const void* const axis_angle[4],
                                 int64_t stride, void* const y[4], void* stream) {
  const glv_status st = transform_args<4>(dt, n, x, axis_angle, stride, y);
  if (st != GLV_OK || n == 0) return st;
  return hip_status(glv::launch_transform(dt, glv::kTfAxisAngle, n, x, axis_angle, stride, y, (hipStream_t)stream));
}

glv_status glv_rotate_axis_angle_bwd(glv_dtype dt, int64_t n, const void* const axis_angle[4], int64_t stride,
                                     const void* const grad_y[4], void* const grad_x[4], void* stream) {
  const glv_status st = transform_bwd_args<4, 9>(dt, n, nullptr, axis_angle, stride, grad_y, grad_x, nullptr);
  if (st != GLV_OK || n == 0) return st;
  return hip_status(glv::launch_transform_bwd(dt, glv::kTfAxisAngle, n, nullptr, axis_angle, stride, grad_y,
                                              grad_x, nullptr, (hipStream_t)stream));
}

glv_status glv_mass_histogram(glv_dtype dt, int64_t n, const void* m, double lo, double hi, int64_t n_bins,
                              unsigned long long* counts, void* stream) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (n < 0 || n_bins < 1) return GLV_EINVAL_SIZE;
  const double scale = (double)n_bins / (hi - lo);
  if (!(std::isfinite(lo) && std::isfinite(hi) && lo < hi && std::isfinite(scale) && scale > 0.0))
    return GLV_EINVAL_SIZE;
  if (n == 0) return GLV_OK;
  if (!m || !counts) return GLV_EINVAL_NULL;
  if (overlap(rng(counts, n_bins + 2, 8), rng(m, n, elem(dt)))) return GLV_EINVAL_ALIAS;
  return hip_status(glv::launch_histogram(dt, n, m, lo, hi, n_bins, counts, (hipStream_t)stream));
}

glv_status glv_event_best_pair(glv_dtype dt, int64_t ne, const int64_t* pair_offsets, const void* pair_m,
                               double target, int64_t* best_rank, void* best_m, void* stream) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (ne < 0) return GLV_EINVAL_SIZE;
  if (ne == 0) return GLV_OK;
  if (!pair_offsets || !pair_m || !best_rank || !best_m) return GLV_EINVAL_NULL;
  std::vector<Range> outs{rng(best_rank, ne, 8), rng(best_m, ne, elem(dt))};
  std::vector<Range> ins{rng(pair_offsets, ne + 1, 8)};
  if (any_overlap(outs, ins)) return GLV_EINVAL_ALIAS;
  return hip_status(glv::launch_best_pair(dt, ne, pair_offsets, pair_m, target, best_rank, best_m,
                                          (hipStream_t)stream));
}

glv_status glv_pair_offsets(int64_t ne, const int64_t* off, int64_t* po, void* stream) {
  if (ne < 0) return GLV_EINVAL_SIZE;
  if (!off || !po) return GLV_EINVAL_NULL;
  if (overlap(rng(off, ne + 1, 8), rng(po, ne + 1, 8))) return GLV_EINVAL_ALIAS;
  return hip_status(glv::launch_pair_offsets(ne, off, po, (hipStream_t)stream));
}

glv_status glv_validate_offsets(int64_t ne, const int64_t* off, int64_t np, long long* bad, void* stream) {
  if (ne < 0 || np < 0) return GLV_EINVAL_SIZE;
  if (!off || !bad) return GLV_EINVAL_NULL;
  if (overlap(rng(off, ne + 1, 8), rng(bad, 1, 8))) return GLV_EINVAL_ALIAS;
  return hip_status(glv::launch_validate_offsets(ne, off, np, bad, (hipStream_t)stream));
}

glv_status glv_event_reduce(glv_dtype dt, glv_coords co, glv_mode mode, int64_t ne, const int64_t* off,
                            const int64_t* poff, const void* const p[4], void* const total[4], void* em, void* pm,
                            unsigned long long* fallback, const glv_tiling* tiling, void* stream) {
  glv_status st = validate_event_reduce(dt, co, mode, ne, off, poff, p, total, em, pm);
  if (st != GLV_OK) return st;
  glv::Tiling t;
  st = resolve_tiling(dt, co, mode, tiling, false, &t);
  if (st != GLV_OK) return st;
  if (ne == 0 || (!total && !em && !pm)) return GLV_OK;
  return hip_status(
      glv::launch_event_reduce(dt, co, mode, ne, off, poff, p, total, em, pm, fallback, t, (hipStream_t)stream));
}

glv_status glv_event_reduce_best_pair(glv_dtype dt, glv_coords co, glv_mode mode, int64_t ne, const int64_t* off,
                                      const int64_t* poff, const void* const p[4], double target, int64_t* best_rank,
                                      void* best_m, unsigned long long* fallback, const glv_tiling* tiling,
                                      void* stream) {
  glv_status st = check_event_args(dt, co, mode, ne, off, p);
  if (st != GLV_OK || ne == 0) return st;
  if (!poff) return GLV_EINVAL_OFFSETS;
  if (!best_rank || !best_m) return GLV_EINVAL_NULL;
  std::vector<Range> outs{rng(best_rank, ne, 8), rng(best_m, ne, elem(dt))};
  std::vector<Range> ins{rng(off, ne + 1, 8), rng(poff, ne + 1, 8)};
  if (fallback) outs.push_back(rng(fallback, 1, 8));
  if (any_overlap(outs, ins)) return GLV_EINVAL_ALIAS;
  for (int k = 0; k < 4; ++k) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p[k]);
    for (const Range& r : outs)
      if (a >= r.lo && a < r.hi) return GLV_EINVAL_ALIAS;
  }
  glv::Tiling t;
  st = resolve_tiling(dt, co, mode, tiling, false, &t, true);
  if (st != GLV_OK) return st;
  const glv::BestOut b{best_rank, best_m, target};
  return hip_status(glv::launch_event_reduce(dt, co, mode, ne, off, poff, p, nullptr, nullptr, nullptr, fallback, t,
                                             (hipStream_t)stream, &b));
}

glv_status glv_invariant_mass_histogram(glv_dtype dt, glv_coords co, glv_mode mode, int64_t n, const void* const a[4],
                                        const void* const b[4], double lo, double hi, int64_t n_bins,
                                        unsigned long long* counts, unsigned long long* fallback, void* stream) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (!coords_ok(co)) return GLV_EINVAL_COORDS;
  glv_status ms = mode_ok(mode, co);
  if (ms != GLV_OK) return ms;
  if (n < 0 || n_bins < 1) return GLV_EINVAL_SIZE;
  const double scale = (double)n_bins / (hi - lo);
  if (!(std::isfinite(lo) && std::isfinite(hi) && lo < hi && std::isfinite(scale) && scale > 0.0))
    return GLV_EINVAL_SIZE;
  if (n == 0) return GLV_OK;
  if (!nonnull<4>(a) || !nonnull<4>(b) || !counts) return GLV_EINVAL_NULL;
  const size_t es = elem(dt);
  std::vector<Range> ins;
  for (int k = 0; k < 4; ++k) {
    ins.push_back(rng(a[k], n, es));
    ins.push_back(rng(b[k], n, es));
  }
  std::vector<Range> outs{rng(counts, n_bins + 2, 8)};
  if (fallback) outs.push_back(rng(fallback, 1, 8));
  if (any_overlap(outs, ins)) return GLV_EINVAL_ALIAS;
  return hip_status(glv::launch_mass_histogram(dt, co, mode, n, a, b, lo, hi, n_bins, counts, fallback,
                                               (hipStream_t)stream));
}

glv_status validate_event_reduce_bwd(glv_dtype dt, glv_coords co, int64_t ne, const int64_t* off,
                                     const int64_t* poff, const void* const p[4], const void* const gt[4],
                                     const void* gem, const void* gpair, void* const gp[4]) {
  glv_status st = check_event_args(dt, co, GLV_PLAIN, ne, off, p);
  if (st != GLV_OK || ne == 0) return st;
  if (!nonnull<4>((const void* const*)gp)) return GLV_EINVAL_NULL;
  if (gt && !nonnull<4>(gt)) return GLV_EINVAL_NULL;
  if (gpair && !poff) return GLV_EINVAL_OFFSETS;
  for (int k = 0; k < 4; ++k) {
    for (int j = 0; j < 4; ++j)
      if (gp[k] == p[j] || (j != k && gp[k] == gp[j])) return GLV_EINVAL_ALIAS;
    if (gp[k] == gpair || gp[k] == gem || (gt && gp[k] == gt[0])) return GLV_EINVAL_ALIAS;
    if (overlap(rng(off, ne + 1, 8), rng(gp[k], 1, elem(dt)))) return GLV_EINVAL_ALIAS;
  }
  return GLV_OK;
}

glv_status glv_event_reduce_bwd(glv_dtype dt, glv_coords co, int64_t ne, const int64_t* off, const int64_t* poff,
                                const void* const p[4], const void* const gt[4], const void* gem,
                                const void* gpair, void* const gp[4], const glv_tiling* tiling, void* stream) {
  glv_status st = validate_event_reduce_bwd(dt, co, ne, off, poff, p, gt, gem, gpair, gp);
  if (st != GLV_OK || ne == 0) return st;
  glv::Tiling t;
  st = resolve_tiling(dt, co, GLV_PLAIN, tiling, true, &t);
  if (st != GLV_OK) return st;
  if (ne == 0) return GLV_OK;
  return hip_status(
      glv::launch_event_reduce_bwd(dt, co, ne, off, poff, p, gt, gem, gpair, gp, t, (hipStream_t)stream));
}

glv_status glv_event_reduce_bwd_totals(glv_dtype dt, glv_coords co, int64_t ne, const int64_t* off,
                                       const int64_t* poff, const void* const p[4], const void* const tot[4],
                                       const void* const gt[4], const void* gem, const void* gpair,
                                       void* const gp[4], const glv_tiling* tiling, void* stream) {
  glv_status st = validate_event_reduce_bwd(dt, co, ne, off, poff, p, gt, gem, gpair, gp);
  if (st != GLV_OK || ne == 0) return st;
  if (!tot || !nonnull<4>(tot)) return GLV_EINVAL_NULL;
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 4; ++j)
      if (overlap(rng(tot[j], ne, elem(dt)), rng(gp[k], 1, elem(dt)))) return GLV_EINVAL_ALIAS;
  glv::Tiling t;
  st = resolve_tiling(dt, co, GLV_PLAIN, tiling, true, &t);
  if (st != GLV_OK) return st;
  return hip_status(glv::launch_event_reduce_bwd(dt, co, ne, off, poff, p, gt, gem, gpair, gp, t,
                                                 (hipStream_t)stream, gem ? tot : nullptr));
}

glv_status glv_current_tiling(glv_dtype dt, glv_coords co, glv_mode mode, glv_tiling* out) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (!coords_ok(co)) return GLV_EINVAL_COORDS;
  glv_status ms = mode_ok(mode, co);
  if (ms != GLV_OK) return ms;
  if (!out) return GLV_EINVAL_NULL;
  glv::Tiling t;
  glv_status st = resolve_tiling(dt, co, mode, nullptr, false, &t);
  if (st != GLV_OK) return st;
  write_tiling(t, out);
  return GLV_OK;
}

glv_status glv_current_tiling_bwd(glv_dtype dt, glv_coords co, glv_tiling* out) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (!coords_ok(co)) return GLV_EINVAL_COORDS;
  if (!out) return GLV_EINVAL_NULL;
  glv::Tiling t;
  glv_status st = resolve_tiling(dt, co, GLV_PLAIN, nullptr, true, &t);
  if (st != GLV_OK) return st;
  write_tiling(t, out);
  return GLV_OK;
}

glv_status glv_autotune_event_reduce(glv_dtype dt, glv_coords co, glv_mode mode, int64_t ne, const int64_t* off,
                                     const int64_t* poff, const void* const p[4], void* const total[4], void* em,
                                     void* pm, glv_tiling* best, void* stream) {
  glv_status st = validate_event_reduce(dt, co, mode, ne, off, poff, p, total, em, pm);
  if (st != GLV_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // candidates: workgroup size x events per tile x staged particles x pairs per round
  std::vector<glv::Tiling> cands;
  const int blocks[] = {64, 256};
  const int epbs[] = {16, 32, 64};
  const int caps[] = {64, 128, 256, 512};
  const int qcaps[] = {256, 512, 1024};
  for (int b : blocks)
    for (int e : epbs)
      for (int c : caps)
        for (int q : qcaps) {
          glv::Tiling t{b, e, c, q};
          if (tiling_valid(dt, mode, false, t)) cands.push_back(t);
        }
  auto launch = [&](const glv::Tiling& t) {
    return glv::launch_event_reduce(dt, co, mode, ne, off, poff, p, total, em, pm, nullptr, t, s);
  };
  const bool work = ne > 0 && (total || em || pm);
  return autotune_common(dt, co, mode, false, ne, off, cands, default_tiling(dt, mode), work, launch, best, s);
}

glv_status glv_autotune_event_reduce_bwd(glv_dtype dt, glv_coords co, int64_t ne, const int64_t* off,
                                         const int64_t* poff, const void* const p[4], const void* const gt[4],
                                         const void* gem, const void* gpair, void* const gp[4], glv_tiling* best,
                                         void* stream) {
  glv_status st = validate_event_reduce_bwd(dt, co, ne, off, poff, p, gt, gem, gpair, gp);
  if (st != GLV_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // candidates: workgroup size x events per tile x staged particles x staged pairs
  std::vector<glv::Tiling> cands;
  // one staged particle per thread: the staging capacity is the workgroup;
  // two or four staged pair upstreams per thread
  const int blocks[] = {64, 128, 256, 512};
  const int epbs[] = {16, 32, 64};
  const int per_thread[] = {2, 4};
  for (int b : blocks)
    for (int e : epbs)
      for (int k : per_thread) {
        glv::Tiling t{b, e, b, std::min(k * b, 4096)};
        if (tiling_valid(dt, GLV_PLAIN, true, t)) cands.push_back(t);
      }
  auto launch = [&](const glv::Tiling& t) {
    return glv::launch_event_reduce_bwd(dt, co, ne, off, poff, p, gt, gem, gpair, gp, t, s);
  };
  return autotune_common(dt, co, GLV_PLAIN, true, ne, off, cands, default_tiling_bwd(dt), ne > 0, launch, best, s);
}

glv_status glv_autotune_key(glv_dtype dt, glv_coords co, glv_mode mode, int32_t backward, int64_t ne,
                            const int64_t* off, char* buf, int64_t len, void* stream) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (!coords_ok(co)) return GLV_EINVAL_COORDS;
  glv_status ms = mode_ok(backward ? GLV_PLAIN : mode, co);
  if (ms != GLV_OK) return ms;
  if (ne < 0 || len < 1) return GLV_EINVAL_SIZE;
  if (!buf || (ne > 0 && !off)) return GLV_EINVAL_NULL;
  std::string key;
  const glv_status st = dataset_key(dt, co, mode, backward != 0, ne, off, (hipStream_t)stream, &key);
  if (st != GLV_OK) return st;
  if ((int64_t)key.size() + 1 > len) return GLV_EINVAL_SIZE;
  memcpy(buf, key.c_str(), key.size() + 1);
  return GLV_OK;
}

glv_status glv_autotune_lookup(glv_dtype dt, glv_coords co, glv_mode mode, int32_t backward, int64_t ne,
                               const int64_t* off, glv_tiling* out, int32_t* found, void* stream) {
  if (!dtype_ok(dt)) return GLV_EINVAL_DTYPE;
  if (!coords_ok(co)) return GLV_EINVAL_COORDS;
  const bool bwd = backward != 0;
  if (bwd) mode = GLV_PLAIN;
  glv_status ms = mode_ok(mode, co);
  if (ms != GLV_OK) return ms;
  if (ne < 0) return GLV_EINVAL_SIZE;
  if (ne > 0 && !off) return GLV_EINVAL_NULL;
  std::string key;
  glv_status st = dataset_key(dt, co, mode, bwd, ne, off, (hipStream_t)stream, &key);
  if (st != GLV_OK) return st;
  glv::Tiling t = bwd ? default_tiling_bwd(dt) : default_tiling(dt, mode);
  bool hit = glv::tune::lookup_process(key, &t);
  if (!hit) {
    const char* path = cache_path();
    if (!path) {
      fprintf(stderr, "glv: no autotuned tiling for %s (GLV_AUTOTUNE_CACHE not set); using the default\n",
              key.c_str());
    } else {
      glv::tune::Entries entries;
      const CacheFile cf = read_cache(path, dt, mode, bwd, &entries);
      for (const auto& e : entries) {
        if (e.first == key) {
          t = e.second;
          hit = true;
        }
      }
      if (!hit && cf == CacheFile::kUsable)
        fprintf(stderr, "glv: %s has no tiling for %s; using the default\n", path, key.c_str());
      if (!hit && cf == CacheFile::kMissing)
        fprintf(stderr, "glv: autotune cache %s does not exist; using the default tiling\n", path);
    }
    if (hit) glv::tune::remember_process(key, t);
  }
  remember_tiling(dt, co, bwd ? kBwdKey : (int)mode, t);
  if (out) write_tiling(t, out);
  if (found) *found = hit ? 1 : 0;
  return GLV_OK;
}

void glv_autotune_forget(void) {
  glv::tune::forget_process();
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tiles.clear();
}

}  // extern "C"
