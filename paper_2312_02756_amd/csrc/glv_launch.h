// Host-side launchers of the gfx950 kernels.  Called by the C ABI after the
// arguments have been validated; each enqueues on `s` and returns the first
// HIP error seen (hipSuccess otherwise).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "glv.h"

namespace glv {

hipError_t launch_mass(glv_dtype dt, glv_coords co, glv_mode mode, int64_t n, const void* const a[4],
                       const void* const b[4], void* m, unsigned long long* fallback, hipStream_t s);

hipError_t launch_mass_bwd(glv_dtype dt, glv_coords co, int64_t n, const void* const a[4],
                           const void* const b[4], const void* gm, void* const ga[4],
                           void* const gb[4], hipStream_t s);

// Pair masses binned into a histogram (added to counts[n_bins + 2]) as they
// are computed, without storing them.
hipError_t launch_mass_histogram(glv_dtype dt, glv_coords co, glv_mode mode, int64_t n, const void* const a[4],
                                 const void* const b[4], double lo, double hi, int64_t n_bins,
                                 unsigned long long* counts, unsigned long long* fallback, hipStream_t s);

// Reverse mode of the cancellation-free (compensated) pair mass, PtEtaPhiM legs.
hipError_t launch_mass_comp_bwd(glv_dtype dt, int64_t n, const void* const a[4], const void* const b[4],
                                const void* gm, void* const ga[4], void* const gb[4], hipStream_t s);

hipError_t launch_boost(glv_dtype dt, int64_t n, const void* const x[4], const void* const beta[3],
                        int64_t beta_stride, void* const y[4], hipStream_t s);

hipError_t launch_boost_bwd(glv_dtype dt, int64_t n, const void* const x[4],
                            const void* const beta[3], int64_t beta_stride,
                            const void* const gy[4], void* const gx[4], void* const gbeta[3],
                            hipStream_t s);

hipError_t launch_convert(glv_dtype dt, glv_coords from, glv_coords to, int64_t n, const void* const in[4],
                          void* const out[4], hipStream_t s);

hipError_t launch_convert_bwd(glv_dtype dt, glv_coords from, glv_coords to, int64_t n, const void* const in[4],
                              const void* const gout[4], void* const gin[4], hipStream_t s);

// General transformations: a 4x4 Lorentz matrix (16 parameter columns), a
// 3x3 rotation matrix (9) or an axis and an angle (4), per item (stride 1)
// or one for all items (stride 0).  The reverse mode's matrix gradient (gm,
// NULL = not wanted) exists for the two matrix kinds at stride 1.
enum { kTfLorentz = 0, kTfRot3 = 1, kTfAxisAngle = 2 };

hipError_t launch_transform(glv_dtype dt, int kind, int64_t n, const void* const x[4], const void* const* m,
                            int64_t m_stride, void* const y[4], hipStream_t s);

hipError_t launch_transform_bwd(glv_dtype dt, int kind, int64_t n, const void* const x[4], const void* const* m,
                                int64_t m_stride, const void* const gy[4], void* const gx[4], void* const* gm,
                                hipStream_t s);

// Histogram of n masses into n_bins equal bins of [lo, hi) plus under- and
// overflow, added to counts[n_bins + 2].
hipError_t launch_histogram(glv_dtype dt, int64_t n, const void* m, double lo, double hi, int64_t n_bins,
                            unsigned long long* counts, hipStream_t s);

// Per event, the rank and mass of its pair closest to target.
hipError_t launch_best_pair(glv_dtype dt, int64_t n_events, const int64_t* pair_offsets, const void* pair_m,
                            double target, int64_t* rank, void* best_m, hipStream_t s);

hipError_t launch_pair_offsets(int64_t n_events, const int64_t* offsets, int64_t* pair_offsets,
                               hipStream_t s);

hipError_t launch_validate_offsets(int64_t n_events, const int64_t* offsets, int64_t n_particles,
                                   long long* bad, hipStream_t s);

// Largest workgroup of the jagged kernels (their register budget is sized
// for it: 512 threads leave up to 256 VGPRs per lane).
constexpr int kMaxBlock = 512;

// Tiling with every field resolved (non-zero, inside its allowed set).
struct Tiling {
  int block;
  int events_per_tile;
  int lds_particles;
  int pairs_per_round;  // forward: pairs a wavefront evaluates per round (the backward ignores it)
};

// LDS bytes one workgroup of the forward reduction needs for a tiling (with
// the fused best-pair selection if `best`).
size_t event_reduce_lds_bytes(glv_dtype dt, glv_mode mode, const Tiling& t, bool best = false);
size_t event_reduce_bwd_lds_bytes(glv_dtype dt, const Tiling& t);

// Outputs of the fused per-event best-pair selection.
struct BestOut {
  int64_t* rank;
  void* mass;
  double target;
};

// With `best`, the per-event best pair instead of pair masses (pair_m is
// then ignored).
hipError_t launch_event_reduce(glv_dtype dt, glv_coords co, glv_mode mode, int64_t n_events,
                               const int64_t* offsets, const int64_t* pair_offsets,
                               const void* const p[4], void* const total[4], void* event_m,
                               void* pair_m, unsigned long long* fallback, const Tiling& t,
                               hipStream_t s, const BestOut* best = nullptr);

hipError_t launch_event_reduce_bwd(glv_dtype dt, glv_coords co, int64_t n_events,
                                   const int64_t* offsets, const int64_t* pair_offsets,
                                   const void* const p[4], const void* const gt[4],
                                   const void* gem, const void* gpair, void* const gp[4],
                                   const Tiling& t, hipStream_t s, const void* const tot[4] = nullptr);

}  // namespace glv
