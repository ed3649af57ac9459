/*
 * glv.h -- C ABI of the batched Lorentz-vector library for AMD Instinct MI355X
 * (gfx950).
 *
 * The library computes, over millions of independent items held as
 * structure-of-arrays (SoA) columns in GPU memory,
 *   - the invariant mass of pairs of 4-vectors given in any of three 4D
 *     coordinate systems (GenVectorX, arXiv 2312.02756, Sec. 4.1 and Fig. 1:
 *     m[i] = mass(v1[i] + v2[i]); coordinate systems Sec. 3.1),
 *   - the Lorentz boost of Cartesian 4-vectors (Sec. 4.1, ApplyBoost: a 4D
 *     Lorentz transformation held as a 4x4 matrix),
 *   - a per-event reduction over jagged (CSR) events: each event's total
 *     4-vector, its mass and the masses of all its particle pairs (the pair
 *     mass of Fig. 1 applied inside every event),
 * and the reverse-mode derivative (vector-Jacobian product, "_bwd") of each.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every data pointer is a DEVICE pointer owned by the caller.  The
 *   library never allocates, frees or copies between host and device, and
 *   never synchronises (except the glv_autotune_* calls, which time kernels
 *   and therefore waits for `stream`).  Each call validates its arguments on
 *   the host without reading device memory, enqueues its kernels on `stream`
 *   (a hipStream_t; NULL = the default stream) and returns.
 * Layout.  A 4-vector column set is four separate contiguous arrays, one per
 *   component, each of n elements of the call's dtype.  Component order:
 *     GLV_PXPYPZE   (px, py, pz, E)
 *     GLV_PTETAPHIM (pt, eta, phi, M)   E = sqrt((pt cosh eta)^2 + M^2)
 *     GLV_PTETAPHIE (pt, eta, phi, E)
 *     GLV_PXPYPZM   (px, py, pz, M)     E = sqrt(px^2 + py^2 + pz^2 + M^2)
 *   with px = pt cos(phi), py = pt sin(phi), pz = pt sinh(eta).  (Sec. 3.1
 *   leaves the coordinate system to the user; these are the four 4D systems
 *   of GenVector.)  Only M^2 enters, so the sign of a given M does not.
 * Sums are formed in Cartesian components, never converted back.
 * Mass.  q = E^2 - |P|^2; m = sqrt(q), and m = -sqrt(-q) for a spacelike
 *   q < 0 (values are not validated: NaN in gives NaN out, |beta| >= 1 gives
 *   inf/NaN).  The derivative of m is taken as 0 where m = 0.
 * Sizes are int64_t element counts; a negative count returns
 *   GLV_EINVAL_SIZE.  A count of 0 is valid, launches nothing and reads no
 *   pointer (they may be NULL), except that glv_pair_offsets still writes
 *   pair_offsets[0] and glv_validate_offsets still reads offsets[0].
 * Alignment.  Any element-aligned pointer is accepted; columns aligned to 16
 *   bytes take the vectorised path.
 * Errors.  A glv_status is returned; on GLV_EHIP the HIP error code is
 *   available from glv_last_hip_error() (per thread).  Nothing is enqueued
 *   when validation fails.
 */
#ifndef GLV_H
#define GLV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GLV_ABI_VERSION 2

typedef enum glv_status {
  GLV_OK = 0,
  GLV_EINVAL_NULL = 1,    /* a required pointer is NULL                        */
  GLV_EINVAL_SIZE = 2,    /* negative element or event count                   */
  GLV_EINVAL_DTYPE = 3,   /* dtype is not GLV_F32 / GLV_F64                    */
  GLV_EINVAL_COORDS = 4,  /* coords is not one of glv_coords                   */
  GLV_EINVAL_MODE = 5,    /* mode unknown, or not available for these coords  */
  GLV_EINVAL_ALIAS = 6,   /* an output overlaps an input (or another output)   */
  GLV_EINVAL_STRIDE = 7,  /* beta_stride not 0 or 1, or 0 where 1 is required  */
  GLV_EINVAL_OFFSETS = 8, /* offsets / pair_offsets missing where needed       */
  GLV_EINVAL_TILING = 9,  /* a glv_tiling field is outside its allowed set     */
  GLV_EHIP = 10           /* a HIP call failed (see glv_last_hip_error)        */
} glv_status;

typedef enum glv_dtype { GLV_F32 = 1, GLV_F64 = 2 } glv_dtype;

typedef enum glv_coords { GLV_PXPYPZE = 0, GLV_PTETAPHIM = 1, GLV_PTETAPHIE = 2, GLV_PXPYPZM = 3 } glv_coords;

/* GLV_PLAIN: the definition (convert, add, E^2 - |P|^2).
 * GLV_COMPENSATED (PtEtaPhiM only): the cancellation-free form
 *   m^2 = Ma^2 + Mb^2 + 2 (t1 + t2 + t3),
 *   t1 = 2 mTa mTb sinh^2(dy/2), t2 = 2 pta ptb sin^2(dphi/2),
 *   t3 = (pta^2 Mb^2 + ptb^2 Ma^2 + Ma^2 Mb^2) / (mTa mTb + pta ptb),
 * with mT = sqrt(pt^2 + M^2) and the rapidity difference
 *   dy = (eta_a - eta_b) + (delta_a - delta_b),
 *   delta = y - eta = -asinh(M^2 sinh(eta) / (mT (pt cosh(eta) + E))).
 * Every term is >= 0, so light, nearly collinear pairs keep their digits.
 * The azimuth difference is exact for azimuths in [-pi, pi] (the seam at
 * +-pi is reduced with a two-part pi); other azimuths are accepted, but the
 * rounding of their difference is not covered by the guarantee below.
 * In FP32 each item carries a running bound on the relative error of m^2;
 * an item whose bound exceeds 2^-18 is recomputed in FP64 from its widened
 * inputs and counted in *fallback_count.  In FP64 the same form is evaluated
 * throughout (no fallback). */
typedef enum glv_mode { GLV_PLAIN = 0, GLV_COMPENSATED = 1 } glv_mode;

/* Work decomposition of glv_event_reduce, glv_event_reduce_best_pair and
 * glv_event_reduce_bwd.  It changes
 * speed only: pair masses, totals and gradients of every event that fits the
 * tiling's staging capacity, and plain event masses, are identical for every
 * such tiling; the compensated event mass (a sum of per-pair terms, summed in
 * an order that follows the tiling) may differ in the last bit between
 * tilings but is reproducible for a given tiling.  An event that does not fit
 * goes to a second launch of the same call: its plain pair masses are the
 * same, its sums take another order, and a compensated pair mass may differ
 * in the last bit (that launch fuses the arithmetic differently, which can
 * also move a pair across the FP64-redo threshold); all stay within the
 * stated accuracy.
 * Forward (glv_event_reduce): every wavefront (64 threads) of a workgroup
 * works alone on its own tile of consecutive events.
 *   block            threads per workgroup: 64, 128, 256 or 512
 *   events_per_tile  events of one wavefront's tile: 1 .. 64
 *   lds_particles    particles a wavefront stages at once: 64 .. 4096
 *                    (larger events go to the second launch)
 *   pairs_per_round  a multiple of 64 in 64 .. 4096: pairs a wavefront
 *                    evaluates per round, each lane a run of consecutive
 *                    pairs.  FP64 masses pass through LDS in rounds of 64 m
 *                    pairs, m the largest odd number <= pairs_per_round / 64;
 *                    the FP32 plain mode takes a chunk's pairs in one round;
 *                    the compensated mode and glv_event_reduce_best_pair
 *                    take rounds of pairs_per_round
 * Backward (glv_event_reduce_bwd): a workgroup takes tiles of
 * events_per_tile consecutive events and stages at most one particle per
 * thread.
 *   block, events_per_tile   as for the forward
 *   lds_particles    particles staged at once, clamped to block
 *   pairs_per_round  pair upstreams staged at once, a multiple of 64 in
 *                    64 .. 4096 (events with more pairs, or more particles
 *                    than the staging capacity, go to the second launch)
 * Fields set to 0 take the library's current choice (the autotuned one if
 * glv_autotune_event_reduce, or glv_autotune_event_reduce_bwd for the
 * backward, ran for this device/dtype/coords/mode, otherwise a built-in
 * default).  A tiling whose workgroup would need more than 64 KiB of LDS is
 * rejected with GLV_EINVAL_TILING: per wavefront the forward keeps 4 values
 * per staged particle (12 in the compensated mode), per pair of a round one
 * value in FP64 (none in FP32), 8 more bytes in the compensated mode, one
 * value and 4 bytes for glv_event_reduce_best_pair (instead of the FP64
 * value), and 12 bytes per event of the tile; per workgroup the backward
 * keeps 4 values and 2 bytes per staged particle, one value per staged pair
 * upstream (plus 2), and 4.5 values and 32 bytes per event of the tile. */
typedef struct glv_tiling {
  int32_t block;
  int32_t events_per_tile;
  int32_t lds_particles;
  int32_t pairs_per_round;
} glv_tiling;

/* Pair invariant mass (Sec. 4.1, Fig. 1): m[i] = mass(conv(a_i) + conv(b_i)),
 * i in [0, n).
 *   a, b            4 column pointers each (component order of `coords`)
 *   m               n outputs; must not overlap any input
 *   fallback_count  device uint64; if not NULL and mode is GLV_COMPENSATED with
 *                   GLV_F32, the number of items recomputed in FP64 is ADDED to
 *                   it (the caller zeroes it).  Ignored otherwise.
 * GLV_COMPENSATED requires GLV_PTETAPHIM (else GLV_EINVAL_MODE). */
glv_status glv_invariant_mass(glv_dtype dtype, glv_coords coords, glv_mode mode, int64_t n,
                              const void* const a[4], const void* const b[4], void* m,
                              unsigned long long* fallback_count, void* stream);

/* Reverse mode of the pair mass (plain definition; any coords):
 *   grad_a[k][i] = grad_m[i] * dm_i / d a_k[i], grad_b likewise.
 * With (P, E) the summed vector, dm/d(Cartesian leg) = (-P, E) / |m|, chained
 * through the conversion's Jacobian.  Gradient columns must not overlap any
 * input or each other. */
glv_status glv_invariant_mass_bwd(glv_dtype dtype, glv_coords coords, int64_t n,
                                  const void* const a[4], const void* const b[4],
                                  const void* grad_m, void* const grad_a[4], void* const grad_b[4],
                                  void* stream);

/* Reverse mode of the cancellation-free pair mass (the GLV_COMPENSATED form,
 * PtEtaPhiM legs only; not in the paper): the same gradients as
 * glv_invariant_mass_bwd, computed from K = E_a E_b - p_a.p_b written as
 * mTa mTb cosh(dy) - pta ptb cos(dphi) and its derivatives, so that nearly
 * collinear light pairs keep their digits in FP32 (the plain form subtracts
 * E dE from P.dp).  m dm = Ma dMa + Mb dMb + dK with, for leg a (leg b with
 * dy and dphi negated), dK/dpta = (pta mTb/mTa) 2 sinh^2(dy/2) + ptb 2
 * sin^2(dphi/2) + (pta^2 Mb^2 - ptb^2 Ma^2)/((pta mTb + ptb mTa) mTa) + mTa
 * mTb sinh(dy) dya/dpta, dK/detaa = mTa mTb sinh(dy) pta cosh(etaa)/Ea,
 * dK/dphia = pta ptb sin(dphi), dK/dMa = (Ma/mTa) mTb cosh(dy) + mTa mTb
 * sinh(dy) dya/dMa.  No FP64 redo.  Zero where m = 0; a leg with pt = M = 0
 * gets zero rows.  Arguments, aliasing and errors as glv_invariant_mass_bwd
 * (no coords argument). */
glv_status glv_invariant_mass_comp_bwd(glv_dtype dtype, int64_t n, const void* const a[4], const void* const b[4],
                                       const void* grad_m, void* const grad_a[4], void* const grad_b[4],
                                       void* stream);

/* Active Lorentz boost (Sec. 4.1, ApplyBoost) of Cartesian vectors x by
 * velocity beta: with g = 1/sqrt(1 - beta^2), k = g^2/(1 + g), s = beta.p,
 *   E' = g (E + s),   p' = p + (k s + g E) beta.
 *   x, y        4 columns (px, py, pz, E); y may equal x column for column
 *               (in place); any other overlap is GLV_EINVAL_ALIAS
 *   beta        3 columns (bx, by, bz)
 *   beta_stride 1: n velocities, one per item; 0: beta[k][0] for every item
 * In FP32, g and k are formed in FP64 from the widened velocity. */
glv_status glv_boost(glv_dtype dtype, int64_t n, const void* const x[4], const void* const beta[3],
                     int64_t beta_stride, void* const y[4], void* stream);

/* Reverse mode of the boost, y = L(beta) x:
 *   grad_x = L(beta) grad_y        (L is symmetric),
 *   grad_beta = gE [g^3 (E + s) beta + g p]
 *             + (gp.beta) [k' g^3 s beta + k p + g^3 E beta] + (k s + g E) gp,
 *   k' = g (g + 2)/(1 + g)^2, grad_y = (gp, gE).
 * grad_beta may be NULL (not wanted); if given, beta_stride must be 1
 * (GLV_EINVAL_STRIDE otherwise).  Outputs must not overlap inputs. */
glv_status glv_boost_bwd(glv_dtype dtype, int64_t n, const void* const x[4],
                         const void* const beta[3], int64_t beta_stride,
                         const void* const grad_y[4], void* const grad_x[4],
                         void* const grad_beta[3], void* stream);

/* Coordinate conversion (Sec. 3.1: a 4D vector in any of its systems):
 * out = the `to` coordinates of the vectors in[] given in `from`, through
 * their Cartesian components (from == to copies):
 *   to PxPyPzE    the conversions above;
 *   to PtEtaPhiM  pt = hypot(px, py), eta = asinh(pz / pt), phi = atan2(py, px)
 *                 in [-pi, pi], M = the mass of the vector with the pair mass's
 *                 sign convention (-sqrt(-q) when spacelike);
 *   to PtEtaPhiE  the same with E;
 *   to PxPyPzM    px, py, pz and that M.
 * On the beam axis (pt = 0) eta is +inf or -inf by the sign of pz, 0 when
 * pz = 0.  in and out are 4 columns of n elements; out may be in itself
 * (column for column), otherwise no output overlaps an input or another
 * output (GLV_EINVAL_ALIAS).  Errors: GLV_EINVAL_DTYPE, _COORDS, _SIZE (n <
 * 0), _NULL. */
glv_status glv_convert(glv_dtype dtype, glv_coords from, glv_coords to, int64_t n, const void* const in[4],
                       void* const out[4], void* stream);

/* Reverse mode of glv_convert: grad_in = (d out / d in)^T grad_out per item
 * (the Cartesian gradient of the target coordinates, chained through the
 * source conversion's Jacobian; from == to copies).  On the beam axis the pt,
 * eta and phi rows of the inverse are taken as zero; the M row is zero where
 * M = 0.  grad_in may be grad_out itself (column for column); otherwise no
 * output overlaps an input or another output. */
glv_status glv_convert_bwd(glv_dtype dtype, glv_coords from, glv_coords to, int64_t n,
                           const void* const in[4], const void* const grad_out[4], void* const grad_in[4],
                           void* stream);

/* General Lorentz transformation (Sec. 3.1: Lorentz transformations, such
 * as LorentzRotation, held as a 4x4 matrix; Sec. 4.1: ApplyBoost applies
 * one): y = L x per item on Cartesian vectors x = (px, py, pz, E), with
 * y_r = sum_c L[4r + c] x_c.  L holds 16 column pointers in row-major order:
 * L_stride 1 = one matrix per item (each column n elements), 0 = one matrix
 * for all items (each pointer at one element).  L is not checked to be a
 * Lorentz transformation: any 4x4 matrix is applied.  y may be x itself
 * (column for column); otherwise no output overlaps an input or another
 * output (GLV_EINVAL_ALIAS).  Errors: GLV_EINVAL_DTYPE, _SIZE, _STRIDE
 * (L_stride not 0 or 1), _NULL. */
glv_status glv_lorentz_transform(glv_dtype dtype, int64_t n, const void* const x[4], const void* const L[16],
                                 int64_t L_stride, void* const y[4], void* stream);

/* Reverse mode: grad_x = L^T grad_y; grad_L (NULL = not wanted) receives the
 * per-item gradient grad_L[4r + c] = grad_y_r x_c and needs L_stride 1
 * (GLV_EINVAL_STRIDE otherwise) and x; x may be NULL without grad_L.  No
 * output overlaps an input or another output. */
glv_status glv_lorentz_transform_bwd(glv_dtype dtype, int64_t n, const void* const x[4], const void* const L[16],
                                     int64_t L_stride, const void* const grad_y[4], void* const grad_x[4],
                                     void* const grad_L[16], void* stream);

/* Rotation3D (Sec. 3.1: a rotation held as a 3x3 matrix) applied to the
 * spatial part of Cartesian vectors: (px, py, pz)' = R (px, py, pz), E' = E,
 * R in 9 row-major column pointers with R_stride as L_stride above (R is not
 * checked to be orthogonal).  Aliasing and errors as glv_lorentz_transform. */
glv_status glv_rotate(glv_dtype dtype, int64_t n, const void* const x[4], const void* const R[9], int64_t R_stride,
                      void* const y[4], void* stream);

/* Reverse mode: grad_p = R^T grad_p', grad_E = grad_E'; grad_R (NULL = not
 * wanted; R_stride 1 and x needed) receives grad_R[3r + c] = grad_p'_r p_c. */
glv_status glv_rotate_bwd(glv_dtype dtype, int64_t n, const void* const x[4], const void* const R[9],
                          int64_t R_stride, const void* const grad_y[4], void* const grad_x[4],
                          void* const grad_R[9], void* stream);

/* AxisAngle (Sec. 3.1: the same rotation held as an axis and an angle):
 * axis_angle = (ax, ay, az, angle in radians) columns, per item (stride 1)
 * or one for all (stride 0).  The axis is normalised, u = a/|a|, and the
 * spatial part rotated by Rodrigues' formula
 * R = cos(t) I + sin(t) [u]x + (1 - cos(t)) u u^T; a zero axis gives the
 * identity; E' = E.  Aliasing and errors as glv_lorentz_transform. */
glv_status glv_rotate_axis_angle(glv_dtype dtype, int64_t n, const void* const x[4],
                                 const void* const axis_angle[4], int64_t stride, void* const y[4], void* stream);

/* Reverse mode with respect to the vectors: grad_p = R^T grad_p' (the
 * rotation by the opposite angle), grad_E = grad_E'.  The gradient with
 * respect to the axis and angle is not provided.  grad_x overlaps no input. */
glv_status glv_rotate_axis_angle_bwd(glv_dtype dtype, int64_t n, const void* const axis_angle[4], int64_t stride,
                                     const void* const grad_y[4], void* const grad_x[4], void* stream);

/* Histogram of masses (the analysis step after the mass; not in the paper,
 * whose Sec. 6 places GenVector inside ROOT, which analyses such data):
 * n values m (dtype) into n_bins equal bins of [lo, hi).  counts holds
 * n_bins + 2 uint64 and the call ADDS to it (clear it first for one
 * histogram): counts[0] = values below lo, counts[n_bins + 1] = values at or
 * above hi, counts[1 + b] with b = floor((v - lo) * (n_bins / (hi - lo)))
 * evaluated in binary64 (b clamped to n_bins - 1); NaN is not counted.
 * Errors: GLV_EINVAL_DTYPE; _SIZE (n < 0, n_bins < 1, lo or hi not finite,
 * lo >= hi, or n_bins / (hi - lo) not finite); _NULL; _ALIAS (counts
 * overlaps m). */
glv_status glv_mass_histogram(glv_dtype dtype, int64_t n, const void* m, double lo, double hi, int64_t n_bins,
                              unsigned long long* counts, void* stream);

/* Per CSR event, its pair whose mass lies closest to `target` (the analysis
 * step after the jagged reduction; not in the paper): pair_offsets from
 * glv_pair_offsets and pair_m as glv_event_reduce writes them (lexicographic
 * i < j within each event; trusted, like the offsets there).  best_rank[e]
 * (int64) = the rank within the event of the pair with the smallest
 * |m - target| in binary64, the lowest rank among equal distances, NaN
 * masses never chosen; -1 and a NaN best_m[e] (dtype) for an event without
 * such a pair.  The outputs overlap neither each other nor pair_offsets
 * (GLV_EINVAL_ALIAS) nor, unchecked, pair_m.  Errors: GLV_EINVAL_DTYPE,
 * _SIZE (n_events < 0), _NULL. */
glv_status glv_event_best_pair(glv_dtype dtype, int64_t n_events, const int64_t* pair_offsets, const void* pair_m,
                               double target, int64_t* best_rank, void* best_m, void* stream);

/* The per-event best pair of glv_event_best_pair chosen inside the jagged
 * reduction, without writing pair masses (the analysis step fused into the
 * reduction; not in the paper, whose Sec. 6 places GenVector inside ROOT).
 * The pair masses are bitwise those glv_event_reduce writes for the same
 * arguments and tiling; best_rank[e] (int64) and best_m[e] (dtype) follow
 * glv_event_best_pair's rule (smallest |m - target| in binary64, lowest rank
 * among equal distances, NaN masses never chosen, -1 and NaN for an event
 * without a chosen pair).
 *   offsets, pair_offsets (required), p, tiling, fallback_count
 *                 as in glv_event_reduce; fields set to 0 take this
 *                 call's built-in default (64, 64, 128, 1024), not the
 *                 autotuned choice of glv_event_reduce
 * The outputs must not overlap each other, the offsets or the particle
 * columns (GLV_EINVAL_ALIAS).  Errors as glv_event_reduce, and
 * GLV_EINVAL_OFFSETS without pair_offsets. */
glv_status glv_event_reduce_best_pair(glv_dtype dtype, glv_coords coords, glv_mode mode, int64_t n_events,
                                      const int64_t* offsets, const int64_t* pair_offsets, const void* const p[4],
                                      double target, int64_t* best_rank, void* best_m,
                                      unsigned long long* fallback_count, const glv_tiling* tiling, void* stream);

/* Pair masses binned into glv_mass_histogram's bins as they are computed,
 * never stored (the histogram of the analysis step fused into the mass
 * kernel; not in the paper): the masses are bitwise those glv_invariant_mass
 * writes for the same dtype, coords, mode and legs, and each is counted as
 * glv_mass_histogram counts a value (the call ADDS to counts, n_bins + 2
 * uint64; NaN not counted).  fallback_count as in glv_invariant_mass.
 * Errors: those of glv_invariant_mass for the legs and of
 * glv_mass_histogram for the bins; counts must not overlap a leg column
 * (GLV_EINVAL_ALIAS). */
glv_status glv_invariant_mass_histogram(glv_dtype dtype, glv_coords coords, glv_mode mode, int64_t n,
                                        const void* const a[4], const void* const b[4], double lo, double hi,
                                        int64_t n_bins, unsigned long long* counts,
                                        unsigned long long* fallback_count, void* stream);

/* Pair offsets of CSR events: pair_offsets[0] = 0,
 * pair_offsets[e+1] = pair_offsets[e] + c_e (c_e - 1) / 2 with
 * c_e = offsets[e+1] - offsets[e].  Both arrays hold n_events + 1 int64. */
glv_status glv_pair_offsets(int64_t n_events, const int64_t* offsets, int64_t* pair_offsets,
                            void* stream);

/* Per-event reduction of CSR events.  Two launches on `stream`: the main one
 * reduces every event that fits the tiling's staging capacity; a short
 * second one scans the offsets for larger events (and, in the FP32
 * GLV_COMPENSATED mode, for events the first marked for the FP64 redo) and
 * reduces those from global memory.
 *   offsets       n_events + 1 int64, offsets[0] = 0, non-decreasing
 *                 (trusted: see glv_validate_offsets)
 *   pair_offsets  from glv_pair_offsets; required when pair_m or a
 *                 GLV_COMPENSATED event mass is requested
 *   p             4 particle columns in `coords`, offsets[n_events] entries
 * Outputs (each may be NULL = not wanted):
 *   total[4]  per-event sum of the particles' Cartesian vectors: four sums of
 *             the particles whose index in the event is r mod 4, each in index
 *             order, combined as ((P0 + P1) + (P2 + P3)); events beyond the
 *             staging capacity by a fixed-tree workgroup sum
 *   event_m   mass of the total: GLV_PLAIN from total; GLV_COMPENSATED as
 *             m^2 = sum_i M_i^2 + 2 sum_{i<j} (E_i E_j - p_i.p_j) with each pair
 *             product from the cancellation-free form
 *   pair_m    masses of the pairs i < j of each event, at
 *             pair_offsets[e] + i (2n - i - 1)/2 + (j - i - 1)
 *   fallback_count  as in glv_invariant_mass (pairs recomputed in FP64)
 *   tiling    NULL or a glv_tiling (fields 0 = library's choice) */
glv_status glv_event_reduce(glv_dtype dtype, glv_coords coords, glv_mode mode, int64_t n_events,
                            const int64_t* offsets, const int64_t* pair_offsets,
                            const void* const p[4], void* const total[4], void* event_m,
                            void* pair_m, unsigned long long* fallback_count,
                            const glv_tiling* tiling, void* stream);

/* Reverse mode of the plain per-event reduction.  For particle i of event e,
 *   g_i = grad_total[e] + grad_event_m[e] dm(V_e)/dV
 *       + sum_{j != i} grad_pair_m[pair(i, j)] dm(v_i + v_j)/dv,
 * chained to the particle's coordinates.  Any upstream pointer may be NULL
 * (zero); grad_total is all-or-nothing (4 columns or NULL).  grad_p[4] must
 * not overlap inputs. */
glv_status glv_event_reduce_bwd(glv_dtype dtype, glv_coords coords, int64_t n_events,
                                const int64_t* offsets, const int64_t* pair_offsets,
                                const void* const p[4], const void* const grad_total[4],
                                const void* grad_event_m, const void* grad_pair_m,
                                void* const grad_p[4], const glv_tiling* tiling, void* stream);

/* The same reverse mode given the forward's event totals (not in the paper):
 * total[4] holds each event's total 4-vector as glv_event_reduce wrote it for
 * these particles, in dtype, n_events entries per column, so that the
 * event-mass term g_m dm(V)/dV takes V from it instead of summing the event's
 * particles again -- for a caller that kept the forward's outputs.  The
 * forward sums an event in the same order and
 * precision as the backward would, so the result is bitwise that of
 * glv_event_reduce_bwd wherever both staged the event (an event beyond the
 * staging capacity of either is summed in another order).  total is read
 * only when grad_event_m is given; it must be 4 non-NULL columns (else
 * GLV_EINVAL_NULL) that do not overlap grad_p (GLV_EINVAL_ALIAS).  All other
 * arguments and errors as in glv_event_reduce_bwd. */
glv_status glv_event_reduce_bwd_totals(glv_dtype dtype, glv_coords coords, int64_t n_events,
                                       const int64_t* offsets, const int64_t* pair_offsets,
                                       const void* const p[4], const void* const total[4],
                                       const void* const grad_total[4], const void* grad_event_m,
                                       const void* grad_pair_m, void* const grad_p[4],
                                       const glv_tiling* tiling, void* stream);

/* Debug helper: counts violations of offsets[0] = 0, offsets non-decreasing,
 * offsets[n_events] = n_particles, and ADDS the count to *bad_count (device
 * int64, zeroed by the caller).  Asynchronous like every other call. */
glv_status glv_validate_offsets(int64_t n_events, const int64_t* offsets, int64_t n_particles,
                                long long* bad_count, void* stream);

/* Autotuning of the jagged reduction (not in the paper: its data are arrays
 * of particles of varying size, Sec. 5.1).  The best tiling depends on the
 * device and on the distribution of event sizes, so a tuned choice is kept
 * under a key made of the device architecture, dtype, coordinate system,
 * direction (forward with its mode, or backward) and a signature of the
 * dataset: the order of magnitude of the event count and the share of events
 * in each size class (0, then [2^(b-1), 2^b)), in 5 % steps, over all events
 * or, beyond 65,536 events, over 32 evenly spread runs of 2,048 consecutive
 * events (copied to the host: the autotuning calls synchronise `stream`).
 *
 * Persistent cache: if the environment variable GLV_AUTOTUNE_CACHE names a
 * file, choices are read from and added to it, as JSON:
 *   {"format": "glv-autotune-1", "entries": [
 *     {"key": "<key>", "tiling": [block, events_per_tile, lds_particles,
 *                                 pairs_per_round]}, ...]}
 * A missing file is created.  A file that is not exactly this (or holds a
 * tiling outside the allowed sets) is corrupt: it is reported on stderr,
 * ignored and never rewritten, and the call goes on as without a file. */

/* Tiling choice for a forward dataset: the one of this process's earlier
 * choices or of the cache file under this dataset's key; otherwise times
 * candidate tilings (workgroup size x events per tile x staged particles x
 * pairs per round) on the caller's data -- the arguments are those of
 * glv_event_reduce, outputs included, which end up holding a valid result --
 * keeps the fastest under the key (and in the cache file).  The choice becomes
 * this process's current one for (device, dtype, coords, mode) and is written
 * to *best if not NULL.  Synchronises `stream`. */
glv_status glv_autotune_event_reduce(glv_dtype dtype, glv_coords coords, glv_mode mode,
                                     int64_t n_events, const int64_t* offsets,
                                     const int64_t* pair_offsets, const void* const p[4],
                                     void* const total[4], void* event_m, void* pair_m,
                                     glv_tiling* best, void* stream);

/* The tiling glv_event_reduce would use for these arguments (the current
 * choice or the default), written to *out. */
glv_status glv_current_tiling(glv_dtype dtype, glv_coords coords, glv_mode mode, glv_tiling* out);

/* The same for glv_event_reduce_bwd, with its arguments (grad_p ends up
 * holding a valid result); the choice becomes the current backward one for
 * (device, dtype, coords).  Synchronises `stream`. */
glv_status glv_autotune_event_reduce_bwd(glv_dtype dtype, glv_coords coords, int64_t n_events,
                                         const int64_t* offsets, const int64_t* pair_offsets,
                                         const void* const p[4], const void* const grad_total[4],
                                         const void* grad_event_m, const void* grad_pair_m,
                                         void* const grad_p[4], glv_tiling* best, void* stream);

/* The tiling glv_event_reduce_bwd would use (the current backward choice or
 * the default), written to *out. */
glv_status glv_current_tiling_bwd(glv_dtype dtype, glv_coords coords, glv_tiling* out);

/* The cache key of a dataset (NUL-terminated, into buf of len bytes;
 * GLV_EINVAL_SIZE if it does not fit).  backward = 0: the forward in `mode`;
 * 1: the backward (mode ignored).  n_events = 0 needs no offsets and no GPU.
 * Synchronises `stream` when it reads offsets. */
glv_status glv_autotune_key(glv_dtype dtype, glv_coords coords, glv_mode mode, int32_t backward,
                            int64_t n_events, const int64_t* offsets, char* buf, int64_t len,
                            void* stream);

/* Tiling choice without timing, for callers that must not time kernels
 * (serving loops): looks the dataset's key up in this process's choices and
 * in the cache file.  Found: *found = 1.  Not found -- no such entry, no
 * GLV_AUTOTUNE_CACHE, a missing or a corrupt file -- *found = 0, the
 * built-in default, a warning on stderr, and still GLV_OK.  Either way the
 * result becomes the current choice (as glv_autotune_event_reduce /
 * glv_autotune_event_reduce_bwd would make it) and is written to *out if not
 * NULL.  Synchronises `stream` when it reads offsets (n_events > 0). */
glv_status glv_autotune_lookup(glv_dtype dtype, glv_coords coords, glv_mode mode, int32_t backward,
                               int64_t n_events, const int64_t* offsets, glv_tiling* out, int32_t* found,
                               void* stream);

/* Forgets this process's tuned choices (the cache file is left as it is):
 * afterwards the calls above consult the cache file again and the current
 * choices are the defaults. */
void glv_autotune_forget(void);

const char* glv_status_str(glv_status s);
int glv_abi_version(void);
int glv_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GLV_H */
