/*
 * glv_oracle.c -- CPU oracle for batched Lorentz-vector kernels.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg load the shared library built from it.  It shares no
 * source with the GPU path.
 *
 * Plain C11, compiled with -ffp-contract=off -fno-fast-math: every formula
 * is evaluated as written, left to right, in binary64; the "_q" entry points
 * repeat the definitions in binary128 (libquadmath) for brute-force pinning.
 * Loops over independent items are split across OpenMP threads; no loop is
 * blocked, fused or reordered.
 *
 * Paper: GenVectorX (arXiv 2312.02756).
 *   Sec. 3.1   coordinate systems of a 4D vector (Cartesian, polar-like),
 *              templated on the scalar type.
 *   Sec. 4.1   InvariantMasses: mass of the sum of two 4-vectors given in any
 *              4D coordinate system; ApplyBoost: a 4D Lorentz transformation
 *              held as a 4x4 matrix, applied to an array of vectors.
 *   Fig. 1/2   the pair-mass kernel: each work item adds the two vectors at
 *              its index and stores the mass of that sum.
 * The reverse-mode derivatives, the cancellation-free pair mass and the
 * per-event (jagged) reduction are not in the paper; each function below says
 * what it is derived from.
 *
 * Readings of points the paper leaves open:
 *   - conversions are the standard collider definitions:
 *       px = pt cos(phi), py = pt sin(phi), pz = pt sinh(eta),
 *       E  = sqrt((pt cosh(eta))^2 + M^2)      (PtEtaPhiM), E given (PtEtaPhiE);
 *   - a spacelike sum (E^2 - |p|^2 = q < 0) has mass -sqrt(-q);
 *   - the gradient of the mass is zero where m = 0;
 *   - the boost is active: E' = gamma (E + beta.p).
 *
 * parity pinned: every entry point is checked in the CPU test-suite against
 * closed forms, invariants, binary128 brute force and finite differences.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_PXPYPZE = 0, ORC_PTETAPHIM = 1, ORC_PTETAPHIE = 2, ORC_PXPYPZM = 3 };
enum { ORC_PLAIN = 0, ORC_ACCURATE = 1 };

typedef __float128 quad;

/* ---------------------------------------------------------------- threads */

void orc_set_threads(int k) {
#ifdef _OPENMP
  if (k > 0) omp_set_num_threads(k);
#else
  (void)k;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------- conversion */

/* Cartesian (px, py, pz, E) of one vector given in `coords` (Sec. 3.1, 4.1);
 * PxPyPzM has E = sqrt(|p|^2 + M^2). */
static void cart(int coords, double c0, double c1, double c2, double c3, double v[4]) {
  if (coords == ORC_PXPYPZE || coords == ORC_PXPYPZM) {
    v[0] = c0;
    v[1] = c1;
    v[2] = c2;
    v[3] = (coords == ORC_PXPYPZE) ? c3 : sqrt(c0 * c0 + c1 * c1 + c2 * c2 + c3 * c3);
    return;
  }
  double pt = c0, eta = c1, phi = c2;
  v[0] = pt * cos(phi);
  v[1] = pt * sin(phi);
  v[2] = pt * sinh(eta);
  if (coords == ORC_PTETAPHIM) {
    double pc = pt * cosh(eta);
    v[3] = sqrt(pc * pc + c3 * c3);
  } else {
    v[3] = c3;
  }
}

static void cart_q(int coords, double c0, double c1, double c2, double c3, quad v[4]) {
  if (coords == ORC_PXPYPZE || coords == ORC_PXPYPZM) {
    v[0] = c0;
    v[1] = c1;
    v[2] = c2;
    if (coords == ORC_PXPYPZE) {
      v[3] = c3;
    } else {
      quad x = c0, y = c1, z = c2, mm = c3;
      v[3] = sqrtq(x * x + y * y + z * z + mm * mm);
    }
    return;
  }
  quad pt = c0, eta = c1, phi = c2;
  v[0] = pt * cosq(phi);
  v[1] = pt * sinq(phi);
  v[2] = pt * sinhq(eta);
  if (coords == ORC_PTETAPHIM) {
    quad pc = pt * coshq(eta);
    quad mm = c3;
    v[3] = sqrtq(pc * pc + mm * mm);
  } else {
    v[3] = c3;
  }
}

/* Array form of `cart`, for pinning the conversion on its own. */
void orc_to_cartesian(int coords, int64_t n, const double* c0, const double* c1, const double* c2,
                      const double* c3, double* px, double* py, double* pz, double* e) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double v[4];
    cart(coords, c0[i], c1[i], c2[i], c3[i], v);
    px[i] = v[0];
    py[i] = v[1];
    pz[i] = v[2];
    e[i] = v[3];
  }
}

/* --------------------------------------------------------------- the mass */

/* Mass of a Cartesian 4-vector: q = E^2 - px^2 - py^2 - pz^2 (left to right);
 * m = sqrt(q), or -sqrt(-q) for a spacelike vector. */
static double mass_of(const double w[4]) {
  double q = w[3] * w[3] - w[0] * w[0] - w[1] * w[1] - w[2] * w[2];
  return q >= 0.0 ? sqrt(q) : -sqrt(-q);
}

static quad mass_of_q(const quad w[4]) {
  quad q = w[3] * w[3] - w[0] * w[0] - w[1] * w[1] - w[2] * w[2];
  return q >= 0 ? sqrtq(q) : -sqrtq(-q);
}

/* Pair invariant mass, the definition (Sec. 4.1, Fig. 1): convert both legs,
 * add them, take the mass of the sum.  If `scale` is not NULL it receives
 * S = E^2 + px^2 + py^2 + pz^2 of the sum, the size of the terms that cancel
 * in q (used by tests to state rounding tolerances). */
void orc_mass_plain(int coords, int64_t n, const double* a0, const double* a1, const double* a2,
                    const double* a3, const double* b0, const double* b1, const double* b2,
                    const double* b3, double* m, double* scale) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double va[4], vb[4], w[4];
    cart(coords, a0[i], a1[i], a2[i], a3[i], va);
    cart(coords, b0[i], b1[i], b2[i], b3[i], vb);
    for (int k = 0; k < 4; ++k) w[k] = va[k] + vb[k];
    m[i] = mass_of(w);
    if (scale) scale[i] = w[3] * w[3] + w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  }
}

/* The same definition in binary128, rounded to binary64 at the end.  If
 * `m_lo` is not NULL it receives the rounding remainder, so m + m_lo carries
 * the binary128 result to about 106 bits (for finite differences). */
void orc_mass_plain_q(int coords, int64_t n, const double* a0, const double* a1, const double* a2,
                      const double* a3, const double* b0, const double* b1, const double* b2,
                      const double* b3, double* m, double* m_lo) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    quad va[4], vb[4], w[4];
    cart_q(coords, a0[i], a1[i], a2[i], a3[i], va);
    cart_q(coords, b0[i], b1[i], b2[i], b3[i], vb);
    for (int k = 0; k < 4; ++k) w[k] = va[k] + vb[k];
    quad r = mass_of_q(w);
    m[i] = (double)r;
    if (m_lo) m_lo[i] = (double)(r - (quad)m[i]);
  }
}

/* ------------------------------------------------- cancellation-free mass */

/* Angle difference a - b reduced to (-pi, pi].  pi is split into a double
 * head and a tail; near the seam the head is subtracted from each angle
 * separately (both subtractions are exact), so a difference close to +-2 pi
 * keeps its small remainder exactly. */
static double dphi_reduced(double a, double b) {
  const double pi_hi = 3.141592653589793116;      /* double nearest pi */
  const double pi_lo = 1.2246467991473532e-16;    /* pi - pi_hi */
  double d = a - b;
  if (d > pi_hi) return ((a - pi_hi) - (b + pi_hi)) - 2.0 * pi_lo;
  if (d <= -pi_hi) return ((a + pi_hi) - (b - pi_hi)) + 2.0 * pi_lo;
  return d;
}

/* Per-leg terms of the cancellation-free form: M^2, mT = sqrt(pt^2 + M^2)
 * and delta = y - eta, the rapidity minus the pseudorapidity.
 *
 * Derivation (not in the paper): sinh(y) = (pt/mT) sinh(eta).  With
 * asinh(u) - asinh(v) = asinh(u sqrt(1+v^2) - v sqrt(1+u^2)) and
 * pt^2 - mT^2 = -M^2 this gives
 *     delta = -asinh( M^2 sinh(eta) / (mT (pt cosh(eta) + E)) ),
 * a quotient of positive terms, so delta keeps full relative accuracy. */
static void leg_terms(double pt, double eta, double mass, double* m2, double* mt, double* delta) {
  double mm = mass * mass;
  double t = sqrt(pt * pt + mm);
  double sh = sinh(eta), ch = cosh(eta);
  double pc = pt * ch;
  double e = sqrt(pc * pc + mm);
  *m2 = mm;
  *mt = t;
  *delta = (t > 0.0) ? -asinh(mm * sh / (t * (pc + e))) : 0.0;
}

/* Pair mass of two PtEtaPhiM legs in a form with no cancellation.
 *
 * With rapidities y and transverse masses mT,
 *   E_a E_b - p_a.p_b = mT_a mT_b cosh(y_a - y_b) - pt_a pt_b cos(phi_a - phi_b),
 * and writing cosh x = 1 + 2 sinh^2(x/2), cos x = 1 - 2 sin^2(x/2):
 *   m^2 = M_a^2 + M_b^2 + 2 (t1 + t2 + t3),
 *   t1 = 2 mT_a mT_b sinh^2(dy/2),  dy = (eta_a - eta_b) + (delta_a - delta_b),
 *   t2 = 2 pt_a pt_b sin^2(dphi/2),
 *   t3 = mT_a mT_b - pt_a pt_b
 *      = (pt_a^2 M_b^2 + pt_b^2 M_a^2 + M_a^2 M_b^2) / (mT_a mT_b + pt_a pt_b).
 * Every term is >= 0.  It reaches the same value as the definition (up to
 * rounding); it is the reference for the accurate and compensated modes.
 * If `kterm` is not NULL it receives t1 + t2 + t3 (= E_a E_b - p_a.p_b). */
static double mass_acc_pair(double pta, double etaa, double phia, double ma, double ptb,
                            double etab, double phib, double mb, double* kterm) {
  double m2a, mta, da, m2b, mtb, db;
  leg_terms(pta, etaa, ma, &m2a, &mta, &da);
  leg_terms(ptb, etab, mb, &m2b, &mtb, &db);
  double dy = (etaa - etab) + (da - db);
  double s1 = sinh(0.5 * dy);
  double t1 = 2.0 * mta * mtb * (s1 * s1);
  double s2 = sin(0.5 * dphi_reduced(phia, phib));
  double t2 = 2.0 * pta * ptb * (s2 * s2);
  double num = pta * pta * m2b + ptb * ptb * m2a + m2a * m2b;
  double den = mta * mtb + pta * ptb;
  double t3 = (num == 0.0) ? 0.0 : num / den;
  double k = t1 + t2 + t3;
  if (kterm) *kterm = k;
  return sqrt(m2a + m2b + 2.0 * k);
}

void orc_mass_accurate(int64_t n, const double* a0, const double* a1, const double* a2,
                       const double* a3, const double* b0, const double* b1, const double* b2,
                       const double* b3, double* m) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    m[i] = mass_acc_pair(a0[i], a1[i], a2[i], a3[i], b0[i], b1[i], b2[i], b3[i], NULL);
}

/* ----------------------------------------------------------------- boost */

/* Active Lorentz boost by velocity beta (Sec. 4.1, ApplyBoost).  In (E, p)
 * order the matrix is [[g, g b^T], [g b, I + k b b^T]] with g = 1/sqrt(1-b^2)
 * and k = (g - 1)/b^2 = g^2/(1 + g):
 *   E' = g (E + b.p),   p' = p + (k (b.p) + g E) b.
 * beta_stride 1: one velocity per item; 0: one velocity for all items. */
void orc_boost(int64_t n, const double* x0, const double* x1, const double* x2, const double* x3,
               const double* bx, const double* by, const double* bz, int64_t beta_stride,
               double* y0, double* y1, double* y2, double* y3) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = i * beta_stride;
    double b[3] = {bx[j], by[j], bz[j]};
    double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    double g = 1.0 / sqrt(1.0 - b2);
    double k = g * g / (1.0 + g);
    double px = x0[i], py = x1[i], pz = x2[i], e = x3[i];
    double s = b[0] * px + b[1] * py + b[2] * pz;
    double c = k * s + g * e;
    y3[i] = g * (e + s);
    y0[i] = px + c * b[0];
    y1[i] = py + c * b[1];
    y2[i] = pz + c * b[2];
  }
}

/* The boost in binary128.  If `lo` is not NULL, lo[0..3] receive the
 * remainders of rounding each output to binary64 (as in orc_mass_plain_q). */
void orc_boost_q(int64_t n, const double* x0, const double* x1, const double* x2, const double* x3,
                 const double* bx, const double* by, const double* bz, int64_t beta_stride,
                 double* y0, double* y1, double* y2, double* y3, double* const* lo) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = i * beta_stride;
    quad b[3] = {bx[j], by[j], bz[j]};
    quad b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    quad g = 1 / sqrtq(1 - b2);
    quad k = g * g / (1 + g);
    quad px = x0[i], py = x1[i], pz = x2[i], e = x3[i];
    quad s = b[0] * px + b[1] * py + b[2] * pz;
    quad c = k * s + g * e;
    quad r[4] = {px + c * b[0], py + c * b[1], pz + c * b[2], g * (e + s)};
    double* y[4] = {y0, y1, y2, y3};
    for (int d = 0; d < 4; ++d) {
      y[d][i] = (double)r[d];
      if (lo) lo[d][i] = (double)(r[d] - (quad)y[d][i]);
    }
  }
}

/* Componentwise size of the boost's terms, (|L| |x|)_i with |L| the matrix
 * of absolute values: the scale for rounding tolerances of a boosted vector. */
void orc_boost_scale(int64_t n, const double* x0, const double* x1, const double* x2,
                     const double* x3, const double* bx, const double* by, const double* bz,
                     int64_t beta_stride, double* s0, double* s1, double* s2, double* s3) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = i * beta_stride;
    double b[3] = {fabs(bx[j]), fabs(by[j]), fabs(bz[j])};
    double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    double g = 1.0 / sqrt(1.0 - b2);
    double k = g * g / (1.0 + g);
    double px = fabs(x0[i]), py = fabs(x1[i]), pz = fabs(x2[i]), e = fabs(x3[i]);
    double s = b[0] * px + b[1] * py + b[2] * pz;
    double c = k * s + g * e;
    s3[i] = g * (e + s);
    s0[i] = px + c * b[0];
    s1[i] = py + c * b[1];
    s2[i] = pz + c * b[2];
  }
}

/* ---------------------------------------------- conversion, either way */

/* Coordinates `coords` of a Cartesian 4-vector v = (px, py, pz, E), the
 * inverse of `cart` (Sec. 3.1: any system of a 4D vector): pt = hypot(px, py),
 * eta = asinh(pz / pt), phi = atan2(py, px), and M = the mass of v with the
 * pair mass's sign convention (-sqrt(-q) for a spacelike v), or E itself;
 * PxPyPzM keeps (px, py, pz) and takes that M.
 * On the beam axis (pt = 0) eta is +-inf by the sign of pz, 0 when pz = 0. */
static void coords_of(int coords, const double v[4], double c[4]) {
  if (coords == ORC_PXPYPZE || coords == ORC_PXPYPZM) {
    for (int k = 0; k < 3; ++k) c[k] = v[k];
    c[3] = (coords == ORC_PXPYPZE) ? v[3] : mass_of(v);
    return;
  }
  double pt = hypot(v[0], v[1]);
  c[0] = pt;
  if (pt > 0.0)
    c[1] = asinh(v[2] / pt);
  else
    c[1] = (v[2] > 0.0) ? INFINITY : ((v[2] < 0.0) ? -INFINITY : 0.0);
  c[2] = atan2(v[1], v[0]);
  c[3] = (coords == ORC_PTETAPHIM) ? mass_of(v) : v[3];
}

/* Conversion of n vectors from system `from` to system `to`: through the
 * Cartesian components, except that from == to copies. */
void orc_convert(int from, int to, int64_t n, const double* i0, const double* i1, const double* i2,
                 const double* i3, double* o0, double* o1, double* o2, double* o3) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double c[4];
    if (from == to) {
      c[0] = i0[i];
      c[1] = i1[i];
      c[2] = i2[i];
      c[3] = i3[i];
    } else {
      double v[4];
      cart(from, i0[i], i1[i], i2[i], i3[i], v);
      coords_of(to, v, c);
    }
    o0[i] = c[0];
    o1[i] = c[1];
    o2[i] = c[2];
    o3[i] = c[3];
  }
}

/* ------------------------------------------------------------- gradients */

/* d m / d (Cartesian sum) = (-Px, -Py, -Pz, E) / |m|, zero where m = 0.
 * (From m^2 = E^2 - |P|^2; for the spacelike convention m = -sqrt(-q) the
 * derivative dm/dq is again 1/(2|m|).) */
static void dmass_dcart(const double w[4], double m, double u[4]) {
  double am = fabs(m);
  if (am == 0.0) {
    u[0] = u[1] = u[2] = u[3] = 0.0;
    return;
  }
  u[0] = -w[0] / am;
  u[1] = -w[1] / am;
  u[2] = -w[2] / am;
  u[3] = w[3] / am;
}

/* Chain a Cartesian gradient u = dL/d(px,py,pz,E) of one vector back to its
 * own coordinates (the Jacobian of the conversion in `cart`). */
static void chain_coords(int coords, double c0, double c1, double c2, double c3, const double u[4],
                         double g[4]) {
  if (coords == ORC_PXPYPZE) {
    for (int k = 0; k < 4; ++k) g[k] = u[k];
    return;
  }
  if (coords == ORC_PXPYPZM) {
    /* E = sqrt(|p|^2 + M^2): dE/dp_k = p_k/E, dE/dM = M/E */
    double e = sqrt(c0 * c0 + c1 * c1 + c2 * c2 + c3 * c3);
    double ue = (e > 0.0) ? u[3] / e : 0.0;
    g[0] = u[0] + ue * c0;
    g[1] = u[1] + ue * c1;
    g[2] = u[2] + ue * c2;
    g[3] = ue * c3;
    return;
  }
  double pt = c0, eta = c1, phi = c2;
  double cp = cos(phi), sp = sin(phi), sh = sinh(eta), ch = cosh(eta);
  double px = pt * cp, py = pt * sp;
  if (coords == ORC_PTETAPHIM) {
    double pc = pt * ch;
    double e = sqrt(pc * pc + c3 * c3);
    /* dE/dpt = pt cosh^2(eta)/E, dE/deta = pt^2 sinh cosh / E, dE/dM = M/E */
    double de_dpt = (e > 0.0) ? pt * ch * ch / e : 0.0;
    double de_deta = (e > 0.0) ? pt * pt * sh * ch / e : 0.0;
    double de_dm = (e > 0.0) ? c3 / e : 0.0;
    g[0] = u[0] * cp + u[1] * sp + u[2] * sh + u[3] * de_dpt;
    g[1] = u[2] * pt * ch + u[3] * de_deta;
    g[2] = -u[0] * py + u[1] * px;
    g[3] = u[3] * de_dm;
  } else {
    g[0] = u[0] * cp + u[1] * sp + u[2] * sh;
    g[1] = u[2] * pt * ch;
    g[2] = -u[0] * py + u[1] * px;
    g[3] = u[3];
  }
}

/* Cartesian gradient u = (d c / d v)^T gc of c = coords_of(coords, v):
 *   d pt  = (px, py, 0, 0) / pt
 *   d eta = (-pz px / (pt^2 p), -pz py / (pt^2 p), 1 / p, 0),  p = |(px, py, pz)|
 *          (eta = asinh(pz / pt) and d asinh(x) = dx / sqrt(1 + x^2))
 *   d phi = (-py, px, 0, 0) / pt^2
 *   d M   = (-px, -py, -pz, E) / |M|   (zero where M = 0), or d E = (0, 0, 0, 1).
 * On the beam axis (pt = 0) the pt, eta and phi rows are taken as zero.
 * PxPyPzM: the identity rows of px, py, pz and the M row above. */
static void dcoords_dcart(int coords, const double v[4], const double gc[4], double u[4]) {
  if (coords == ORC_PXPYPZE) {
    for (int k = 0; k < 4; ++k) u[k] = gc[k];
    return;
  }
  if (coords == ORC_PXPYPZM) {
    double dm[4];
    dmass_dcart(v, mass_of(v), dm);
    for (int k = 0; k < 4; ++k) u[k] = (k < 3 ? gc[k] : 0.0) + gc[3] * dm[k];
    return;
  }
  for (int k = 0; k < 4; ++k) u[k] = 0.0;
  double pt = hypot(v[0], v[1]);
  if (pt > 0.0) {
    double p = sqrt(pt * pt + v[2] * v[2]);
    u[0] += gc[0] * v[0] / pt;
    u[1] += gc[0] * v[1] / pt;
    u[0] += gc[1] * (-v[2] * v[0] / (pt * pt * p));
    u[1] += gc[1] * (-v[2] * v[1] / (pt * pt * p));
    u[2] += gc[1] / p;
    u[0] += gc[2] * (-v[1] / (pt * pt));
    u[1] += gc[2] * (v[0] / (pt * pt));
  }
  if (coords == ORC_PTETAPHIM) {
    double dm[4];
    dmass_dcart(v, mass_of(v), dm);
    for (int k = 0; k < 4; ++k) u[k] += gc[3] * dm[k];
  } else {
    u[3] += gc[3];
  }
}

/* Reverse-mode derivative of orc_convert: g_in = (d out / d in)^T g_out, the
 * Cartesian gradient of the target coordinates chained back through the
 * source conversion; from == to passes g_out through. */
void orc_convert_vjp(int from, int to, int64_t n, const double* i0, const double* i1, const double* i2,
                     const double* i3, const double* g0, const double* g1, const double* g2, const double* g3,
                     double* r0, double* r1, double* r2, double* r3) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double gc[4] = {g0[i], g1[i], g2[i], g3[i]}, g[4];
    if (from == to) {
      for (int k = 0; k < 4; ++k) g[k] = gc[k];
    } else {
      double v[4], u[4];
      cart(from, i0[i], i1[i], i2[i], i3[i], v);
      dcoords_dcart(to, v, gc, u);
      chain_coords(from, i0[i], i1[i], i2[i], i3[i], u, g);
    }
    r0[i] = g[0];
    r1[i] = g[1];
    r2[i] = g[2];
    r3[i] = g[3];
  }
}

/* Reverse-mode derivative (vector-Jacobian product) of the pair mass:
 * grad_a = gm * dm/d(leg a coords), grad_b likewise.  Derived from the
 * definition of Fig. 1 by the chain rule; not in the paper. */
void orc_mass_vjp(int coords, int64_t n, const double* a0, const double* a1, const double* a2,
                  const double* a3, const double* b0, const double* b1, const double* b2,
                  const double* b3, const double* gm, double* ga0, double* ga1, double* ga2,
                  double* ga3, double* gb0, double* gb1, double* gb2, double* gb3) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double va[4], vb[4], w[4], u[4], g[4];
    cart(coords, a0[i], a1[i], a2[i], a3[i], va);
    cart(coords, b0[i], b1[i], b2[i], b3[i], vb);
    for (int k = 0; k < 4; ++k) w[k] = va[k] + vb[k];
    double m = mass_of(w);
    dmass_dcart(w, m, u);
    for (int k = 0; k < 4; ++k) u[k] *= gm[i];
    chain_coords(coords, a0[i], a1[i], a2[i], a3[i], u, g);
    ga0[i] = g[0];
    ga1[i] = g[1];
    ga2[i] = g[2];
    ga3[i] = g[3];
    chain_coords(coords, b0[i], b1[i], b2[i], b3[i], u, g);
    gb0[i] = g[0];
    gb1[i] = g[1];
    gb2[i] = g[2];
    gb3[i] = g[3];
  }
}

/* Rounding scale of the pair-mass VJP: the same chain rule with every factor
 * replaced by its absolute value, |gm| sum_k |u_k| |d v_k / d c|, u = (-P, E)/|m|.
 * The terms of one gradient component can cancel (the eta component subtracts
 * P.dp/deta from E dE/deta), so its rounding error is a few ulps of this sum,
 * not of the result. */
static void chain_coords_abs(int coords, double c0, double c1, double c2, double c3, const double u[4],
                             double g[4]) {
  if (coords == ORC_PXPYPZE) {
    for (int k = 0; k < 4; ++k) g[k] = fabs(u[k]);
    return;
  }
  if (coords == ORC_PXPYPZM) {
    double e = sqrt(c0 * c0 + c1 * c1 + c2 * c2 + c3 * c3);
    double ue = (e > 0.0) ? fabs(u[3]) / e : 0.0;
    g[0] = fabs(u[0]) + ue * fabs(c0);
    g[1] = fabs(u[1]) + ue * fabs(c1);
    g[2] = fabs(u[2]) + ue * fabs(c2);
    g[3] = ue * fabs(c3);
    return;
  }
  double pt = fabs(c0), eta = c1, phi = c2;
  double cp = fabs(cos(phi)), sp = fabs(sin(phi)), sh = fabs(sinh(eta)), ch = cosh(eta);
  double au[4] = {fabs(u[0]), fabs(u[1]), fabs(u[2]), fabs(u[3])};
  g[0] = au[0] * cp + au[1] * sp + au[2] * sh;
  g[1] = au[2] * pt * ch;
  g[2] = au[0] * pt * sp + au[1] * pt * cp;
  g[3] = 0.0;
  if (coords == ORC_PTETAPHIM) {
    double pc = pt * ch;
    double e = sqrt(pc * pc + c3 * c3);
    if (e > 0.0) {
      g[0] += au[3] * pt * ch * ch / e;
      g[1] += au[3] * pt * pt * sh * ch / e;
      g[3] = au[3] * fabs(c3) / e;
    }
  } else {
    g[3] = au[3];
  }
}

void orc_mass_vjp_scale(int coords, int64_t n, const double* a0, const double* a1, const double* a2,
                        const double* a3, const double* b0, const double* b1, const double* b2,
                        const double* b3, const double* gm, double* ga0, double* ga1, double* ga2,
                        double* ga3, double* gb0, double* gb1, double* gb2, double* gb3) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double va[4], vb[4], w[4], u[4], g[4];
    cart(coords, a0[i], a1[i], a2[i], a3[i], va);
    cart(coords, b0[i], b1[i], b2[i], b3[i], vb);
    for (int k = 0; k < 4; ++k) w[k] = va[k] + vb[k];
    double m = mass_of(w);
    dmass_dcart(w, m, u);
    for (int k = 0; k < 4; ++k) u[k] *= fabs(gm[i]);
    chain_coords_abs(coords, a0[i], a1[i], a2[i], a3[i], u, g);
    ga0[i] = g[0];
    ga1[i] = g[1];
    ga2[i] = g[2];
    ga3[i] = g[3];
    chain_coords_abs(coords, b0[i], b1[i], b2[i], b3[i], u, g);
    gb0[i] = g[0];
    gb1[i] = g[1];
    gb2[i] = g[2];
    gb3[i] = g[3];
  }
}

/* Reverse-mode derivative of the boost y = L(beta) x (per-item beta).
 *   grad_x = L(beta)^T gy = L(beta) gy   (L is symmetric);
 *   grad_beta from dg/dbeta = g^3 beta and dk/dbeta = k' g^3 beta with
 *   k' = dk/dg = g (g + 2) / (1 + g)^2:
 *     grad_beta = gE [g^3 (E + s) beta + g p]
 *               + (gp.beta) [k' g^3 s beta + k p + g^3 E beta] + (k s + g E) gp,
 *   s = beta.p, gy = (gp, gE).  Derived by hand; not in the paper. */
void orc_boost_vjp(int64_t n, const double* x0, const double* x1, const double* x2,
                   const double* x3, const double* bx, const double* by, const double* bz,
                   const double* gy0, const double* gy1, const double* gy2, const double* gy3,
                   double* gx0, double* gx1, double* gx2, double* gx3, double* gbx, double* gby,
                   double* gbz) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double b[3] = {bx[i], by[i], bz[i]};
    double p[3] = {x0[i], x1[i], x2[i]};
    double e = x3[i];
    double gp[3] = {gy0[i], gy1[i], gy2[i]};
    double ge = gy3[i];
    double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    double g = 1.0 / sqrt(1.0 - b2);
    double k = g * g / (1.0 + g);
    double kp = g * (g + 2.0) / ((1.0 + g) * (1.0 + g));
    double g3 = g * g * g;
    double s = b[0] * p[0] + b[1] * p[1] + b[2] * p[2];
    double gb = gp[0] * b[0] + gp[1] * b[1] + gp[2] * b[2];
    /* grad_x: the forward boost applied to (gp, gE) */
    double c = k * gb + g * ge;
    gx3[i] = g * (ge + gb);
    gx0[i] = gp[0] + c * b[0];
    gx1[i] = gp[1] + c * b[1];
    gx2[i] = gp[2] + c * b[2];
    double ce = g3 * (e + s);
    double cq = kp * g3 * s + g3 * e;
    double cr = k * s + g * e;
    double out[3];
    for (int d = 0; d < 3; ++d)
      out[d] = ge * (ce * b[d] + g * p[d]) + gb * (cq * b[d] + k * p[d]) + cr * gp[d];
    gbx[i] = out[0];
    gby[i] = out[1];
    gbz[i] = out[2];
  }
}

/* ------------------------------------------------------- jagged events */

/* Pair offsets of CSR events: exclusive prefix sum of n_e (n_e - 1) / 2,
 * n_events + 1 entries.  Pairs of one event are stored in lexicographic
 * order of (i, j), i < j. */
void orc_pair_offsets(int64_t n_events, const int64_t* offsets, int64_t* pair_offsets) {
  int64_t acc = 0;
  pair_offsets[0] = 0;
  for (int64_t e = 0; e < n_events; ++e) {
    int64_t c = offsets[e + 1] - offsets[e];
    acc += c * (c - 1) / 2;
    pair_offsets[e + 1] = acc;
  }
}

/* Per-event reduction of CSR events (the pair mass of Fig. 1 applied inside
 * each event, plus the event's total 4-vector and its mass).
 *   total[e]  = sum of the event's Cartesian vectors, in CSR order;
 *   event_m   = mass of total[e] (ORC_PLAIN), or for ORC_ACCURATE
 *               m^2 = sum_i M_i^2 + 2 sum_{i<j} (E_i E_j - p_i.p_j), the
 *               pair products taken from the cancellation-free form;
 *   pair_m    = pair masses of i < j at pair_offsets[e] + rank(i, j), plain
 *               or cancellation-free.
 * ORC_ACCURATE requires PtEtaPhiM.  Any output may be NULL. */
void orc_event_reduce(int coords, int mode, int64_t n_events, const int64_t* offsets,
                      const int64_t* pair_offsets, const double* p0, const double* p1,
                      const double* p2, const double* p3, double* t0, double* t1, double* t2,
                      double* t3, double* event_m, double* pair_m) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t e = 0; e < n_events; ++e) {
    int64_t lo = offsets[e], hi = offsets[e + 1];
    double tot[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = lo; i < hi; ++i) {
      double v[4];
      cart(coords, p0[i], p1[i], p2[i], p3[i], v);
      for (int k = 0; k < 4; ++k) tot[k] += v[k];
    }
    if (t0) {
      t0[e] = tot[0];
      t1[e] = tot[1];
      t2[e] = tot[2];
      t3[e] = tot[3];
    }
    double ksum = 0.0, msum = 0.0;
    int64_t out = pair_offsets ? pair_offsets[e] : 0;
    for (int64_t i = lo; i < hi; ++i) {
      if (mode == ORC_ACCURATE) msum += p3[i] * p3[i];
      for (int64_t j = i + 1; j < hi; ++j) {
        double mij;
        if (mode == ORC_ACCURATE) {
          double kij;
          mij = mass_acc_pair(p0[i], p1[i], p2[i], p3[i], p0[j], p1[j], p2[j], p3[j], &kij);
          ksum += kij;
        } else {
          double va[4], vb[4], w[4];
          cart(coords, p0[i], p1[i], p2[i], p3[i], va);
          cart(coords, p0[j], p1[j], p2[j], p3[j], vb);
          for (int k = 0; k < 4; ++k) w[k] = va[k] + vb[k];
          mij = mass_of(w);
        }
        if (pair_m) pair_m[out] = mij;
        ++out;
      }
    }
    if (event_m) {
      if (mode == ORC_ACCURATE)
        event_m[e] = sqrt(msum + 2.0 * ksum);
      else
        event_m[e] = mass_of(tot);
    }
  }
}

/* Totals and event masses in binary128 (plain definition), for pinning. */
void orc_event_reduce_q(int coords, int64_t n_events, const int64_t* offsets, const double* p0,
                        const double* p1, const double* p2, const double* p3, double* t0,
                        double* t1, double* t2, double* t3, double* event_m) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t e = 0; e < n_events; ++e) {
    quad tot[4] = {0, 0, 0, 0};
    for (int64_t i = offsets[e]; i < offsets[e + 1]; ++i) {
      quad v[4];
      cart_q(coords, p0[i], p1[i], p2[i], p3[i], v);
      for (int k = 0; k < 4; ++k) tot[k] += v[k];
    }
    t0[e] = (double)tot[0];
    t1[e] = (double)tot[1];
    t2[e] = (double)tot[2];
    t3[e] = (double)tot[3];
    event_m[e] = (double)mass_of_q(tot);
  }
}

/* Reverse-mode derivative of the plain per-event reduction.  For particle i
 * of event e, in Cartesian components,
 *   g_i = g_total + g_em dm(V)/dV + sum_{j != i} g_ij dm(v_i + v_j)/d(v),
 * then chained to the particle's own coordinates.  Any upstream pointer may
 * be NULL (zero).  Derived by the chain rule; not in the paper. */
void orc_event_reduce_vjp(int coords, int64_t n_events, const int64_t* offsets,
                          const int64_t* pair_offsets, const double* p0, const double* p1,
                          const double* p2, const double* p3, const double* gt0,
                          const double* gt1, const double* gt2, const double* gt3,
                          const double* g_em, const double* g_pair, double* gp0, double* gp1,
                          double* gp2, double* gp3) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t e = 0; e < n_events; ++e) {
    int64_t lo = offsets[e], hi = offsets[e + 1], n = hi - lo;
    double tot[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = lo; i < hi; ++i) {
      double v[4];
      cart(coords, p0[i], p1[i], p2[i], p3[i], v);
      for (int k = 0; k < 4; ++k) tot[k] += v[k];
    }
    double ut[4] = {0.0, 0.0, 0.0, 0.0};
    if (g_em) {
      dmass_dcart(tot, mass_of(tot), ut);
      for (int k = 0; k < 4; ++k) ut[k] *= g_em[e];
    }
    for (int64_t i = lo; i < hi; ++i) {
      double vi[4], u[4], g[4];
      cart(coords, p0[i], p1[i], p2[i], p3[i], vi);
      u[0] = gt0 ? gt0[e] : 0.0;
      u[1] = gt1 ? gt1[e] : 0.0;
      u[2] = gt2 ? gt2[e] : 0.0;
      u[3] = gt3 ? gt3[e] : 0.0;
      for (int k = 0; k < 4; ++k) u[k] += ut[k];
      if (g_pair) {
        int64_t a = i - lo;
        for (int64_t j = lo; j < hi; ++j) {
          if (j == i) continue;
          int64_t b = j - lo;
          int64_t r = a < b ? a : b, c = a < b ? b : a;
          int64_t rank = r * (2 * n - r - 1) / 2 + (c - r - 1);
          double gij = g_pair[pair_offsets[e] + rank];
          double vj[4], w[4], uw[4];
          cart(coords, p0[j], p1[j], p2[j], p3[j], vj);
          for (int k = 0; k < 4; ++k) w[k] = vi[k] + vj[k];
          dmass_dcart(w, mass_of(w), uw);
          for (int k = 0; k < 4; ++k) u[k] += gij * uw[k];
        }
      }
      chain_coords(coords, p0[i], p1[i], p2[i], p3[i], u, g);
      gp0[i] = g[0];
      gp1[i] = g[1];
      gp2[i] = g[2];
      gp3[i] = g[3];
    }
  }
}

/* ------------------------------------------------ general transformations */

/* Lorentz transformation held as a 4x4 matrix (Sec. 3.1: Lorentz
 * transformations; Sec. 4.1: ApplyBoost applies one held as a 4x4 matrix),
 * acting on (px, py, pz, E), row-major: y_r = sum_c L[4r + c] x_c, summed
 * left to right.  m[k] points at column k of the matrices; stride 1: one
 * matrix per item (m[k][i]), 0: one matrix for all items (m[k][0]). */
void orc_lorentz_transform(int64_t n, const double* const* x, const double* const* m, int64_t stride,
                           double* const* y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = i * stride;
    double v[4] = {x[0][i], x[1][i], x[2][i], x[3][i]}, r[4];
    for (int a = 0; a < 4; ++a) {
      double s = 0.0;
      for (int c = 0; c < 4; ++c) s += m[4 * a + c][j] * v[c];
      r[a] = s;
    }
    for (int a = 0; a < 4; ++a) y[a][i] = r[a];
  }
}

/* Reverse mode: grad_x = L^T grad_y; grad_m[4r + c] = grad_y_r x_c per item
 * (stride 1 only; grad_m may be NULL). */
void orc_lorentz_transform_vjp(int64_t n, const double* const* x, const double* const* m, int64_t stride,
                               const double* const* gy, double* const* gx, double* const* gm) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = i * stride;
    double g[4] = {gy[0][i], gy[1][i], gy[2][i], gy[3][i]};
    for (int c = 0; c < 4; ++c) {
      double s = 0.0;
      for (int a = 0; a < 4; ++a) s += m[4 * a + c][j] * g[a];
      gx[c][i] = s;
    }
    if (gm)
      for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 4; ++c) gm[4 * a + c][i] = g[a] * x[c][i];
  }
}

/* Rotation3D (Sec. 3.1: a rotation held as a 3x3 matrix) applied to the
 * spatial part of 4-vectors (px, py, pz, E): p' = R p (row-major, left to
 * right), E' = E.  Strides as for orc_lorentz_transform. */
void orc_rotate(int64_t n, const double* const* x, const double* const* r, int64_t stride, double* const* y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = i * stride;
    double v[3] = {x[0][i], x[1][i], x[2][i]}, o[3];
    for (int a = 0; a < 3; ++a) {
      double s = 0.0;
      for (int c = 0; c < 3; ++c) s += r[3 * a + c][j] * v[c];
      o[a] = s;
    }
    for (int a = 0; a < 3; ++a) y[a][i] = o[a];
    y[3][i] = x[3][i];
  }
}

/* Reverse mode: grad_p = R^T grad_p', grad_E = grad_E'; grad_r[3a + c] =
 * grad_p'_a p_c per item (stride 1 only; may be NULL). */
void orc_rotate_vjp(int64_t n, const double* const* x, const double* const* r, int64_t stride,
                    const double* const* gy, double* const* gx, double* const* gr) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = i * stride;
    double g[3] = {gy[0][i], gy[1][i], gy[2][i]};
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int a = 0; a < 3; ++a) s += r[3 * a + c][j] * g[a];
      gx[c][i] = s;
    }
    gx[3][i] = gy[3][i];
    if (gr)
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) gr[3 * a + c][i] = g[a] * x[c][i];
  }
}

/* AxisAngle (Sec. 3.1: the same rotation held as an axis and an angle)
 * applied to the spatial part: with the unit axis u = a / |a| and angle t,
 * Rodrigues' formula p' = p cos t + (u x p) sin t + u (u.p)(1 - cos t);
 * E' = E.  A zero axis gives the identity.  aa[0..2] = axis, aa[3] = angle;
 * strides as for orc_lorentz_transform. */
static void axis_angle_apply(const double a[3], double t, const double p[3], double o[3]) {
  double len = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  if (len == 0.0) {
    for (int k = 0; k < 3; ++k) o[k] = p[k];
    return;
  }
  double u[3] = {a[0] / len, a[1] / len, a[2] / len};
  double c = cos(t), s = sin(t);
  double cr[3] = {u[1] * p[2] - u[2] * p[1], u[2] * p[0] - u[0] * p[2], u[0] * p[1] - u[1] * p[0]};
  double d = u[0] * p[0] + u[1] * p[1] + u[2] * p[2];
  for (int k = 0; k < 3; ++k) o[k] = p[k] * c + cr[k] * s + u[k] * d * (1.0 - c);
}

void orc_rotate_axis_angle(int64_t n, const double* const* x, const double* const* aa, int64_t stride,
                           double* const* y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = i * stride;
    double a[3] = {aa[0][j], aa[1][j], aa[2][j]};
    double p[3] = {x[0][i], x[1][i], x[2][i]}, o[3];
    axis_angle_apply(a, aa[3][j], p, o);
    for (int k = 0; k < 3; ++k) y[k][i] = o[k];
    y[3][i] = x[3][i];
  }
}

/* Reverse mode w.r.t. the vectors: the rotation is orthogonal, so
 * grad_p = R^T grad_p' is the rotation by the opposite angle; grad_E = grad_E'. */
void orc_rotate_axis_angle_vjp(int64_t n, const double* const* aa, int64_t stride, const double* const* gy,
                               double* const* gx) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = i * stride;
    double a[3] = {aa[0][j], aa[1][j], aa[2][j]};
    double g[3] = {gy[0][i], gy[1][i], gy[2][i]}, o[3];
    axis_angle_apply(a, -aa[3][j], g, o);
    for (int k = 0; k < 3; ++k) gx[k][i] = o[k];
    gx[3][i] = gy[3][i];
  }
}

/* ------------------------------------------------------- analysis step */

/* Histogram of n values (masses) over n_bins equal bins of [lo, hi) -- the
 * analysis step that follows the mass (not in the paper; Sec. 6 places
 * GenVector inside ROOT, which analyses and visualises such data).
 * counts[0] receives v < lo, counts[n_bins + 1] receives v >= hi, and v in
 * [lo, hi) goes to counts[1 + b] with b = floor((v - lo) * s), s = n_bins /
 * (hi - lo), both evaluated in binary64, b clamped to n_bins - 1.  NaN is not
 * counted.  The counts are added to what `counts` holds. */
void orc_histogram(int64_t n, const double* v, double lo, double hi, int64_t n_bins, uint64_t* counts) {
  double s = (double)n_bins / (hi - lo);
  for (int64_t i = 0; i < n; ++i) {
    double x = v[i];
    if (x != x) continue;
    if (x < lo) {
      counts[0] += 1;
    } else if (x >= hi) {
      counts[n_bins + 1] += 1;
    } else {
      int64_t b = (int64_t)floor((x - lo) * s);
      if (b > n_bins - 1) b = n_bins - 1;
      counts[1 + b] += 1;
    }
  }
}

/* Per event, its pair (lexicographic rank among i < j, as the pair masses of
 * the jagged reduction are laid out) whose mass lies closest to `target`:
 * the smallest |m - target| in binary64, the lowest rank among equal
 * distances; a NaN mass is never chosen.  An event without a chosen pair
 * gets rank -1 and mass NaN. */
void orc_best_pair(int64_t ne, const int64_t* pair_offsets, const double* pm, double target, int64_t* rank,
                   double* best_m) {
  for (int64_t e = 0; e < ne; ++e) {
    int64_t r = -1;
    double best = 0.0, bm = NAN;
    for (int64_t k = pair_offsets[e]; k < pair_offsets[e + 1]; ++k) {
      double d = fabs(pm[k] - target);
      if (d != d) continue;
      if (r < 0 || d < best) {
        r = k - pair_offsets[e];
        best = d;
        bm = pm[k];
      }
    }
    rank[e] = r;
    best_m[e] = bm;
  }
}

/* -------------------------------------------- the pair-mass VJP, binary128 */

/* The chain rule of orc_mass_vjp for PtEtaPhiM legs carried out in binary128
 * (the Cartesian legs, their sum, (-P, E)/|m|, and the Jacobian of each leg's
 * conversion), each result rounded once to binary64.  The cancellation of
 * E dE - P.dp that costs the binary64 form its digits for nearly collinear
 * light pairs is then far below binary64 rounding: this is the reference for
 * a cancellation-free reverse mode. */
static void chain_ptetaphim_q(double c0, double c1, double c2, double c3, const quad u[4], quad g[4]) {
  quad pt = c0, eta = c1, phi = c2, mm = c3;
  quad cp = cosq(phi), sp = sinq(phi), sh = sinhq(eta), ch = coshq(eta);
  quad pc = pt * ch;
  quad e = sqrtq(pc * pc + mm * mm);
  quad ue = (e > 0) ? u[3] / e : 0;
  g[0] = u[0] * cp + u[1] * sp + u[2] * sh + ue * pt * ch * ch;
  g[1] = u[2] * pt * ch + ue * pt * pt * sh * ch;
  g[2] = -u[0] * pt * sp + u[1] * pt * cp;
  g[3] = ue * mm;
}

void orc_mass_vjp_q(int64_t n, const double* const* a, const double* const* b, const double* gm,
                    double* const* ga, double* const* gb) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    quad va[4], vb[4], w[4], u[4], g[4];
    cart_q(ORC_PTETAPHIM, a[0][i], a[1][i], a[2][i], a[3][i], va);
    cart_q(ORC_PTETAPHIM, b[0][i], b[1][i], b[2][i], b[3][i], vb);
    for (int k = 0; k < 4; ++k) w[k] = va[k] + vb[k];
    quad q = w[3] * w[3] - w[0] * w[0] - w[1] * w[1] - w[2] * w[2];
    quad am = sqrtq(fabsq(q));
    quad s = (am > 0) ? (quad)gm[i] / am : 0;
    u[0] = -w[0] * s;
    u[1] = -w[1] * s;
    u[2] = -w[2] * s;
    u[3] = w[3] * s;
    chain_ptetaphim_q(a[0][i], a[1][i], a[2][i], a[3][i], u, g);
    for (int k = 0; k < 4; ++k) ga[k][i] = (double)g[k];
    chain_ptetaphim_q(b[0][i], b[1][i], b[2][i], b[3][i], u, g);
    for (int k = 0; k < 4; ++k) gb[k][i] = (double)g[k];
  }
}
