"""Pins for the oracle's coordinate conversion and pair masses (CPU only).

Each check compares the oracle with something it does not share code with:
an independent closed form evaluated in mpmath at 60 digits, an exact
identity of binary floating point, or an invariant.  Paper: Sec. 3.1
(coordinate systems), Sec. 4.1 and Fig. 1 (mass of the sum of two vectors).
"""

import math
import os

import mpmath
import numpy as np
import pytest

import oracle
import synth
from tolerances import U64, mass_tol_acc_f64, mass_tol_f64, worst

mpmath.mp.dps = 60


def _mp_mass_rapidity(pta, etaa, phia, ma, ptb, etab, phib, mb):
    """m from rapidities: m^2 = Ma^2 + Mb^2 + 2 (mTa mTb cosh(ya - yb) - pta ptb cos(phia - phib)).

    A different route to the mass than the Cartesian definition the oracle
    implements, so a wrong conversion or sign there shows up here."""
    mp = mpmath
    pta, etaa, phia, ma = map(mp.mpf, (pta, etaa, phia, ma))
    ptb, etab, phib, mb = map(mp.mpf, (ptb, etab, phib, mb))
    mta = mp.sqrt(pta ** 2 + ma ** 2)
    mtb = mp.sqrt(ptb ** 2 + mb ** 2)
    ya = mp.asinh(pta * mp.sinh(etaa) / mta)
    yb = mp.asinh(ptb * mp.sinh(etab) / mtb)
    m2 = ma ** 2 + mb ** 2 + 2 * (mta * mtb * mp.cosh(ya - yb) - pta * ptb * mp.cos(phia - phib))
    return float(mp.sqrt(m2))


def _mp_masses(a, b, idx):
    return np.array([_mp_mass_rapidity(*(c[i] for c in a), *(c[i] for c in b)) for i in idx])


# ------------------------------------------------------------ conversion

def test_conversion_special_angles():
    pt = np.array([1.0, 7.5, 123.25, 4000.0])
    m = np.array([0.0, 0.105, 91.1876, 3.0])
    zero = np.zeros_like(pt)
    px, py, pz, e = oracle.to_cartesian("PtEtaPhiM", (pt, zero, zero, m))
    assert np.array_equal(px, pt) and np.array_equal(py, zero) and np.array_equal(pz, zero)
    assert np.allclose(e, np.hypot(pt, m), rtol=2 * U64, atol=0)
    # phi = pi/2: px ~ 0, py = pt
    px, py, _, _ = oracle.to_cartesian("PtEtaPhiM", (pt, zero, np.full_like(pt, np.pi / 2), m))
    assert np.allclose(py, pt, rtol=2 * U64) and np.all(np.abs(px) <= 1e-15 * pt)


def test_conversion_round_trip_and_shell():
    g = synth.rng(100)
    (a, _b) = synth.pairs_generic(g, 4096)
    px, py, pz, e = oracle.to_cartesian("PtEtaPhiM", a)
    pt, eta, phi, m = a
    assert np.allclose(np.hypot(px, py), pt, rtol=4 * U64, atol=0)
    assert np.allclose(np.arctan2(py, px), phi, rtol=0, atol=8 * U64 * np.pi)
    assert np.allclose(np.arcsinh(pz / pt), eta, rtol=0, atol=16 * U64 * 3)
    # on the mass shell: E^2 - |p|^2 = M^2 within the size of the cancelling terms
    q = e * e - (px * px + py * py + pz * pz)
    assert np.all(np.abs(q - m * m) <= 16 * U64 * (e * e))
    # PtEtaPhiE passes E through; PxPyPzE is the identity
    _, _, _, e2 = oracle.to_cartesian("PtEtaPhiE", (pt, eta, phi, e))
    assert np.array_equal(e2, e)
    out = oracle.to_cartesian("PxPyPzE", (px, py, pz, e))
    assert all(np.array_equal(u, v) for u, v in zip(out, (px, py, pz, e)))


# ------------------------------------------------------------ pair mass

def _sample_sets():
    g = synth.rng(101)
    a0, b0 = synth.pairs_generic(g, 200)
    a2, b2, mask = synth.pairs_stress(g, 400, collinear_frac=0.5)
    return [("generic", a0, b0), ("stress", a2, b2)]


@pytest.mark.parametrize("which", [0, 1])
def test_binary128_mass_matches_rapidity_form(which):
    name, a, b = _sample_sets()[which]
    n = a[0].size
    ref = _mp_masses(a, b, range(n))
    mq = oracle.mass_plain_q("PtEtaPhiM", a, b)
    r, i = worst(np.abs(mq - ref), 4 * U64 * np.abs(ref))
    assert r <= 1.0, (name, i, mq[i], ref[i])


@pytest.mark.parametrize("which", [0, 1])
def test_accurate_mass_matches_rapidity_form(which):
    name, a, b = _sample_sets()[which]
    ref = _mp_masses(a, b, range(a[0].size))
    macc = oracle.mass_accurate(a, b)
    r, i = worst(np.abs(macc - ref), mass_tol_acc_f64(ref))
    assert r <= 1.0, (name, i, macc[i], ref[i])


def test_massless_closed_form():
    """Massless legs: m^2 = 2 pt_a pt_b (cosh(eta_a - eta_b) - cos(phi_a - phi_b))."""
    g = synth.rng(102)
    a, b = synth.pairs_generic(g, 300)
    a = (a[0], a[1], a[2], np.zeros(300))
    b = (b[0], b[1], b[2], np.zeros(300))
    ref = np.array([float(mpmath.sqrt(2 * mpmath.mpf(a[0][i]) * b[0][i]
                                      * (mpmath.cosh(mpmath.mpf(a[1][i]) - b[1][i])
                                         - mpmath.cos(mpmath.mpf(a[2][i]) - b[2][i])))) for i in range(300)])
    mq = oracle.mass_plain_q("PtEtaPhiM", a, b)
    assert np.all(np.abs(mq - ref) <= 4 * U64 * ref)
    m64, s = oracle.mass_plain("PtEtaPhiM", a, b, scale=True)
    r, i = worst(np.abs(m64 - ref), mass_tol_f64(ref, s))
    assert r <= 1.0
    macc = oracle.mass_accurate(a, b)
    assert np.all(np.abs(macc - ref) <= mass_tol_acc_f64(ref))


def test_back_to_back_equal_energy_is_exactly_2E():
    """b = (-p, E): the sum is (0, 0, 0, 2E) and sqrt((2E)^2) = 2E exactly."""
    g = synth.rng(103)
    x, _ = synth.boost_items(g, 10000)
    a = x
    b = (-x[0], -x[1], -x[2], x[3])
    for f in (oracle.mass_plain, oracle.mass_plain_q):
        m = f("PxPyPzE", a, b)
        assert np.array_equal(m, 2 * x[3])


def test_zero_leg_gives_the_other_legs_mass():
    g = synth.rng(104)
    a, _ = synth.pairs_generic(g, 2000)
    z = tuple(np.zeros(2000) for _ in range(4))
    m, s = oracle.mass_plain("PtEtaPhiM", a, z, scale=True)
    r, _ = worst(np.abs(m - a[3]), mass_tol_f64(a[3], s))
    assert r <= 1.0
    mq = oracle.mass_plain_q("PtEtaPhiM", a, z)
    assert np.all(np.abs(mq - a[3]) <= 1e-12 * a[3] + 1e-14)
    macc = oracle.mass_accurate(a, z)
    assert np.all(np.abs(macc - a[3]) <= 4 * U64 * a[3])


def test_swapped_legs_bitwise():
    g = synth.rng(105)
    a, b = synth.pairs_generic(g, 5000)
    for c in ("PtEtaPhiM", "PxPyPzE", "PtEtaPhiE", "PxPyPzM"):
        assert np.array_equal(oracle.mass_plain(c, a, b), oracle.mass_plain(c, b, a))


def test_pxpypzm_pair_closed_forms():
    """Legs at rest: m = M_a + M_b; back to back with |p| = 3, M = 4: m = 2E = 10;
    a massless leg along x and one along -x: m = 2 sqrt(pa pb)."""
    a = (np.array([0.0, 3.0, 2.0]), np.array([0.0, 0.0, 0.0]), np.array([0.0, 0.0, 0.0]), np.array([3.0, 4.0, 0.0]))
    b = (np.array([0.0, -3.0, -8.0]), np.array([0.0, 0.0, 0.0]), np.array([0.0, 0.0, 0.0]), np.array([5.0, 4.0, 0.0]))
    m = oracle.mass_plain("PxPyPzM", a, b)
    assert m.tolist() == [8.0, 10.0, 8.0]
    assert np.array_equal(oracle.mass_plain_q("PxPyPzM", a, b), m)


def test_pxpypzm_agrees_with_ptetaphim():
    """The same physical legs given as PxPyPzM and PtEtaPhiM give the same
    binary128 mass within the rounding of the binary64 Cartesian inputs."""
    g = synth.rng(107)
    a, b = synth.pairs_generic(g, 3000)
    a, b = (a[0], a[1], a[2], a[3] + 1.0), (b[0], b[1], b[2], b[3] + 1.0)
    ca, cb = oracle.to_cartesian("PtEtaPhiM", a), oracle.to_cartesian("PtEtaPhiM", b)
    m1, s = oracle.mass_plain("PtEtaPhiM", a, b, scale=True)
    m2 = oracle.mass_plain_q("PxPyPzM", (ca[0], ca[1], ca[2], a[3]), (cb[0], cb[1], cb[2], b[3]))
    assert np.all(np.abs(m1 - m2) <= 32 * U64 * s / m1)


def test_spacelike_sum_has_negative_mass():
    a = (np.array([3.0, 0.0, 5.0]), np.array([0.0, 4.0, 0.0]), np.array([0.0, 0.0, 0.0]), np.array([1.0, 1.0, 4.0]))
    b = (np.array([0.0, 0.0, 0.0]), np.array([0.0, 0.0, 12.0]), np.array([0.0, 0.0, 0.0]), np.array([1.0, 2.0, 9.0]))
    # sums: (3,0,0,2): q = 4 - 9 = -5; (0,4,0,3): q = 9 - 16 = -7; (5,12,0,13): q = 0
    m = oracle.mass_plain("PxPyPzE", a, b)
    assert m[0] == -math.sqrt(5.0) and m[1] == -math.sqrt(7.0) and m[2] == 0.0
    mq = oracle.mass_plain_q("PxPyPzE", a, b)
    assert np.array_equal(mq, m)


def test_ptetaphie_agrees_with_ptetaphim():
    g = synth.rng(106)
    a, b = synth.pairs_generic(g, 3000)
    ea = oracle.to_cartesian("PtEtaPhiM", a)[3]
    eb = oracle.to_cartesian("PtEtaPhiM", b)[3]
    m1 = oracle.mass_plain("PtEtaPhiM", a, b)
    m2 = oracle.mass_plain("PtEtaPhiE", (a[0], a[1], a[2], ea), (b[0], b[1], b[2], eb))
    assert np.array_equal(m1, m2)


def test_plain_fp64_within_bound_of_binary128():
    """Plain binary64 against binary128 on the generic and the stress workloads,
    inside the conditioning-aware FP64 bound used for the GPU."""
    for name, a, b in _sample_sets():
        m, s = oracle.mass_plain("PtEtaPhiM", a, b, scale=True)
        mq = oracle.mass_plain_q("PtEtaPhiM", a, b)
        r, i = worst(np.abs(m - mq), mass_tol_f64(mq, s))
        assert r <= 1.0, (name, i)
    g = synth.rng(107)
    a, b = synth.pairs_generic(g, 4096)
    m, s = oracle.mass_plain("PtEtaPhiM", a, b, scale=True)
    mq = oracle.mass_plain_q("PtEtaPhiM", a, b)
    r, _ = worst(np.abs(m - mq), mass_tol_f64(mq, s))
    assert r <= 1.0


def test_accurate_fp64_within_8u_of_binary128_on_stress_workload():
    g = synth.rng(108)
    a, b, mask = synth.pairs_stress(g, 20000)
    mq = oracle.mass_plain_q("PtEtaPhiM", a, b)
    macc = oracle.mass_accurate(a, b)
    r, i = worst(np.abs(macc - mq), mass_tol_acc_f64(mq))
    assert r <= 1.0, (i, macc[i], mq[i], bool(mask[i]))
    # the plain form really does lose digits here, which is why the accurate form exists
    mpl = oracle.mass_plain("PtEtaPhiM", a, b)
    assert np.max(np.abs(mpl - mq) / mq) > 1e-9


def test_phi_seam_keeps_small_differences():
    """Legs on either side of phi = +-pi: the accurate form must see the small
    true opening angle, not 2 pi minus it."""
    pt = np.array([50.0, 900.0])
    eta = np.array([0.3, -1.2])
    m = np.array([0.0, 0.0])
    phia = np.array([np.pi - 1e-7, -np.pi + 3e-9])
    phib = np.array([-np.pi + 2e-7, np.pi - 5e-9])
    a = (pt, eta, phia, m)
    b = (pt * 1.5, eta, phib, m)
    ref = _mp_masses(a, b, range(2))
    macc = oracle.mass_accurate(a, b)
    assert np.all(np.abs(macc - ref) <= mass_tol_acc_f64(ref) * 4)


def test_scale_is_sum_of_squares_of_the_sum():
    """The tolerance scale S = E^2 + |P|^2 of the summed vector."""
    g = synth.rng(109)
    a, b = synth.pairs_generic(g, 3000)
    _, s = oracle.mass_plain("PtEtaPhiM", a, b, scale=True)
    ca = oracle.to_cartesian("PtEtaPhiM", a)
    cb = oracle.to_cartesian("PtEtaPhiM", b)
    w = [u + v for u, v in zip(ca, cb)]
    assert np.allclose(s, sum(c * c for c in w), rtol=1e-14, atol=0)


def _golden():
    import importlib.util
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_fixtures.py")
    spec = importlib.util.spec_from_file_location("make_fixtures", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_golden_pair_masses_reproduce_and_closed_forms():
    """tests/golden/pair_masses.txt is exactly what the oracle writes today, and
    its closed-form cases hold: identical massless legs give 0 in the
    cancellation-free form (and a value at the binary128 rounding scale,
    sqrt(u128) E, by the definition), a zero leg gives the other leg's M,
    equal back-to-back massless legs give 2E, identical massive legs 2M."""
    g = _golden()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "pair_masses.txt")
    assert open(path).read() == g.render()
    labels, a, b, m_q, m_acc = g.load(path)
    at = {lab: i for i, lab in enumerate(labels)}
    i = at["identical_massless"]
    assert m_acc[i] == 0.0
    assert m_q[i] <= 16 * 2.0 ** -56.5 * 2 * a[0][i] * math.cosh(a[1][i])
    assert m_q[at["zero_leg"]] == b[3][at["zero_leg"]]
    i = at["back_to_back_equal"]
    assert m_q[i] == 2.0 * a[0][i]
    i = at["identical_massive"]
    assert abs(m_q[i] - 2.0 * a[3][i]) <= 4 * U64 * m_q[i]
    # elsewhere the cancellation-free form agrees with binary128 within its bound
    keep = np.array([lab != "identical_massless" for lab in labels])
    assert np.all(np.abs(m_acc - m_q)[keep] <= mass_tol_acc_f64(m_q[keep]))
