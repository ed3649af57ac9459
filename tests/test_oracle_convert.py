"""Pins of the oracle's stand-alone coordinate conversion (Sec. 3.1: a 4D
vector in any of its coordinate systems; PxPyPzE, PtEtaPhiM, PtEtaPhiE and
PxPyPzM)
and of its reverse mode.  CPU only."""
import math

import mpmath
import numpy as np
import pytest

import oracle
import synth

SYSTEMS = ["PxPyPzE", "PtEtaPhiM", "PtEtaPhiE", "PxPyPzM"]
U = 2.0 ** -53


def _cart_random(n, seed, spacelike_frac=0.2):
    g = synth.rng(seed)
    px, py, pz = g.normal(0, 50, n), g.normal(0, 50, n), g.normal(0, 80, n)
    p2 = px * px + py * py + pz * pz
    m = g.uniform(0.5, 90, n)
    space = g.random(n) < spacelike_frac
    m = np.where(space, np.minimum(m, 0.9 * np.sqrt(p2)), m)  # spacelike: E^2 = |p|^2 - m^2 > 0
    e = np.sqrt(p2 + np.where(space, -1.0, 1.0) * m * m)
    return px, py, pz, e


def test_closed_values_and_beam_axis():
    cols = tuple(np.array(v, dtype=np.float64) for v in
                 ([3.0, 0.0, -1.0, 0.0, 0.0], [4.0, 2.0, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 5.0, 0.0],
                  [13.0, 2.0, 2.0, 6.0, 1.0]))
    pt, eta, phi, m = oracle.convert("PxPyPzE", "PtEtaPhiM", cols)
    assert pt.tolist() == [5.0, 2.0, 1.0, 0.0, 0.0]
    assert eta[0] == 0.0 and eta[3] == math.inf and eta[4] == 0.0
    assert phi[0] == math.atan2(4.0, 3.0) and phi[1] == math.pi / 2 and phi[2] == math.pi
    assert m[0] == 12.0 and m[1] == 0.0 and m[2] == math.sqrt(3.0) and m[3] == math.sqrt(11.0) and m[4] == 1.0
    # spacelike: the pair mass's convention, -sqrt(-q)
    s = oracle.convert("PxPyPzE", "PtEtaPhiM", tuple(np.array([x]) for x in (3.0, 4.0, 0.0, 4.0)))
    assert s[3][0] == -3.0
    _, _, _, e = oracle.convert("PxPyPzE", "PtEtaPhiE", cols)
    assert np.array_equal(e, cols[3])


def test_pxpypzm_closed_values():
    """PxPyPzM: E = sqrt(|p|^2 + M^2) on Pythagorean quadruples, p = 0 (E = |M|),
    M = 0 (E = |p|), only M^2 entering; back again the masses are exact."""
    pm = tuple(np.array(v, dtype=np.float64) for v in
               ([3.0, 1.0, 0.0, 0.0, 2.0, -6.0], [4.0, 2.0, 0.0, 0.0, 3.0, 0.0], [12.0, 2.0, 0.0, 0.0, 6.0, 0.0],
                [0.0, 4.0, 5.0, -5.0, 0.0, 8.0]))
    px, py, pz, e = oracle.convert("PxPyPzM", "PxPyPzE", pm)
    assert e.tolist() == [13.0, 5.0, 5.0, 5.0, 7.0, 10.0]
    assert all(np.array_equal(a, b) for a, b in zip((px, py, pz), pm[:3]))
    back = oracle.convert("PxPyPzE", "PxPyPzM", (px, py, pz, e))
    assert back[3].tolist() == [0.0, 4.0, 5.0, 5.0, 0.0, 8.0]  # |M|: the sign of M does not enter
    s = oracle.convert("PxPyPzE", "PxPyPzM", tuple(np.array([x]) for x in (3.0, 4.0, 0.0, 4.0)))
    assert s[3][0] == -3.0  # spacelike: -sqrt(-q)
    pt, eta, phi, m = oracle.convert("PxPyPzM", "PtEtaPhiM", pm)
    assert pt[0] == 5.0 and phi[0] == math.atan2(4.0, 3.0) and m[0] == 0.0 and m[1] == 4.0


def test_pxpypzm_energy_against_mpmath():
    px, py, pz, e = _cart_random(1000, 809, spacelike_frac=0.0)
    m = synth.rng(810).uniform(-50, 50, 1000)
    _, _, _, en = oracle.convert("PxPyPzM", "PxPyPzE", (px, py, pz, m))
    mpmath.mp.dps = 50
    for i in range(0, 1000, 3):
        X, Y, Z, M = (mpmath.mpf(float(v[i])) for v in (px, py, pz, m))
        E = float(mpmath.sqrt(X * X + Y * Y + Z * Z + M * M))
        assert abs(en[i] - E) <= 3 * U * E


@pytest.mark.parametrize("src", SYSTEMS)
def test_same_system_copies(src):
    cols = tuple(synth.rng(801).normal(size=64) for _ in range(4))
    out = oracle.convert(src, src, cols)
    assert all(np.array_equal(a, b) for a, b in zip(out, cols))
    g = tuple(synth.rng(802).normal(size=64) for _ in range(4))
    r = oracle.convert_vjp(src, src, cols, g)
    assert all(np.array_equal(a, b) for a, b in zip(r, g))


def test_inverse_against_mpmath():
    """The Cartesian -> (pt, eta, phi, M) formulas at 50 digits."""
    px, py, pz, e = _cart_random(2000, 803)
    pt, eta, phi, m = oracle.convert("PxPyPzE", "PtEtaPhiM", (px, py, pz, e))
    mpmath.mp.dps = 50
    for i in range(0, 2000, 7):
        X, Y, Z, E = (mpmath.mpf(float(v[i])) for v in (px, py, pz, e))
        PT = mpmath.hypot(X, Y)
        q = E * E - X * X - Y * Y - Z * Z
        M = mpmath.sqrt(q) if q >= 0 else -mpmath.sqrt(-q)
        assert abs(pt[i] - float(PT)) <= 2 * U * float(PT)
        assert abs(eta[i] - float(mpmath.asinh(Z / PT))) <= 4 * U * (abs(float(mpmath.asinh(Z / PT))) + 1e-300) + 4 * U
        assert abs(phi[i] - float(mpmath.atan2(Y, X))) <= 2 * U * math.pi
        S = float(E * E + X * X + Y * Y + Z * Z)
        assert abs(m[i] - float(M)) <= 4 * U * abs(float(M)) + 8 * U * S / (2 * abs(float(M)))


def test_round_trips():
    """PtEtaPhiM -> PxPyPzE -> PtEtaPhiM and PtEtaPhiE -> PtEtaPhiM ->
    PtEtaPhiE return the input within rounding (M through E^2 - |p|^2)."""
    a, _ = synth.pairs_generic(synth.rng(804), 5000)
    a = (a[0], a[1], a[2], a[3] + 5.0)  # masses comparable to pt: a well-conditioned M
    v = oracle.convert("PtEtaPhiM", "PxPyPzE", a)
    b = oracle.convert("PxPyPzE", "PtEtaPhiM", v)
    assert np.all(np.abs(b[0] - a[0]) <= 4 * U * a[0])
    assert np.all(np.abs(b[1] - a[1]) <= 16 * U * (1 + np.abs(a[1])))
    assert np.all(np.abs(b[2] - a[2]) <= 8 * U * np.pi)
    S = v[3] ** 2 + v[0] ** 2 + v[1] ** 2 + v[2] ** 2
    assert np.all(np.abs(b[3] - a[3]) <= 16 * U * S / (2 * a[3]))
    pe = oracle.convert("PtEtaPhiM", "PtEtaPhiE", a)
    assert np.array_equal(pe[0], a[0]) or np.all(np.abs(pe[0] - a[0]) <= 4 * U * a[0])
    back = oracle.convert("PtEtaPhiE", "PtEtaPhiM", pe)
    assert np.all(np.abs(back[3] - a[3]) <= 16 * U * S / (2 * a[3]))


def _fd_check(src, dst, cols, g, rel=1e-6):
    """Central differences of <g, convert(src, dst, x)> in each input, with
    steps h and h/2 combined by Richardson extrapolation (error O(h^4))."""
    an = oracle.convert_vjp(src, dst, cols, g)

    def central(k, h):
        up, dn = list(cols), list(cols)
        up[k] = cols[k] + h
        dn[k] = cols[k] - h
        fu, fd = oracle.convert(src, dst, up), oracle.convert(src, dst, dn)
        return sum(gg * (u - d) for gg, u, d in zip(g, fu, fd)) / (2 * h)

    # rounding of one evaluation of <g, convert(x)>: 8 u of each output, and for
    # a mass output 8 u S / (2|M|) (E^2 - |p|^2 cancels; S = E^2 + |p|^2)
    out = oracle.convert(src, dst, cols)
    v = oracle.convert(src, "PxPyPzE", cols)
    S = v[3] ** 2 + v[0] ** 2 + v[1] ** 2 + v[2] ** 2
    eps = sum(np.abs(gg) * 8 * U * (np.abs(o) + 1) for gg, o in zip(g, out))
    if dst in ("PtEtaPhiM", "PxPyPzM"):
        eps = eps + np.abs(g[3]) * 8 * U * S / (2 * np.maximum(np.abs(out[3]), 1e-300))
    for k in range(4):
        ang = src.startswith("PtEtaPhi") and k in (1, 2)  # eta, phi: absolute steps
        h = np.full(cols[k].size, 1e-6) if ang else 1e-6 * np.maximum(1.0, np.abs(cols[k]))
        num = (4 * central(k, h / 2) - central(k, h)) / 3
        scale = np.max(np.abs(np.stack(an)), axis=0) + np.abs(num)
        # Richardson of central differences: rounding noise at most 3 eps / h
        bad = np.abs(num - an[k]) > rel * scale + 3 * eps / h + 1e-9
        assert not np.any(bad), (src, dst, k, np.nonzero(bad)[0][:5], num[bad][:3], an[k][bad][:3])


@pytest.mark.parametrize("src", SYSTEMS)
@pytest.mark.parametrize("dst", SYSTEMS)
def test_vjp_against_finite_differences(src, dst):
    a, _ = synth.pairs_generic(synth.rng(805), 400)
    a = (a[0], a[1], a[2], a[3] + 5.0)
    cols = oracle.convert("PtEtaPhiM", src, a)
    g = tuple(synth.rng(806).normal(size=400) for _ in range(4))
    _fd_check(src, dst, cols, g)


@pytest.mark.parametrize("src,dst", [("PtEtaPhiM", "PxPyPzE"), ("PtEtaPhiE", "PxPyPzE"),
                                     ("PtEtaPhiM", "PtEtaPhiE"), ("PxPyPzE", "PtEtaPhiM"),
                                     ("PxPyPzM", "PxPyPzE"), ("PxPyPzM", "PtEtaPhiM"), ("PtEtaPhiE", "PxPyPzM")])
def test_vjp_of_a_round_trip_is_the_identity(src, dst):
    """For y = convert(src, dst, x): J_{src->dst}(x)^T J_{dst->src}(y)^T g = g."""
    a, _ = synth.pairs_generic(synth.rng(807), 1000)
    a = (a[0], a[1], a[2], a[3] + 5.0)
    x = oracle.convert("PtEtaPhiM", src, a)
    y = oracle.convert(src, dst, x)
    g = tuple(synth.rng(808).normal(size=1000) for _ in range(4))
    t = oracle.convert_vjp(dst, src, y, g)
    r = oracle.convert_vjp(src, dst, x, t)
    for k in range(4):
        assert np.all(np.abs(r[k] - g[k]) <= 1e-9 * (1 + np.max(np.abs(np.stack(t)), axis=0))), k
