"""Pins for the oracle's Lorentz boost (CPU only).  Paper: Sec. 4.1
(ApplyBoost: a 4D Lorentz transformation held as a 4x4 matrix).

The boost is pinned by the rapidity form (a different formula for the same
transformation), group properties and invariants."""

import numpy as np

import oracle
import synth
from tolerances import U64


def _items(n, seed):
    return synth.boost_items(synth.rng(seed), n)


def _rapidity_form(x, beta):
    """Boost written with rapidity z = atanh|beta| along n = beta/|beta|:
    E' = E cosh z + p_par sinh z, p_par' = p_par cosh z + E sinh z, p_perp' = p_perp."""
    px, py, pz, e = (np.asarray(c, dtype=np.longdouble) for c in x)
    bx, by, bz = (np.asarray(c, dtype=np.longdouble) for c in beta)
    bm = np.sqrt(bx * bx + by * by + bz * bz)
    z = np.arctanh(bm)
    nx, ny, nz = bx / bm, by / bm, bz / bm
    ppar = px * nx + py * ny + pz * nz
    ch, sh = np.cosh(z), np.sinh(z)
    e2 = e * ch + ppar * sh
    ppar2 = ppar * ch + e * sh
    d = ppar2 - ppar
    return tuple(np.asarray(c, dtype=np.float64) for c in (px + d * nx, py + d * ny, pz + d * nz, e2))


def test_zero_velocity_is_identity():
    x, beta = _items(5000, 200)
    zero = tuple(np.zeros(5000) for _ in range(3))
    for f in (oracle.boost, oracle.boost_q):
        y = f(x, zero)
        assert all(np.array_equal(u, v) for u, v in zip(y, x))


def test_matches_rapidity_form():
    x, beta = _items(20000, 201)
    ref = _rapidity_form(x, beta)
    scale = oracle.boost_scale(x, beta)
    for f, tol in ((oracle.boost, 1e-13), (oracle.boost_q, 1e-16)):
        y = f(x, beta)
        for k in range(4):
            # long double rapidity form is good to ~1e-18 * gamma^2 * scale
            assert np.all(np.abs(y[k] - ref[k]) <= tol * scale[k] * 50), (f.__name__, k)


def test_inverse_boost_restores_vector():
    x, beta = _items(20000, 202)
    nb = tuple(-b for b in beta)
    y = oracle.boost(oracle.boost(x, beta), nb)
    b2 = sum(b * b for b in beta)
    g2 = 1.0 / (1.0 - b2)
    norm = np.abs(x[3]) + np.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2)
    for k in range(4):
        assert np.all(np.abs(y[k] - x[k]) <= 64 * U64 * g2 * norm)


def test_mass_is_invariant():
    x, beta = _items(20000, 203)
    y = oracle.boost_q(x, beta)
    m2x = x[3] ** 2 - x[0] ** 2 - x[1] ** 2 - x[2] ** 2
    m2y = y[3] ** 2 - y[0] ** 2 - y[1] ** 2 - y[2] ** 2
    sy = y[3] ** 2 + y[0] ** 2 + y[1] ** 2 + y[2] ** 2
    assert np.all(np.abs(m2y - m2x) <= 32 * U64 * sy)


def test_rest_frame():
    """beta = -p/E takes a vector to rest: p' = 0, E' = m."""
    x, _ = _items(10000, 204)
    px, py, pz, e = x
    beta = (-px / e, -py / e, -pz / e)
    m = np.sqrt(np.maximum(e * e - px * px - py * py - pz * pz, 0.0))
    keep = m > 1.0  # a light, fast vector needs gamma ~ E/m: stay well conditioned
    y = oracle.boost_q(x, beta)
    g = e / np.maximum(m, 1e-300)
    for k in range(3):
        assert np.all(np.abs(y[k][keep]) <= 64 * U64 * (g * g * e)[keep])
    assert np.all(np.abs(y[3] - m)[keep] <= 64 * U64 * (g * g * e)[keep])


def test_particle_at_rest_gets_gamma_m():
    """(M, 0) boosts to E' = gamma M, p' = gamma M beta."""
    g = synth.rng(205)
    n = 3000
    mass = g.uniform(0.1, 100.0, n)
    _, beta = _items(n, 206)
    zero = np.zeros(n)
    y = oracle.boost((zero, zero, zero, mass), beta)
    b2 = sum(b * b for b in beta)
    gam = 1.0 / np.sqrt(1.0 - b2)
    assert np.allclose(y[3], gam * mass, rtol=8 * U64 * 100, atol=0)
    for k in range(3):
        assert np.allclose(y[k], gam * mass * beta[k], rtol=1e-13, atol=1e-14 * gam * mass)


def test_collinear_composition():
    """Two boosts along z compose to one with velocity (b1 + b2)/(1 + b1 b2)."""
    g = synth.rng(207)
    n = 5000
    x, _ = _items(n, 208)
    b1 = g.uniform(-0.95, 0.95, n)
    b2 = g.uniform(-0.95, 0.95, n)
    z = np.zeros(n)
    y = oracle.boost_q(oracle.boost_q(x, (z, z, b1)), (z, z, b2))
    bc = (b1 + b2) / (1.0 + b1 * b2)
    yc = oracle.boost_q(x, (z, z, bc))
    norm = np.abs(x[3]) + np.abs(x[2])
    g2 = 1.0 / (1.0 - bc * bc) + 1.0 / (1.0 - b1 * b1) + 1.0 / (1.0 - b2 * b2)
    for k in range(4):
        assert np.all(np.abs(y[k] - yc[k]) <= 64 * U64 * g2 * (norm + np.abs(x[k])))


def test_broadcast_velocity_equals_repeated():
    x, beta = _items(4000, 209)
    one = tuple(np.array([b[0]]) for b in beta)
    rep = tuple(np.full(4000, b[0]) for b in beta)
    y0 = oracle.boost(x, one, beta_stride=0)
    y1 = oracle.boost(x, rep, beta_stride=1)
    assert all(np.array_equal(u, v) for u, v in zip(y0, y1))


def test_binary64_within_bound_of_binary128():
    x, beta = _items(50000, 210)
    y = oracle.boost(x, beta)
    yq = oracle.boost_q(x, beta)
    s = oracle.boost_scale(x, beta)
    # gamma = 1/sqrt(1 - beta^2) magnifies the rounding of beta^2 by gamma^2
    g2 = 1.0 / (1.0 - sum(b * b for b in beta))
    for k in range(4):
        assert np.all(np.abs(y[k] - yq[k]) <= 8 * U64 * g2 * s[k])


def test_scale_is_boost_of_absolute_values():
    """(|L| |x|): for non-negative x and beta it is the boost itself."""
    x, beta = _items(3000, 211)
    ax = tuple(np.abs(c) for c in x)
    ab = tuple(np.abs(c) for c in beta)
    assert all(np.array_equal(u, v) for u, v in zip(oracle.boost_scale(x, beta), oracle.boost(ax, ab)))
