"""Pins for the oracle's reverse-mode derivatives (CPU only).

The analytic vector-Jacobian products are checked against central finite
differences of the binary128 forward pass (which shares none of the gradient
formulas), and against identities that follow from symmetries of the mass:
homogeneity (Euler), rotation invariance in phi, longitudinal boost invariance
for massless legs, and Lorentz invariance for the boost."""

import numpy as np
import pytest

import oracle
import synth


def _fd_mass(coords, a, b, step_rel, step_abs_angle):
    """Central differences of m w.r.t. every coordinate of both legs, on the
    binary128 forward pass carried to ~106 bits (value + remainder), so a
    small step costs no accuracy.  Returns 8 arrays: d m / d a_k (k = 0..3)
    then d m / d b_k."""
    out = []
    angle = {"PtEtaPhiM": (1, 2), "PtEtaPhiE": (1, 2), "PxPyPzE": (), "PxPyPzM": ()}[coords]
    for leg in (0, 1):
        for k in range(4):
            x = (a, b)[leg][k]
            h = step_abs_angle * np.ones_like(x) if k in angle else step_rel * np.maximum(1.0, np.abs(x))
            xp, xm = x + h, x - h
            hh = xp - xm
            def with_col(col):
                legs = [list(a), list(b)]
                legs[leg][k] = col
                return oracle.mass_plain_q(coords, legs[0], legs[1], lo=True)
            (hp, lp), (hm, lm) = with_col(xp), with_col(xm)
            out.append(((hp - hm) + (lp - lm)) / hh)
    return out


@pytest.mark.parametrize("coords", ["PtEtaPhiM", "PtEtaPhiE", "PxPyPzE", "PxPyPzM"])
def test_mass_vjp_matches_finite_differences(coords):
    g = synth.rng(300)
    n = 3000
    a, b = synth.pairs_generic(g, n)
    if coords != "PtEtaPhiM":
        ca = oracle.to_cartesian("PtEtaPhiM", a)
        cb = oracle.to_cartesian("PtEtaPhiM", b)
        if coords == "PtEtaPhiE":
            a = (a[0], a[1], a[2], ca[3])
            b = (b[0], b[1], b[2], cb[3])
        elif coords == "PxPyPzM":
            a = (ca[0], ca[1], ca[2], a[3] + 1.0)
            b = (cb[0], cb[1], cb[2], b[3] + 1.0)
        else:
            a, b = ca, cb
    gm = g.standard_normal(n)
    ga, gb = oracle.mass_vjp(coords, a, b, gm)
    an = np.stack(list(ga) + list(gb))
    fd = np.stack(_fd_mass(coords, a, b, 1e-9, 1e-9)) * gm
    m, s = oracle.mass_plain(coords, a, b, scale=True)
    kappa = s / (m * m)
    keep = kappa <= 1e4
    assert keep.sum() > 0.99 * n
    err = np.max(np.abs(fd - an), axis=0)
    ref = np.max(np.abs(an), axis=0)
    assert np.all(err[keep] <= 1e-6 * ref[keep])


def test_mass_vjp_identities():
    g = synth.rng(301)
    n = 5000
    a, b = synth.pairs_generic(g, n)
    one = np.ones(n)
    (ga, gb) = oracle.mass_vjp("PtEtaPhiM", a, b, one)
    m, s = oracle.mass_plain("PtEtaPhiM", a, b, scale=True)
    # Euler: m is homogeneous of degree 1 in (pt, M) of both legs; each term is
    # of size S/m, so rounding moves the sum by a few u * S / m
    euler = a[0] * ga[0] + a[3] * ga[3] + b[0] * gb[0] + b[3] * gb[3]
    assert np.all(np.abs(euler - m) <= 1e-13 * m + 64 * 2.0 ** -53 * s / m)
    # rotating both legs by the same phi leaves m unchanged
    cond = 64 * 2.0 ** -53 * s / m  # rounding size of one derivative term
    assert np.all(np.abs(ga[2] + gb[2]) <= cond)
    # massless legs: shifting both pseudorapidities is a longitudinal boost
    z = np.zeros(n)
    a0 = (a[0], a[1], a[2], z)
    b0 = (b[0], b[1], b[2], z)
    (ga0, gb0) = oracle.mass_vjp("PtEtaPhiM", a0, b0, one)
    m0, s0 = oracle.mass_plain("PtEtaPhiM", a0, b0, scale=True)
    assert np.all(np.abs(ga0[1] + gb0[1]) <= 64 * 2.0 ** -53 * s0 / m0)
    # Cartesian legs: m is homogeneous of degree 1 in all components
    ca = oracle.to_cartesian("PtEtaPhiM", a)
    cb = oracle.to_cartesian("PtEtaPhiM", b)
    (gca, gcb) = oracle.mass_vjp("PxPyPzE", ca, cb, one)
    e2 = sum(ca[k] * gca[k] + cb[k] * gcb[k] for k in range(4))
    mc, s = oracle.mass_plain("PxPyPzE", ca, cb, scale=True)
    assert np.all(np.abs(e2 - mc) <= 1e-12 * mc + 64 * 2.0 ** -53 * s / mc)


def test_mass_vjp_zero_mass_is_zero():
    a = (np.array([3.0]), np.array([4.0]), np.array([0.0]), np.array([5.0]))
    b = (np.array([3.0]), np.array([4.0]), np.array([0.0]), np.array([5.0]))
    ga, gb = oracle.mass_vjp("PxPyPzE", a, b, np.array([1.0]))
    assert all(v[0] == 0.0 for v in ga + gb)


def _fd_boost(x, beta, gy, h_rel=1e-8, h_beta=1e-8):
    def loss(xx, bb):
        y, lo = oracle.boost_q(xx, bb, lo=True)
        return sum(gy[c] * y[c] for c in range(4)), sum(gy[c] * lo[c] for c in range(4))

    def diff(p, m):
        return (p[0] - m[0]) + (p[1] - m[1])
    gx, gbeta = [], []
    for k in range(4):
        h = h_rel * np.maximum(1.0, np.abs(x[k]))
        xp, xm = list(x), list(x)
        xp[k] = x[k] + h
        xm[k] = x[k] - h
        gx.append(diff(loss(xp, beta), loss(xm, beta)) / (xp[k] - xm[k]))
    for k in range(3):
        bp, bm = list(beta), list(beta)
        bp[k] = beta[k] + h_beta
        bm[k] = beta[k] - h_beta
        gbeta.append(diff(loss(x, bp), loss(x, bm)) / (bp[k] - bm[k]))
    return gx, gbeta


def test_boost_vjp_matches_finite_differences():
    g = synth.rng(302)
    n = 3000
    x, beta = synth.boost_items(g, n)
    # keep |beta| <= 0.98 so beta +- h stays inside the light cone
    beta = tuple(b * 0.98 / 0.99 for b in beta)
    gy = synth.upstream(g, n, 4)
    gx, gbeta = oracle.boost_vjp(x, beta, gy)
    fx, fb = _fd_boost(x, beta, gy)
    an = np.stack(list(gx) + list(gbeta))
    fd = np.stack(fx + fb)
    err = np.max(np.abs(an - fd), axis=0)
    ref = np.max(np.abs(an), axis=0)
    assert np.all(err <= 1e-6 * ref)


def test_boost_vjp_of_invariant_mass():
    """With upstream gradient dm/dy the mass of the boosted vector does not
    depend on beta (grad_beta = 0) and grad_x is dm/dx."""
    g = synth.rng(303)
    n = 5000
    x, beta = synth.boost_items(g, n)
    y = oracle.boost(x, beta)
    my = np.sqrt(y[3] ** 2 - y[0] ** 2 - y[1] ** 2 - y[2] ** 2)
    keep = my > 1.0
    gy = (-y[0] / my, -y[1] / my, -y[2] / my, y[3] / my)
    gx, gbeta = oracle.boost_vjp(x, beta, gy)
    mx = np.sqrt(x[3] ** 2 - x[0] ** 2 - x[1] ** 2 - x[2] ** 2)
    want = (-x[0] / mx, -x[1] / mx, -x[2] / mx, x[3] / mx)
    scale = (np.abs(x[3]) + np.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2)) / mx
    g2 = 1.0 / (1.0 - sum(b * b for b in beta))
    for k in range(4):
        assert np.all((np.abs(gx[k] - want[k]) <= 1e-12 * g2 * scale * scale)[keep])
    ey = (np.abs(y[3]) + np.sqrt(y[0] ** 2 + y[1] ** 2 + y[2] ** 2)) / my
    for k in range(3):
        assert np.all((np.abs(gbeta[k]) <= 1e-11 * g2 * g2 * ey * (np.abs(x[3]) + 1))[keep])


def test_boost_vjp_grad_x_is_forward_boost_of_upstream():
    g = synth.rng(304)
    n = 4000
    x, beta = synth.boost_items(g, n)
    gy = synth.upstream(g, n, 4)
    gx, _ = oracle.boost_vjp(x, beta, gy)
    fwd = oracle.boost(gy, beta)
    for k in range(4):
        assert np.array_equal(gx[k], fwd[k])


def test_mass_vjp_scale_bounds_the_vjp():
    """The absolute-value evaluation dominates the VJP componentwise
    (triangle inequality) and equals |VJP| for Cartesian legs."""
    g = synth.rng(305)
    n = 5000
    a, b = synth.pairs_generic(g, n)
    gm = g.standard_normal(n)
    for coords in ("PtEtaPhiM", "PtEtaPhiE"):
        va, vb = oracle.mass_vjp(coords, a, b, gm)
        sa, sb = oracle.mass_vjp_scale(coords, a, b, gm)
        for v, s in zip(va + vb, sa + sb):
            assert np.all(s >= np.abs(v) * (1 - 1e-14))
    ca, cb = oracle.to_cartesian("PtEtaPhiM", a), oracle.to_cartesian("PtEtaPhiM", b)
    pa, pb = (ca[0], ca[1], ca[2], a[3] + 1.0), (cb[0], cb[1], cb[2], b[3] + 1.0)
    va, vb = oracle.mass_vjp("PxPyPzM", pa, pb, gm)
    sa, sb = oracle.mass_vjp_scale("PxPyPzM", pa, pb, gm)
    for v, s in zip(va + vb, sa + sb):
        assert np.all(s >= np.abs(v) * (1 - 1e-14))
    va, vb = oracle.mass_vjp("PxPyPzE", ca, cb, gm)
    sa, sb = oracle.mass_vjp_scale("PxPyPzE", ca, cb, gm)
    for v, s in zip(va + vb, sa + sb):
        assert np.array_equal(s, np.abs(v))


def test_mass_vjp_q_pins():
    """The binary128 VJP: equal to the binary64 one on generic pairs; on the
    collinear light stress pairs equal to central differences of the binary128
    forward (where binary64 loses its digits); phi rotation of both legs
    leaves m unchanged (the two phi components cancel); Euler homogeneity."""
    g = synth.rng(310)
    a, b = synth.pairs_generic(g, 2000)
    gm = g.standard_normal(2000)
    qa, qb = oracle.mass_vjp_q(a, b, gm)
    da, db = oracle.mass_vjp("PtEtaPhiM", a, b, gm)
    ref = np.max(np.abs(np.stack(qa + qb)), axis=0)
    assert np.all(np.abs(np.stack(qa + qb) - np.stack(da + db)) <= 1e-9 * ref)
    sa, sb, _ = synth.pairs_stress(synth.rng(311), 600, collinear_frac=1.0)
    one = np.ones(600)
    qa, qb = oracle.mass_vjp_q(sa, sb, one)
    an = np.stack(list(qa) + list(qb))
    fd = np.stack(_fd_mass("PtEtaPhiM", sa, sb, 1e-12, 1e-12))
    ref = np.max(np.abs(an), axis=0)
    assert np.all(np.abs(fd - an) <= 1e-9 * ref)
    da, db = oracle.mass_vjp("PtEtaPhiM", sa, sb, one)
    assert np.max(np.abs(np.stack(list(da) + list(db)) - an) / ref) > 1e-8  # binary64 loses ~10 digits here
    assert np.all(np.abs(qa[2] + qb[2]) <= 4 * 2.0 ** -53 * np.abs(qa[2]) + 1e-300)
    m = oracle.mass_plain_q("PtEtaPhiM", sa, sb)
    terms = np.stack([sa[0] * qa[0], sa[3] * qa[3], sb[0] * qb[0], sb[3] * qb[3]])
    assert np.all(np.abs(terms.sum(axis=0) - m) <= 8 * 2.0 ** -53 * np.abs(terms).sum(axis=0))
