"""Pins for the oracle's per-event (jagged) reduction (CPU only).

Pair masses are re-derived by brute force over itertools.combinations (which
fixes the lexicographic pair order independently of the rank formula), totals
against exactly rounded sums (math.fsum), event masses against binary128 and
against the pair identity m_tot^2 = sum_{i<j} m_ij^2 - (n - 2) sum_i M_i^2."""

import itertools
import math

import numpy as np
import pytest

import oracle
import synth
from tolerances import U64, mass_tol_acc_f64, mass_tol_f64, worst


def _events(n_events, seed, mean=8.0, cap=64):
    return synth.jagged_events(synth.rng(seed), n_events, mean=mean, cap=cap)


def _brute_pairs(offsets):
    ii, jj = [], []
    for e in range(offsets.size - 1):
        for i, j in itertools.combinations(range(offsets[e], offsets[e + 1]), 2):
            ii.append(i)
            jj.append(j)
    return np.array(ii, dtype=np.int64), np.array(jj, dtype=np.int64)


def test_pair_offsets_count():
    off, _ = _events(3000, 400)
    po = oracle.pair_offsets(off)
    c = np.diff(off)
    assert po[0] == 0 and np.array_equal(np.diff(po), c * (c - 1) // 2)


@pytest.mark.parametrize("mode", [oracle.PLAIN, oracle.ACCURATE])
def test_pair_masses_brute_force(mode):
    off, p = _events(1500, 401)
    tot, em, pm, po = oracle.event_reduce("PtEtaPhiM", off, p, mode=mode)
    ii, jj = _brute_pairs(off)
    assert pm.size == ii.size == po[-1]
    a = tuple(c[ii] for c in p)
    b = tuple(c[jj] for c in p)
    want = oracle.mass_plain("PtEtaPhiM", a, b) if mode == oracle.PLAIN else oracle.mass_accurate(a, b)
    assert np.array_equal(pm, want)


def test_totals_against_exact_sums():
    off, p = _events(800, 402)
    tot, em, _, _ = oracle.event_reduce("PtEtaPhiM", off, p)
    cart = oracle.to_cartesian("PtEtaPhiM", p)
    for e in range(off.size - 1):
        lo, hi = off[e], off[e + 1]
        for k in range(4):
            seg = cart[k][lo:hi]
            exact = math.fsum(seg)
            bound = (hi - lo) * U64 * float(np.sum(np.abs(seg))) + 0.0
            assert abs(tot[k][e] - exact) <= bound


def test_event_mass_plain_and_accurate_against_binary128():
    off, p = _events(3000, 403)
    tq, emq = oracle.event_reduce_q("PtEtaPhiM", off, p)
    tot, em, _, _ = oracle.event_reduce("PtEtaPhiM", off, p, mode=oracle.PLAIN)
    s = tq[3] ** 2 + tq[0] ** 2 + tq[1] ** 2 + tq[2] ** 2
    n = np.diff(off)
    r, i = worst(np.abs(em - emq), mass_tol_f64(emq, s * np.maximum(n, 1)))
    assert r <= 1.0, i
    _, ema, _, _ = oracle.event_reduce("PtEtaPhiM", off, p, mode=oracle.ACCURATE)
    # the accurate event mass is a sum of positive terms: a few u per term
    r, i = worst(np.abs(ema - emq), 4 * mass_tol_acc_f64(emq) + 1e-300)
    assert r <= 1.0, (i, ema[i], emq[i], n[i])


def test_pair_identity():
    off, p = _events(2000, 404)
    tot, em, pm, po = oracle.event_reduce("PtEtaPhiM", off, p, mode=oracle.ACCURATE)
    _, emq = oracle.event_reduce_q("PtEtaPhiM", off, p)
    m2 = p[3] ** 2
    for e in range(off.size - 1):
        n = off[e + 1] - off[e]
        if n < 2:
            continue
        lhs = emq[e] ** 2
        rhs = math.fsum((pm[po[e]:po[e + 1]] ** 2).tolist()) - (n - 2) * math.fsum(m2[off[e]:off[e + 1]].tolist())
        scale = math.fsum((pm[po[e]:po[e + 1]] ** 2).tolist()) + (n - 2) * math.fsum(m2[off[e]:off[e + 1]].tolist())
        assert abs(lhs - rhs) <= 64 * U64 * scale


def test_small_events():
    """n = 0: zero total, zero mass; n = 1: the particle's own mass;
    n = 2: event mass equals the pair mass (plain: bitwise)."""
    off = np.array([0, 0, 1, 3, 3, 5], dtype=np.int64)
    g = synth.rng(405)
    a, _ = synth.pairs_generic(g, 5)
    tot, em, pm, po = oracle.event_reduce("PtEtaPhiM", off, a)
    assert [t[0] for t in tot] == [0.0] * 4 and em[0] == 0.0 and em[3] == 0.0
    assert abs(em[1] - a[3][0]) <= 1e-6
    assert list(po) == [0, 0, 0, 1, 1, 2]
    assert em[2] == pm[0] and em[4] == pm[1]
    _, ema, pma, _ = oracle.event_reduce("PtEtaPhiM", off, a, mode=oracle.ACCURATE)
    assert ema[1] == a[3][0] and ema[0] == 0.0
    assert abs(ema[2] - pma[0]) <= 4 * U64 * pma[0]


def _fd_event(coords, off, p, g_total, g_em, g_pair, h=1e-6):
    """Central differences of L = g_total.total + g_em.event_m + g_pair.pair_m,
    every piece evaluated in binary128 (pairs by brute force over i < j)."""
    ii, jj = _brute_pairs(off)

    def loss(pp):
        tot, em = oracle.event_reduce_q(coords, off, pp)
        pm, pl = oracle.mass_plain_q(coords, tuple(c[ii] for c in pp), tuple(c[jj] for c in pp), lo=True)
        val = math.fsum(np.concatenate([g_em * em, g_pair * pm, g_pair * pl]
                                       + [g_total[k] * tot[k] for k in range(4)]).tolist())
        return val
    out = []
    for k in range(4):
        col = np.empty(p[0].size)
        for i in range(p[0].size):
            step = h * max(1.0, abs(p[k][i]))
            pp = [c.copy() for c in p]
            pp[k][i] += step
            up = loss(pp)
            pp[k][i] -= 2 * step
            dn = loss(pp)
            col[i] = (up - dn) / (2 * step)
        out.append(col)
    return out


@pytest.mark.parametrize("coords", ["PtEtaPhiM", "PxPyPzE", "PxPyPzM"])
def test_event_vjp_matches_finite_differences(coords):
    g = synth.rng(406)
    off = np.array([0, 2, 2, 3, 7, 13], dtype=np.int64)
    # Cartesian particles come from the heavy boost workload: a light particle
    # alone in its event has a mass too ill-conditioned for finite differences
    p = synth.pairs_generic(g, 13)[0] if coords == "PtEtaPhiM" else synth.boost_items(g, 13)[0]
    if coords == "PxPyPzM":
        p = oracle.convert("PxPyPzE", "PxPyPzM", p)
    ne = off.size - 1
    po = oracle.pair_offsets(off)
    gt = synth.upstream(g, ne, 4)
    gem = g.standard_normal(ne)
    gpr = g.standard_normal(int(po[-1]))
    an = oracle.event_reduce_vjp(coords, off, p, gt, gem, gpr)
    fd = _fd_event(coords, off, p, gt, gem, gpr)
    for k in range(4):
        assert np.allclose(an[k], fd[k], rtol=1e-6, atol=1e-6 * np.max(np.abs(an[k])))


def test_event_vjp_reduces_to_pair_and_total_parts():
    g = synth.rng(407)
    a, b = synth.pairs_generic(g, 500)
    # n = 2 events with only the pair gradient: the pair-mass vjp
    p = tuple(np.stack([x, y], axis=1).reshape(-1) for x, y in zip(a, b))
    off = np.arange(0, 1001, 2, dtype=np.int64)
    gpr = g.standard_normal(500)
    gp = oracle.event_reduce_vjp("PtEtaPhiM", off, p, g_pair=gpr)
    ga, gb = oracle.mass_vjp("PtEtaPhiM", a, b, gpr)
    for k in range(4):
        assert np.allclose(gp[k][0::2], ga[k], rtol=1e-13, atol=1e-13 * np.abs(ga[k]).max())
        assert np.allclose(gp[k][1::2], gb[k], rtol=1e-13, atol=1e-13 * np.abs(gb[k]).max())
    # only the total's gradient: every particle gets it through its own Jacobian
    gt = synth.upstream(g, 500, 4)
    gp = oracle.event_reduce_vjp("PxPyPzE", off, p, g_total=gt)
    for k in range(4):
        assert np.array_equal(gp[k][0::2], gt[k]) and np.array_equal(gp[k][1::2], gt[k])
