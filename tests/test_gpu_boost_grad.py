"""GPU parity of the boost and of the reverse-mode kernels (mass and boost)
against the CPU oracle, plus torch.autograd checks of the wrappers."""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import gpu, host, widened
from tolerances import U32, U64, boost_tol, worst

pytestmark = pytest.mark.gpu

glv = pytest.importorskip("paper_2312_02756_amd.glv")
ag = pytest.importorskip("paper_2312_02756_amd.autograd")


def _np(dtype):
    return np.float64 if dtype == torch.float64 else np.float32


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [1, 5, 64, 1001, 65536])
def test_boost_per_item(n, dtype):
    x, beta = synth.boost_items(synth.rng(600 + n), n)
    y = host(glv.glv_boost(gpu(x, dtype), gpu(beta, dtype)))
    wx, wb = widened(x, dtype), widened(beta, dtype)
    y_or = oracle.boost(wx, wb)
    s = oracle.boost_scale(wx, wb)
    for k in range(4):
        r, i = worst(np.abs(y[k].astype(np.float64) - y_or[k]), boost_tol(s[k], _np(dtype)))
        assert r <= 1.0, (k, i)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_boost_broadcast_in_place_and_identity(dtype):
    n = 40000
    x, beta = synth.boost_items(synth.rng(601), n)
    one = tuple(np.array([b[3]]) for b in beta)
    gx = gpu(x, dtype)
    glv.glv_boost(gx, gpu(one, dtype), out=gx)  # in place
    y = host(gx)
    wx, wb = widened(x, dtype), widened(one, dtype)
    y_or = oracle.boost(wx, wb, beta_stride=0)
    s = oracle.boost_scale(wx, wb, beta_stride=0)
    for k in range(4):
        r, _ = worst(np.abs(y[k].astype(np.float64) - y_or[k]), boost_tol(s[k], _np(dtype)))
        assert r <= 1.0
    zero = tuple(np.zeros(n) for _ in range(3))
    y0 = host(glv.glv_boost(gpu(x, dtype), gpu(zero, dtype)))
    for k in range(4):
        assert np.array_equal(y0[k], np.asarray(x[k], dtype=_np(dtype)))


def test_boost_full_size():
    """2^24 per-item boosts in the benchmark's launch shape, every item."""
    n = 1 << 24
    x, beta = synth.boost_items(synth.rng(synth.LARGE), n)
    y = host(glv.glv_boost(gpu(x, torch.float64), gpu(beta, torch.float64)))
    y_or, s = oracle.boost(x, beta), oracle.boost_scale(x, beta)
    for k in range(4):
        r, i = worst(np.abs(y[k] - y_or[k]), boost_tol(s[k], np.float64))
        assert r <= 1.0, (k, i)


# -------------------------------------------------------------- mass bwd

def _mass_vjp_tol(a, b, coords, dtype, g_or, gm):
    """Per component: base * |g|_inf + 64 u (|.|-scale of its chain-rule terms
    + kappa |g_c|), kappa = S/m^2 (the rounding of m itself)."""
    m, s = oracle.mass_plain(coords, a, b, scale=True)
    kappa = s / np.maximum(m * m, 1e-300)
    sa, sb = oracle.mass_vjp_scale(coords, a, b, gm)
    u = U64 if dtype == torch.float64 else U32
    base = 1e-12 if dtype == torch.float64 else 1e-5
    g = np.abs(np.stack(g_or))
    return base * np.max(g, axis=0) + 64 * u * (np.stack(list(sa) + list(sb)) + kappa * g)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("coords", ["PtEtaPhiM", "PtEtaPhiE", "PxPyPzE", "PxPyPzM"])
def test_mass_bwd_against_oracle(coords, dtype):
    n = 65536 + 3
    g = synth.rng(610)
    a, b = synth.pairs_generic(g, n)
    if coords != "PtEtaPhiM":
        ca, cb = oracle.to_cartesian("PtEtaPhiM", a), oracle.to_cartesian("PtEtaPhiM", b)
        if coords == "PxPyPzE":
            a, b = ca, cb
        elif coords == "PxPyPzM":
            a, b = (ca[0], ca[1], ca[2], a[3]), (cb[0], cb[1], cb[2], b[3])
        else:
            a, b = (a[0], a[1], a[2], ca[3]), (b[0], b[1], b[2], cb[3])
    gm = g.standard_normal(n)
    ga, gb = glv.glv_invariant_mass_bwd(gpu(a, dtype), gpu(b, dtype), gpu([gm], dtype)[0], coords=coords)
    ga, gb = host(ga), host(gb)
    wa, wb, wg = widened(a, dtype), widened(b, dtype), widened([gm], dtype)[0]
    oa, ob = oracle.mass_vjp(coords, wa, wb, wg)
    g_or = list(oa) + list(ob)
    g_gpu = [c.astype(np.float64) for c in list(ga) + list(gb)]
    err = np.abs(np.stack(g_gpu) - np.stack(g_or))
    r, i = worst(err.ravel(), _mass_vjp_tol(wa, wb, coords, dtype, g_or, wg).ravel())
    i = i % n
    assert r <= 1.0, (i, [c[i] for c in g_gpu], [c[i] for c in g_or])


def test_mass_bwd_full_size():
    """The pair mass's reverse mode on 2^24 items, every item."""
    n = 1 << 24
    g = synth.rng(synth.GRADS)
    a, b = synth.pairs_generic(g, n)
    gm = g.standard_normal(n)
    ga, gb = glv.glv_invariant_mass_bwd(gpu(a, torch.float64), gpu(b, torch.float64), gpu([gm], torch.float64)[0])
    got = np.stack([host(c) for c in list(ga) + list(gb)])
    oa, ob = oracle.mass_vjp("PtEtaPhiM", a, b, gm)
    g_or = list(oa) + list(ob)
    err = np.abs(got - np.stack(g_or))
    r, i = worst(err.ravel(), _mass_vjp_tol(a, b, "PtEtaPhiM", torch.float64, g_or, gm).ravel())
    assert r <= 1.0, (i % n, i // n)


# ------------------------------------------------------------- boost bwd

def _boost_vjp_scale(x, beta, gy):
    """Absolute-value scale of each VJP formula (same expressions on |.|)."""
    ax, ab, agy = [np.abs(c) for c in x], [np.abs(c) for c in beta], [np.abs(c) for c in gy]
    gx, gbeta = oracle.boost_vjp(ax, ab, agy)
    return gx, gbeta


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_boost_bwd_against_oracle(dtype):
    n = 65536 + 7
    g = synth.rng(620)
    x, beta = synth.boost_items(g, n)
    gy = synth.upstream(g, n, 4)
    gx, gbeta = glv.glv_boost_bwd(gpu(x, dtype), gpu(beta, dtype), gpu(gy, dtype))
    gx, gbeta = host(gx), host(gbeta)
    wx, wb, wg = widened(x, dtype), widened(beta, dtype), widened(gy, dtype)
    ox, ob = oracle.boost_vjp(wx, wb, wg)
    sx, sb = _boost_vjp_scale(wx, wb, wg)
    tolf = 1e-12 if dtype == torch.float64 else 2.0 ** -17
    for k in range(4):
        r, i = worst(np.abs(gx[k].astype(np.float64) - ox[k]), tolf * sx[k])
        assert r <= 1.0, ("gx", k, i)
    for k in range(3):
        r, i = worst(np.abs(gbeta[k].astype(np.float64) - ob[k]), tolf * sb[k])
        assert r <= 1.0, ("gbeta", k, i)


def test_boost_bwd_full_size():
    """The boost's reverse mode on 2^24 items with the benchmark's upstreams
    (the same draws, in the same order) and launch shape, every item."""
    n = 1 << 24
    x, beta = synth.boost_items(synth.rng(synth.LARGE), n)
    gr = synth.rng(synth.GRADS)
    synth.upstream(gr, n, 1)  # the mass upstream is drawn first
    gy = synth.upstream(gr, n, 4)
    gx, gbeta = glv.glv_boost_bwd(gpu(x, torch.float64), gpu(beta, torch.float64), gpu(gy, torch.float64))
    gx, gbeta = host(gx), host(gbeta)
    ox, ob = oracle.boost_vjp(x, beta, gy)
    sx, sb = _boost_vjp_scale(x, beta, gy)
    for k in range(4):
        r, i = worst(np.abs(gx[k] - ox[k]), 1e-12 * sx[k])
        assert r <= 1.0, ("gx", k, i)
    for k in range(3):
        r, i = worst(np.abs(gbeta[k] - ob[k]), 1e-12 * sb[k])
        assert r <= 1.0, ("gbeta", k, i)


def test_boost_bwd_broadcast_grad_x_only():
    n = 5000
    x, beta = synth.boost_items(synth.rng(621), n)
    one = tuple(np.array([b[0]]) for b in beta)
    gy = synth.upstream(synth.rng(622), n, 4)
    gx, gb = glv.glv_boost_bwd(gpu(x, torch.float64), gpu(one, torch.float64), gpu(gy, torch.float64),
                               want_beta=False)
    assert gb is None
    want = oracle.boost(gy, one, beta_stride=0)  # grad_x is the forward boost of grad_y
    s = oracle.boost_scale(gy, one, beta_stride=0)
    for k in range(4):
        assert np.all(np.abs(host(gx[k]) - want[k]) <= 1e-12 * s[k])


# ------------------------------------------------------------- autograd

def test_autograd_gradcheck_fp64():
    g = synth.rng(630)
    a, b = synth.pairs_generic(g, 16)
    cols = tuple(t.clone().requires_grad_(True) for t in gpu(a, torch.float64) + gpu(b, torch.float64))
    assert torch.autograd.gradcheck(lambda *c: ag.InvariantMass.apply("PtEtaPhiM", "plain", *c), cols,
                                    eps=1e-6, atol=1e-6, rtol=1e-5)
    x, beta = synth.boost_items(g, 16)
    cols = tuple(t.clone().requires_grad_(True) for t in gpu(x, torch.float64) + gpu(beta, torch.float64))
    assert torch.autograd.gradcheck(lambda *c: ag.Boost.apply(*c), cols, eps=1e-6, atol=1e-6, rtol=1e-5)


def test_autograd_mass_of_boosted_pair():
    """Chain boost -> mass through autograd; the mass is boost invariant, so
    the gradient w.r.t. beta vanishes (both legs boosted by the same beta)."""
    n = 1000
    g = synth.rng(631)
    x1, beta = synth.boost_items(g, n)
    x2, _ = synth.boost_items(g, n)
    bt = tuple(t.requires_grad_(True) for t in gpu(beta, torch.float64))
    y1 = ag.boost(gpu(x1, torch.float64), bt)
    y2 = ag.boost(gpu(x2, torch.float64), bt)
    m = ag.invariant_mass(y1, y2, coords="PxPyPzE")
    m.sum().backward()
    m_unboosted = host(glv.glv_invariant_mass(gpu(x1, torch.float64), gpu(x2, torch.float64), coords="PxPyPzE"))
    assert np.allclose(host(m), m_unboosted, rtol=1e-9)
    # each leg's share is of size (E1 + E2)^2 / m * gamma^3; they cancel
    scale = (np.abs(x1[3]) + np.abs(x2[3])) ** 2 / m_unboosted / (1.0 - sum(b * b for b in beta)) ** 1.5
    for t in bt:
        assert np.all(np.abs(host(t.grad)) <= 1e-12 * scale)


@pytest.mark.parametrize("coords", ["PtEtaPhiM", "PxPyPzE"])
def test_autograd_gradcheck_event_reduce(coords):
    """torch.autograd.gradcheck of the jagged reduction's wrapper: every
    output (totals, event masses, pair masses) against central differences,
    on events of 0 to 6 particles."""
    counts = np.array([3, 0, 1, 2, 6, 4], dtype=np.int64)
    off = np.zeros(counts.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    g = synth.rng(640)
    if coords == "PxPyPzE":
        # heavy vectors (M up to 100 GeV): with light ones E^2 - |P|^2 is so
        # curved in px that central differences at eps = 1e-6 are off by ~1e-3
        p, _ = synth.boost_items(g, int(off[-1]))
    else:
        p, _ = synth.pairs_generic(g, int(off[-1]))
    cols = tuple(t.clone().requires_grad_(True) for t in gpu(p, torch.float64))
    go = torch.from_numpy(off).to("cuda:0")
    po = glv.glv_pair_offsets(go)

    def f(*c):
        total, em, pm = ag.event_reduce(c, go, po, coords=coords)
        return (*total, em, pm)

    assert torch.autograd.gradcheck(f, cols, eps=1e-6, atol=1e-6, rtol=1e-5)


@pytest.mark.parametrize("n", [1, 2, 3, 65, 1001])
def test_bwd_misaligned_views_match_aligned(n):
    """The mass and boost reverse modes on views one element in (not 16-byte
    aligned: one item per lane) give bitwise the same gradients as the aligned
    vector path on the overlapping items."""
    a, b = synth.pairs_generic(synth.rng(630 + n), n + 1)
    gm = synth.upstream(synth.rng(631 + n), n + 1, 1)[0]
    ga, gb, ggm = gpu(a, torch.float64), gpu(b, torch.float64), gpu([gm], torch.float64)[0]
    full = glv.glv_invariant_mass_bwd(ga, gb, ggm)
    part = glv.glv_invariant_mass_bwd(tuple(t[1:] for t in ga), tuple(t[1:] for t in gb), ggm[1:])
    for leg_f, leg_p in zip(full, part):
        for cf, cp in zip(leg_f, leg_p):
            assert torch.equal(cf[1:], cp)
    x, beta = synth.boost_items(synth.rng(632 + n), n + 1)
    gy = synth.upstream(synth.rng(633 + n), n + 1, 4)
    gx, gbeta, ggy = gpu(x, torch.float64), gpu(beta, torch.float64), gpu(gy, torch.float64)
    fx, fb = glv.glv_boost_bwd(gx, gbeta, ggy)
    px, pb = glv.glv_boost_bwd(tuple(t[1:] for t in gx), tuple(t[1:] for t in gbeta), tuple(t[1:] for t in ggy))
    for cf, cp in zip(list(fx) + list(fb), list(px) + list(pb)):
        assert torch.equal(cf[1:], cp)
