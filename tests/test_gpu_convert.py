"""GPU parity of the stand-alone coordinate conversion (Sec. 3.1) and its
reverse mode against the oracle, for every pair of systems."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import gpu, host, widened
from tolerances import U32, U64, worst

pytestmark = pytest.mark.gpu
glv = pytest.importorskip("paper_2312_02756_amd.glv")

SYSTEMS = ["PxPyPzE", "PtEtaPhiM", "PtEtaPhiE", "PxPyPzM"]


def _vectors(n, seed, system):
    """Vectors in `system`: pt >= 1 GeV, |eta| <= 2.5, masses of 0.5-90 GeV
    (a fifth spacelike when given as PxPyPzE)."""
    g = synth.rng(seed)
    a, _ = synth.pairs_generic(g, n)
    m = g.uniform(0.5, 90.0, n)
    ptm = (a[0] + 1.0, a[1], a[2], m)
    cols = oracle.convert("PtEtaPhiM", system, ptm)
    if system == "PxPyPzE":
        p2 = cols[0] ** 2 + cols[1] ** 2 + cols[2] ** 2
        space = g.random(n) < 0.2
        mm = np.minimum(m, 0.9 * np.sqrt(p2))
        cols = (cols[0], cols[1], cols[2], np.where(space, np.sqrt(p2 - mm * mm), cols[3]))
    return cols


def _tol(dst, want, cart_or, u):
    """Per component of the target system: 16 u times the component's own
    scale (pt; 1 + |eta|; pi; |M| + S / (2|M|) with S = E^2 + |p|^2, the
    cancellation in E^2 - |p|^2; E; the largest Cartesian component)."""
    S = cart_or[3] ** 2 + cart_or[0] ** 2 + cart_or[1] ** 2 + cart_or[2] ** 2
    am = np.maximum(np.abs(want[3]), 1e-300)
    if dst in ("PxPyPzE", "PxPyPzM"):
        big = np.max(np.abs(np.stack(cart_or)), axis=0)
        scales = (big, big, big, np.abs(want[3]) if dst == "PxPyPzE" else am + S / (2 * am))
    else:
        last = am + S / (2 * am) if dst == "PtEtaPhiM" else np.abs(want[3])
        scales = (np.abs(want[0]), 1 + np.abs(want[1]), np.full(want[0].shape, np.pi), last)
    return [16 * u * s + 1e-300 for s in scales]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("src", SYSTEMS)
@pytest.mark.parametrize("dst", SYSTEMS)
def test_convert_against_oracle(src, dst, dtype):
    n = 4097
    cols = _vectors(n + 1, 900 + SYSTEMS.index(src), src)
    u = U64 if dtype == torch.float64 else U32
    gc = gpu(cols, dtype)
    for sl, view in ((slice(0, n), tuple(t[:n] for t in gc)), (slice(1, n + 1), tuple(t[1:] for t in gc))):
        got = [host(c).astype(np.float64) for c in glv.glv_convert(view, src, dst)]
        w = widened(tuple(c[sl] for c in cols), dtype)
        want = oracle.convert(src, dst, w)
        if src == dst:
            assert all(np.array_equal(g_, w_) for g_, w_ in zip(got, w))
            continue
        tol = _tol(dst, want, oracle.convert(src, "PxPyPzE", w), u)
        for k in range(4):
            r, i = worst(np.abs(got[k] - want[k]), tol[k])
            assert r <= 1.0, (src, dst, k, i, got[k][i], want[k][i])


def test_convert_in_place_and_beam_axis():
    cols = _vectors(1000, 910, "PtEtaPhiM")
    gc = gpu(cols, torch.float64)
    ref = glv.glv_convert(gc, "PtEtaPhiM", "PxPyPzE")
    same = glv.glv_convert(gc, "PtEtaPhiM", "PxPyPzE", out=gc)
    assert all(torch.equal(a, b) for a, b in zip(ref, same)) and same[0].data_ptr() == gc[0].data_ptr()
    axis = tuple(torch.tensor(v, dtype=torch.float64, device="cuda:0") for v in
                 ([0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [5.0, -5.0, 0.0], [6.0, 6.0, 1.0]))
    pt, eta, phi, m = (host(c) for c in glv.glv_convert(axis, "PxPyPzE", "PtEtaPhiM"))
    assert pt.tolist() == [0.0, 0.0, 0.0] and eta.tolist() == [np.inf, -np.inf, 0.0]
    assert np.allclose(m, [np.sqrt(11.0), np.sqrt(11.0), 1.0], rtol=1e-15)


def _kappa(src, dst, cols):
    """Conditioning of an item's gradient: S / M^2 where a side given with M
    (PtEtaPhiM, PxPyPzM) forms M from E^2 - |p|^2, else 1."""
    if "PtEtaPhiM" not in (src, dst) and "PxPyPzM" not in (src, dst):
        return np.ones(cols[0].size)
    v = oracle.convert(src, "PxPyPzE", cols)
    S = v[3] ** 2 + v[0] ** 2 + v[1] ** 2 + v[2] ** 2
    q = np.abs(v[3] ** 2 - v[0] ** 2 - v[1] ** 2 - v[2] ** 2)
    return S / np.maximum(q, 1e-300)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("src", SYSTEMS)
@pytest.mark.parametrize("dst", SYSTEMS)
def test_convert_bwd_against_oracle(src, dst, dtype):
    n = 2049
    cols = _vectors(n, 920 + SYSTEMS.index(src), src)
    g = tuple(synth.rng(921).normal(size=n) for _ in range(4))
    got = [host(c).astype(np.float64) for c in glv.glv_convert_bwd(gpu(cols, dtype), gpu(g, dtype), src, dst)]
    w, wg = widened(cols, dtype), widened(g, dtype)
    want = oracle.convert_vjp(src, dst, w, wg)
    if src == dst:
        assert all(np.array_equal(a, b) for a, b in zip(got, wg))
        return
    u = U64 if dtype == torch.float64 else U32
    base = 1e-12 if dtype == torch.float64 else 1e-5
    ref = np.max(np.abs(np.stack(want)), axis=0)
    tol = (base + 64 * u * _kappa(src, dst, w)) * ref + 1e-300
    for k in range(4):
        r, i = worst(np.abs(got[k] - want[k]), tol)
        assert r <= 1.0, (src, dst, k, i, got[k][i], want[k][i])


def test_convert_full_size_sampled():
    """2^24 FP64 vectors PtEtaPhiM -> PxPyPzE -> PtEtaPhiM and the reverse
    mode of the second step, in the measured launch shape; 65,536 samples."""
    n = 1 << 24
    a, _ = synth.pairs_generic(synth.rng(synth.LARGE), n)
    ga = gpu(a, torch.float64)
    cart = glv.glv_convert(ga, "PtEtaPhiM", "PxPyPzE")
    back = [host(c) for c in glv.glv_convert(cart, "PxPyPzE", "PtEtaPhiM")]
    gup = gpu(synth.upstream(synth.rng(synth.GRADS), n, 4), torch.float64)
    gr = [host(c) for c in glv.glv_convert_bwd(cart, gup, "PxPyPzE", "PtEtaPhiM")]
    cart = [host(c) for c in cart]
    idx = np.sort(np.random.default_rng(12).choice(n, 65536, replace=False))
    cs = tuple(c[idx] for c in cart)
    want = oracle.convert("PxPyPzE", "PtEtaPhiM", cs)
    tol = _tol("PtEtaPhiM", want, cs, U64)
    for k in range(4):
        r, i = worst(np.abs(back[k][idx] - want[k]), tol[k])
        assert r <= 1.0, ("fwd", k, i)
    gs = tuple(host(c)[idx] for c in gup)
    wv = oracle.convert_vjp("PxPyPzE", "PtEtaPhiM", cs, gs)
    ref = np.max(np.abs(np.stack(wv)), axis=0)
    tolg = (1e-12 + 64 * U64 * _kappa("PxPyPzE", "PtEtaPhiM", cs)) * ref + 1e-300
    for k in range(4):
        r, i = worst(np.abs(gr[k][idx] - wv[k]), tolg)
        assert r <= 1.0, ("bwd", k, i)
