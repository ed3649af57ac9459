"""GPU parity of the jagged per-event reduction (one launch: totals, event
mass, all pair masses), its reverse mode, the pair-offset scan, the offset
check and the autotuner, against the CPU oracle."""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import event_abs_scale, gpu, host, widened
from tolerances import U32, U64, mass_tol_comp_f32, mass_tol_f32, mass_tol_f64, worst

pytestmark = pytest.mark.gpu

glv = pytest.importorskip("paper_2312_02756_amd.glv")

DEV = "cuda:0"


def _off(off):
    return torch.from_numpy(off).to(DEV)


def _events(ne, seed, mean=8.0, cap=64):
    return synth.jagged_events(synth.rng(seed), ne, mean=mean, cap=cap)


def _pairs_or(off, p, coords, accurate=False):
    """Oracle pair masses and their scales by brute force over i < j."""
    ii, jj = [np.zeros(0, dtype=np.int64)], [np.zeros(0, dtype=np.int64)]
    for e in range(off.size - 1):
        n = int(off[e + 1] - off[e])
        if n >= 2:
            r, c = np.triu_indices(n, 1)  # row-major upper triangle: lexicographic i < j
            ii.append(off[e] + r)
            jj.append(off[e] + c)
    ii, jj = np.concatenate(ii), np.concatenate(jj)
    a, b = tuple(c[ii] for c in p), tuple(c[jj] for c in p)
    if accurate:
        return oracle.mass_accurate(a, b), None
    return oracle.mass_plain(coords, a, b, scale=True)


def _check_forward(off, p, dtype, coords, mode, total, em, pm, label):
    wp = widened(p, dtype)
    tot_or, em_or, pm_or, po = oracle.event_reduce(coords, off, wp,
                                                   mode=oracle.ACCURATE if mode == "compensated" else oracle.PLAIN)
    cart = oracle.to_cartesian(coords, wp)
    S_abs, sums = event_abs_scale(cart, off)
    n = np.maximum(np.diff(off), 1)
    u = U64 if dtype == torch.float64 else U32
    # totals
    for k in range(4):
        tol = (1e-12 * sums[k]) if dtype == torch.float64 else (4 * U32 * sums[k] + U32 * np.abs(tot_or[k]))
        r, i = worst(np.abs(host(total[k]).astype(np.float64) - tot_or[k]), tol + 1e-300)
        assert r <= 1.0, (label, "total", k, i)
    # event masses
    if mode == "compensated":
        tol = mass_tol_comp_f32(em_or) if dtype == torch.float32 else 64 * U64 * em_or + 1e-300
    else:
        tol = 1e-12 * np.abs(em_or) + 64 * u * n * S_abs / (2 * np.maximum(np.abs(em_or), 1e-300))
        if dtype == torch.float32:
            tol = tol + 1e-5 * np.abs(em_or)
    r, i = worst(np.abs(host(em).astype(np.float64) - em_or), tol)
    assert r <= 1.0, (label, "event_m", i, host(em)[i], em_or[i], off[i], off[i + 1])
    # pair masses
    assert pm.numel() == pm_or.size
    if mode == "compensated":
        tol = mass_tol_comp_f32(pm_or) if dtype == torch.float32 else 64 * U64 * pm_or + 1e-300
    else:
        _, s = _pairs_or(off, wp, coords)
        tol = mass_tol_f64(pm_or, s) if dtype == torch.float64 else mass_tol_f32(pm_or, s)
    r, i = worst(np.abs(host(pm).astype(np.float64) - pm_or), tol)
    assert r <= 1.0, (label, "pair_m", i)
    return po


def test_pair_offsets_bitwise():
    for ne in (0, 1, 5, 4095, 4096, 4097, 100000):
        off, _ = _events(ne, 700 + ne)
        po = host(glv.glv_pair_offsets(_off(off)))
        assert np.array_equal(po, oracle.pair_offsets(off)), ne


def test_validate_offsets():
    off, p = _events(1000, 701)
    assert int(glv.glv_validate_offsets(_off(off), p[0].size).item()) == 0
    bad = off.copy()
    bad[10], bad[11] = bad[11] + 5, bad[10]  # not monotone
    assert int(glv.glv_validate_offsets(_off(bad), p[0].size).item()) > 0
    assert int(glv.glv_validate_offsets(_off(off), p[0].size + 1).item()) == 1


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("coords", ["PtEtaPhiM", "PxPyPzE", "PtEtaPhiE", "PxPyPzM"])
def test_event_reduce_plain(coords, dtype):
    off, p = _events(3000, 702)
    if coords != "PtEtaPhiM":
        c = oracle.to_cartesian("PtEtaPhiM", p)
        p = {"PxPyPzE": c, "PtEtaPhiE": (p[0], p[1], p[2], c[3]), "PxPyPzM": (c[0], c[1], c[2], p[3])}[coords]
    total, em, pm = glv.glv_event_reduce(gpu(p, dtype), _off(off), coords=coords)
    _check_forward(off, p, dtype, coords, "plain", total, em, pm, f"{coords} {dtype}")


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_event_reduce_compensated(dtype):
    off, p = _events(3000, 703)
    fb = torch.zeros(1, dtype=torch.int64, device=DEV)
    total, em, pm = glv.glv_event_reduce(gpu(p, dtype), _off(off), mode="compensated", fallback_count=fb)
    _check_forward(off, p, dtype, "PtEtaPhiM", "compensated", total, em, pm, f"comp {dtype}")


def test_event_reduce_edge_events():
    """Empty events, single particles, events larger than the LDS capacity
    (handled from global memory) and a trailing empty event."""
    counts = np.array([0, 1, 2, 0, 3, 700, 64, 0, 1, 65, 1500, 2, 0], dtype=np.int64)
    off = np.zeros(counts.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    a, _ = synth.pairs_generic(synth.rng(704), int(off[-1]))
    for dtype in (torch.float64, torch.float32):
        for tiling in (None, (128, 4, 512, 64), (64, 1, 64, 64), (128, 13, 256, 1024)):
            total, em, pm = glv.glv_event_reduce(gpu(a, dtype), _off(off), tiling=tiling)
            _check_forward(off, a, dtype, "PtEtaPhiM", "plain", total, em, pm, f"edge {dtype} {tiling}")
        total, em, pm = glv.glv_event_reduce(gpu(a, torch.float32), _off(off), mode="compensated",
                                             tiling=(128, 8, 256, 192))
        _check_forward(off, a, torch.float32, "PtEtaPhiM", "compensated", total, em, pm, "edge comp")


def test_tilings_give_identical_pair_masses_and_totals():
    off, p = _events(20000, 705)
    gp, go = gpu(p, torch.float64), _off(off)
    ref = None
    for tiling in [(256, 64, 128, 512), (128, 32, 256, 256), (64, 64, 512, 1024), (256, 17, 64, 64),
                   (512, 5, 128, 192)]:
        total, em, pm = glv.glv_event_reduce(gp, go, tiling=tiling)
        out = [host(pm)] + [host(t) for t in total] + [host(em)]
        if ref is None:
            ref = out
        else:
            for u, v in zip(out, ref):
                assert np.array_equal(u, v), tiling
    # compensated FP32: pair masses identical; event masses reproducible per tiling
    gp32 = gpu(p, torch.float32)
    ref = None
    for tiling in [(256, 64, 128, 512), (128, 32, 256, 256), (512, 7, 64, 128)]:
        _, em1, pm1 = glv.glv_event_reduce(gp32, go, mode="compensated", tiling=tiling)
        _, em2, pm2 = glv.glv_event_reduce(gp32, go, mode="compensated", tiling=tiling)
        assert torch.equal(em1, em2) and torch.equal(pm1, pm2)
        if ref is None:
            ref = host(pm1)
        else:
            assert np.array_equal(host(pm1), ref), tiling


def _quad_order_total(x):
    """((P0 + P1) + (P2 + P3)) in binary64, P_r the index-order sum of the
    event's values whose index is r mod 4: the documented order of the GPU's
    event totals."""
    parts = []
    for r in range(4):
        acc = 0.0
        for v in x[r::4]:
            acc = acc + float(v)
        parts.append(acc)
    return (parts[0] + parts[1]) + (parts[2] + parts[3])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_event_totals_follow_the_documented_order(dtype):
    """Cartesian inputs (staged as given), events of 0 to 64 particles: every
    total is bitwise the four residue-class sums combined as documented (FP32
    data summed in binary64, then rounded), for two tilings."""
    g = synth.rng(741)
    counts = np.concatenate([np.minimum(g.poisson(9, 3000), 64), [0, 1, 2, 3, 4, 5, 63, 64]]).astype(np.int64)
    off = np.zeros(counts.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    n = int(off[-1])
    # cancellation-prone sums: mixed signs and magnitudes
    cols = [g.standard_normal(n) * np.exp(g.uniform(-8, 8, n)) for _ in range(4)]
    pg = gpu(cols, dtype)
    vals = [host(c).astype(np.float64) for c in pg]
    for tiling in (None, (128, 16, 128, 256)):
        total, _, _ = glv.glv_event_reduce(pg, _off(off), coords="PxPyPzE", want_event_m=False, want_pair_m=False,
                                           tiling=tiling)
        got = [host(t) for t in total]
        for k in range(4):
            want = np.array([_quad_order_total(vals[k][off[e]:off[e + 1]]) for e in range(counts.size)])
            want = want.astype(np.float32) if dtype == torch.float32 else want
            assert np.array_equal(got[k], want), (tiling, k)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_tiny_events_take_several_total_passes(dtype):
    """Events of 0 to 6 particles: a chunk then holds up to 64 events, whose
    totals take four passes of 16 quads; the totals keep the documented order
    and the compensated event masses (sum of M^2 handed from each pass's
    quads to the event lanes) stay within the oracle's bound."""
    off, p = _events(4000, 742, mean=1.5, cap=6)
    pg, og = gpu(p, dtype), _off(off)
    for tiling in (None, (128, 64, 128, 256), (64, 64, 256, 128)):
        total, em, pm = glv.glv_event_reduce(pg, og, mode="compensated", tiling=tiling)
        _check_forward(off, p, dtype, "PtEtaPhiM", "compensated", total, em, pm, f"tiny comp {dtype} {tiling}")
    c = oracle.to_cartesian("PtEtaPhiM", widened(p, dtype))
    cg = gpu(c, dtype)
    vals = [host(x).astype(np.float64) for x in cg]
    total, _, _ = glv.glv_event_reduce(cg, og, coords="PxPyPzE", want_event_m=False, want_pair_m=False,
                                       tiling=(128, 64, 128, 256))
    for k in range(4):
        want = np.array([_quad_order_total(vals[k][off[e]:off[e + 1]]) for e in range(off.size - 1)])
        want = want.astype(np.float32) if dtype == torch.float32 else want
        assert np.array_equal(host(total[k]), want), k


def test_event_reduce_full_size_sampled():
    """2^20 events (Poisson(8), clipped at 64) in the benchmark's launch shape;
    a sample of events checked against the oracle, every pair of each."""
    off, p = _events(1 << 20, synth.JAGGED)
    po_all = oracle.pair_offsets(off)
    for dtype, mode in ((torch.float64, "plain"), (torch.float32, "compensated")):
        total, em, pm = glv.glv_event_reduce(gpu(p, dtype), _off(off), mode=mode)
        total, em, pm = host(total), host(em), host(pm)
        assert pm.size == po_all[-1]
        sel = np.sort(np.random.default_rng(11).choice(off.size - 1, 20000, replace=False))
        # rebuild a compact CSR of the sampled events
        cnt = off[sel + 1] - off[sel]
        soff = np.zeros(sel.size + 1, dtype=np.int64)
        soff[1:] = np.cumsum(cnt)
        pidx = np.concatenate([np.arange(off[e], off[e + 1]) for e in sel])
        sp = tuple(c[pidx] for c in p)
        pair_idx = np.concatenate([np.arange(po_all[e], po_all[e + 1]) for e in sel])
        stot = tuple(torch.from_numpy(t[sel]) for t in total)
        _check_forward(soff, sp, dtype, "PtEtaPhiM", mode, stot, torch.from_numpy(em[sel]),
                       torch.from_numpy(pm[pair_idx]), f"full {mode}")


def test_event_reduce_bwd_full_size_sampled():
    """The reverse mode on 2^20 events with the benchmark's upstreams and launch
    shape; the gradients of every particle of 5,000 sampled events checked
    against the oracle's VJP of those events alone (an event's gradients
    depend only on its own particles and upstreams)."""
    off, p = _events(1 << 20, synth.JAGGED)
    ne = off.size - 1
    po_all = oracle.pair_offsets(off)
    gj = synth.rng(synth.JAGGED_GRADS)
    g_tot = synth.upstream(gj, ne, 4)
    g_em = synth.upstream(gj, ne, 1)[0]
    g_pair = synth.upstream(gj, int(po_all[-1]), 1)[0]
    got = glv.glv_event_reduce_bwd(gpu(p, torch.float64), _off(off), grad_total=gpu(g_tot, torch.float64),
                                   grad_event_m=gpu([g_em], torch.float64)[0],
                                   grad_pair_m=gpu([g_pair], torch.float64)[0])
    got = [host(c) for c in got]
    sel = np.sort(np.random.default_rng(13).choice(ne, 5000, replace=False))
    cnt = off[sel + 1] - off[sel]
    soff = np.zeros(sel.size + 1, dtype=np.int64)
    soff[1:] = np.cumsum(cnt)
    pidx = np.concatenate([np.arange(off[e], off[e + 1]) for e in sel])
    qidx = np.concatenate([np.arange(po_all[e], po_all[e + 1]) for e in sel])
    sp = tuple(c[pidx] for c in p)
    want = oracle.event_reduce_vjp("PtEtaPhiM", soff, sp, tuple(t[sel] for t in g_tot), g_em[sel], g_pair[qidx])
    _check_bwd(soff, sp, torch.float64, "PtEtaPhiM", [c[pidx] for c in got], want, "full size")


def test_autotune_picks_a_valid_tiling():
    off, p = _events(1 << 16, 706)
    gp, go = gpu(p, torch.float64), _off(off)
    best = glv.glv_autotune_event_reduce(gp, go)
    assert best[0] in (64, 128, 256, 512) and 1 <= best[1] <= 64 and best[3] % 64 == 0, best
    assert glv.glv_current_tiling(torch.float64, "PtEtaPhiM", "plain") == best
    total, em, pm = glv.glv_event_reduce(gp, go)
    _, em2, pm2 = glv.glv_event_reduce(gp, go, tiling=best)
    assert torch.equal(pm, pm2) and torch.equal(em, em2)


# ---------------------------------------------------------------- backward

def _check_bwd(off, wp, dtype, coords, got, want, label):
    """Per particle: the largest error over its 4 gradient components against
    (base + 64 u kappa) times the largest oracle component, with kappa the
    worst conditioning S/m^2 of its event's mass and pair masses times n."""
    ne = off.size - 1
    po = oracle.pair_offsets(off)
    S_abs, _ = event_abs_scale(oracle.to_cartesian(coords, wp), off)
    u = U64 if dtype == torch.float64 else U32
    base = 1e-12 if dtype == torch.float64 else 1e-5
    cnt = np.diff(off)
    ev = np.repeat(np.arange(ne), cnt)
    _, em_or, pm_or, _ = oracle.event_reduce(coords, off, wp)
    kappa_ev = S_abs / np.maximum(em_or ** 2, 1e-300)
    _, s_pairs = _pairs_or(off, wp, coords)
    kp = s_pairs / np.maximum(pm_or ** 2, 1e-300)
    kappa_pair_ev = np.zeros(ne)
    np.maximum.at(kappa_pair_ev, np.repeat(np.arange(ne), np.diff(po)), kp)
    kappa = np.maximum(kappa_ev, kappa_pair_ev)[ev] * np.maximum(cnt[ev], 1)
    err = np.max(np.abs(np.stack(got) - np.stack(want)), axis=0)
    ref = np.max(np.abs(np.stack(want)), axis=0)
    r, i = worst(err, (base + 64 * u * kappa) * ref + 1e-300)
    assert r <= 1.0, (label, i, [c[i] for c in got], [c[i] for c in want])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("coords", ["PtEtaPhiM", "PxPyPzE", "PxPyPzM"])
def test_event_reduce_bwd(coords, dtype):
    counts = np.concatenate([np.minimum(synth.rng(707).poisson(8, 2000), 64), [0, 1, 300, 2]]).astype(np.int64)
    off = np.zeros(counts.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    g = synth.rng(708)
    p, _ = synth.pairs_generic(g, int(off[-1]))
    if coords != "PtEtaPhiM":
        c = oracle.to_cartesian("PtEtaPhiM", p)
        p = c if coords == "PxPyPzE" else (c[0], c[1], c[2], p[3])
    ne = counts.size
    po = oracle.pair_offsets(off)
    gt = synth.upstream(g, ne, 4)
    gem = g.standard_normal(ne)
    gpr = g.standard_normal(int(po[-1]))
    wp = widened(p, dtype)
    want = oracle.event_reduce_vjp(coords, off, wp, widened(gt, dtype), widened([gem], dtype)[0],
                                   widened([gpr], dtype)[0])
    for tiling in (None, (128, 16, 128)):
        got = glv.glv_event_reduce_bwd(gpu(p, dtype), _off(off), grad_total=gpu(gt, dtype),
                                       grad_event_m=gpu([gem], dtype)[0], grad_pair_m=gpu([gpr], dtype)[0],
                                       coords=coords, tiling=tiling)
        _check_bwd(off, wp, dtype, coords, [host(c).astype(np.float64) for c in got], want, tiling)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("coords", ["PtEtaPhiM", "PxPyPzE", "PxPyPzM"])
def test_event_reduce_bwd_with_forward_totals(coords, dtype):
    """The reverse mode fed the forward's event totals: bitwise the
    recomputing call on every event both launches stage (the same order of
    summation), within the oracle's bound on the rest (a 300-particle event beyond
    the staged capacity of the small tiling)."""
    counts = np.concatenate([np.minimum(synth.rng(717).poisson(8, 1500), 64), [0, 1, 300, 2, 0]]).astype(np.int64)
    off = np.zeros(counts.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    g = synth.rng(718)
    p, _ = synth.pairs_generic(g, int(off[-1]))
    if coords != "PtEtaPhiM":
        c = oracle.to_cartesian("PtEtaPhiM", p)
        p = c if coords == "PxPyPzE" else (c[0], c[1], c[2], p[3])
    ne = counts.size
    po = oracle.pair_offsets(off)
    gt = synth.upstream(g, ne, 4)
    gem = g.standard_normal(ne)
    gpr = g.standard_normal(int(po[-1]))
    wp = widened(p, dtype)
    want = oracle.event_reduce_vjp(coords, off, wp, widened(gt, dtype), widened([gem], dtype)[0],
                                   widened([gpr], dtype)[0])
    pg, og = gpu(p, dtype), _off(off)
    small = np.repeat(counts <= 64, counts)
    for tiling in (None, (128, 16, 128)):
        tot, _, _ = glv.glv_event_reduce(pg, og, coords=coords, want_event_m=False, want_pair_m=False,
                                         tiling=tiling)
        for with_gt, with_gpr in ((True, True), (False, False)):
            kw = dict(grad_total=gpu(gt, dtype) if with_gt else None, grad_event_m=gpu([gem], dtype)[0],
                      grad_pair_m=gpu([gpr], dtype)[0] if with_gpr else None, coords=coords, tiling=tiling)
            ref = [host(c) for c in glv.glv_event_reduce_bwd(pg, og, **kw)]
            got = [host(c) for c in glv.glv_event_reduce_bwd(pg, og, total=tot, **kw)]
            for k in range(4):
                np.testing.assert_array_equal(got[k][small], ref[k][small], err_msg=f"{tiling} {with_gt} col {k}")
            if with_gt and with_gpr:
                _check_bwd(off, wp, dtype, coords, [c.astype(np.float64) for c in got], want, tiling)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_event_reduce_bwd_pair_cap_and_missing_upstreams(dtype):
    """Events of 40-50 particles against a tiling of 256 staged particles and
    1024 staged pair gradients: the pair cap, not the particle cap, ends the
    chunks, and 50-particle events (1225 pairs) take the separate path; with
    128 staged particles and 512 pair gradients every event of 40 or more takes
    it.  Also without pair upstreams (no pair offsets needed) and without any
    upstream."""
    counts = np.array([40, 3, 50, 0, 45, 1, 2, 40, 41, 50, 7, 44] * 6, dtype=np.int64)
    off = np.zeros(counts.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    g = synth.rng(709)
    p, _ = synth.pairs_generic(g, int(off[-1]))
    ne = counts.size
    po = oracle.pair_offsets(off)
    gt = synth.upstream(g, ne, 4)
    gem = g.standard_normal(ne)
    gpr = g.standard_normal(int(po[-1]))
    wp = widened(p, dtype)
    S_abs, _ = event_abs_scale(oracle.to_cartesian("PtEtaPhiM", wp), off)
    em_or = oracle.event_reduce("PtEtaPhiM", off, wp)[1]
    _, s_pairs = _pairs_or(off, wp, "PtEtaPhiM")
    pm_or = oracle.event_reduce("PtEtaPhiM", off, wp)[2]
    kp = s_pairs / np.maximum(pm_or ** 2, 1e-300)
    kappa_pair_ev = np.zeros(ne)
    np.maximum.at(kappa_pair_ev, np.repeat(np.arange(ne), np.diff(po)), kp)
    cnt = np.diff(off)
    ev = np.repeat(np.arange(ne), cnt)
    kappa = np.maximum(S_abs / np.maximum(em_or ** 2, 1e-300), kappa_pair_ev)[ev] * np.maximum(cnt[ev], 1)
    u = U64 if dtype == torch.float64 else U32
    base = 1e-12 if dtype == torch.float64 else 1e-5
    cases = [(gt, gem, gpr), (gt, gem, None), (None, None, None)]
    for c_gt, c_gem, c_gpr in cases:
        want = oracle.event_reduce_vjp("PtEtaPhiM", off, wp,
                                       None if c_gt is None else widened(c_gt, dtype),
                                       None if c_gem is None else widened([c_gem], dtype)[0],
                                       None if c_gpr is None else widened([c_gpr], dtype)[0])
        for tiling in ((64, 64, 256, 1024), (128, 16, 128, 512), None):
            got = glv.glv_event_reduce_bwd(
                gpu(p, dtype), _off(off), grad_total=None if c_gt is None else gpu(c_gt, dtype),
                grad_event_m=None if c_gem is None else gpu([c_gem], dtype)[0],
                grad_pair_m=None if c_gpr is None else gpu([c_gpr], dtype)[0], tiling=tiling)
            got = np.stack([host(c).astype(np.float64) for c in got])
            want_s = np.stack(want)
            if c_gt is None and c_gem is None and c_gpr is None:
                assert np.array_equal(got, np.zeros_like(got)), tiling
                continue
            err = np.max(np.abs(got - want_s), axis=0)
            ref = np.max(np.abs(want_s), axis=0)
            r, i = worst(err, (base + 64 * u * kappa) * ref + 1e-300)
            assert r <= 1.0, (tiling, c_gpr is None, i, got[:, i], want_s[:, i])


def test_event_reduce_compensated_fp64_redo():
    """Heavy, slow particles (M ~ U[5, 20] GeV, pt ~ LogUniform[0.01, 10] GeV,
    eta ~ U[-4, 4]): pairs at opposite large |eta| exceed the FP32 error bound,
    so their events take the FP64 redo.  Masses against the accurate oracle, a
    non-zero fallback count, and the same pair and event masses whichever of
    them are requested (the redo marks an event through its mass, or through
    its first pair mass when event masses are not wanted)."""
    g = synth.rng(711)
    counts = np.concatenate([np.minimum(g.poisson(6, 1500), 40), [0, 1, 2]]).astype(np.int64)
    off = np.zeros(counts.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    n = int(off[-1])
    p = (np.exp(g.uniform(np.log(0.01), np.log(10.0), n)), g.uniform(-4, 4, n), g.uniform(-np.pi, np.pi, n),
         g.uniform(5.0, 20.0, n))
    wp = widened(p, torch.float32)
    _, em_or, pm_or, _ = oracle.event_reduce("PtEtaPhiM", off, wp, mode=oracle.ACCURATE)
    gp, go = gpu(p, torch.float32), _off(off)
    runs = {}
    for want_e, want_p in ((True, True), (False, True), (True, False)):
        fb = torch.zeros(1, dtype=torch.int64, device=DEV)
        _, em, pm = glv.glv_event_reduce(gp, go, mode="compensated", want_event_m=want_e, want_pair_m=want_p,
                                         fallback_count=fb)
        assert 0 < int(fb.item()) < pm_or.size, (want_e, want_p, int(fb.item()))
        if want_e:
            r, i = worst(np.abs(host(em).astype(np.float64) - em_or), mass_tol_comp_f32(em_or))
            assert r <= 1.0, ("event_m", want_p, i, host(em)[i], em_or[i])
        if want_p:
            r, i = worst(np.abs(host(pm).astype(np.float64) - pm_or), mass_tol_comp_f32(pm_or))
            assert r <= 1.0, ("pair_m", want_e, i, host(pm)[i], pm_or[i])
        runs[(want_e, want_p)] = (host(em) if want_e else None, host(pm) if want_p else None)
    assert np.array_equal(runs[(True, True)][1], runs[(False, True)][1])
    assert np.array_equal(runs[(True, True)][0], runs[(True, False)][0])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_event_reduce_misaligned_pair_output(dtype):
    """Pair masses written through the C-ABI to an address one element past an
    aligned one (the compensated mode stores a lane's two masses at once where
    the address allows): the same values as into an aligned buffer."""
    from paper_2312_02756_amd import _lib
    off, p = _events(3000, 717)
    gp, go = gpu(p, dtype), _off(off)
    po = glv.glv_pair_offsets(go)
    npairs = int(po[-1].item())
    lib = _lib.load()
    stream = torch.cuda.current_stream().cuda_stream
    dt = _lib.GLV_F32 if dtype == torch.float32 else _lib.GLV_F64
    for mode in (_lib.GLV_PLAIN, _lib.GLV_COMPENSATED):
        outs = []
        for shift in (0, 1):
            buf = torch.full((npairs + 2,), -1.0, dtype=dtype, device=DEV)
            em = torch.empty(go.numel() - 1, dtype=dtype, device=DEV)
            rc = lib.glv_event_reduce(dt, _lib.GLV_PTETAPHIM, mode, go.numel() - 1, go.data_ptr(), po.data_ptr(),
                                      _lib.P4(*[c.data_ptr() for c in gp]), None, em.data_ptr(),
                                      buf.data_ptr() + shift * buf.element_size(), None, None, stream)
            assert rc == 0
            b = host(buf)
            assert np.all(b[:shift] == -1.0) and np.all(b[shift + npairs:] == -1.0), (mode, shift)
            outs.append((b[shift:shift + npairs], host(em)))
        assert np.array_equal(outs[0][0], outs[1][0]), mode
        assert np.array_equal(outs[0][1], outs[1][1]), mode


def test_large_event_pair_masses_match_across_paths():
    """Events of 300 and 120 particles: under a 256-particle tiling the first
    goes to the separate large-event launch, under a 1024-particle tiling both
    are staged.  Plain FP64 pair masses are bitwise identical either way; in
    the compensated FP32 mode the separate launch fuses the arithmetic
    differently, so a few pair masses of the large event may differ (within
    2^-18 relative, the FP64-redo threshold) and none of the staged event's.
    Both runs are checked against the oracle."""
    counts = np.array([3, 300, 5, 0, 120, 2, 1, 9], dtype=np.int64)
    off = np.zeros(counts.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    p, _ = synth.pairs_generic(synth.rng(719), int(off[-1]))
    go = _off(off)
    for dtype, mode in ((torch.float64, "plain"), (torch.float32, "compensated")):
        gp = gpu(p, dtype)
        runs = [glv.glv_event_reduce(gp, go, mode=mode, tiling=t) for t in ((128, 64, 256, 512), (64, 64, 1024, 512))]
        a, b = host(runs[0][2]).astype(np.float64), host(runs[1][2]).astype(np.float64)
        if mode == "plain":
            assert np.array_equal(a, b)
        else:
            po = oracle.pair_offsets(off)
            diff = np.nonzero(a != b)[0]
            assert diff.size <= a.size // 1000, diff.size
            assert np.all((diff >= po[1]) & (diff < po[2])), "only the 300-particle event"
            assert np.all(np.abs(a[diff] - b[diff]) <= 2.0 ** -18 * np.abs(b[diff]))
        _check_forward(off, p, dtype, "PtEtaPhiM", mode, *runs[0], "large via separate launch")
        _check_forward(off, p, dtype, "PtEtaPhiM", mode, *runs[1], "large staged")


def test_autotune_bwd_picks_a_valid_tiling():
    """The backward's autotuner returns one of its candidates, makes it the
    current backward tiling, and a launch with the default (now the tuned
    one) equals a launch with that tiling given explicitly."""
    off, p = _events(1 << 16, 721)
    gp, go = gpu(p, torch.float64), _off(off)
    g = synth.rng(722)
    ne = off.size - 1
    po = oracle.pair_offsets(off)
    gt = gpu(synth.upstream(g, ne, 4), torch.float64)
    gem = gpu([g.standard_normal(ne)], torch.float64)[0]
    gpr = gpu([g.standard_normal(int(po[-1]))], torch.float64)[0]
    best = glv.glv_autotune_event_reduce_bwd(gp, go, grad_total=gt, grad_event_m=gem, grad_pair_m=gpr)
    assert best[0] in (64, 128, 256, 512) and best[1] in (16, 32, 64) and best[2] == best[0], best
    assert best[3] in (2 * best[0], min(4 * best[0], 4096)), best
    assert glv.glv_current_tiling_bwd(torch.float64, "PtEtaPhiM") == best
    a = glv.glv_event_reduce_bwd(gp, go, grad_total=gt, grad_event_m=gem, grad_pair_m=gpr)
    b = glv.glv_event_reduce_bwd(gp, go, grad_total=gt, grad_event_m=gem, grad_pair_m=gpr, tiling=best)
    assert all(torch.equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("seed", [731, 732, 733, 734, 735, 736])
def test_random_layouts_and_tilings(seed):
    """Seeded random event layouts (runs of empty and one-particle events,
    Poisson(8) events, now and then 60 to 300 particles) under a random valid
    tiling: the plain FP64 and compensated FP32 forward and the FP64 reverse
    mode against the oracle.  Chunk edges, the pair cap and the separate
    large-event launch all occur."""
    g = np.random.default_rng(seed)
    ne = int(g.integers(200, 3000))
    kind = g.random(ne)
    counts = np.where(kind < 0.15, g.integers(0, 2, ne),
                      np.where(kind < 0.97, np.minimum(g.poisson(8, ne), 64), g.integers(60, 301, ne)))
    counts = counts.astype(np.int64)
    off = np.zeros(ne + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    p, _ = synth.pairs_generic(synth.rng(seed), int(off[-1]))
    block = int(g.choice([64, 128, 256, 512]))
    tiling = (block, int(g.integers(1, 65)), int(g.choice([64, 128, 256, 512, 1024])),
              64 * int(g.integers(1, 17)))
    go = _off(off)
    for dtype, mode in ((torch.float64, "plain"), (torch.float32, "compensated")):
        try:
            out = glv.glv_event_reduce(gpu(p, dtype), go, mode=mode, tiling=tiling)
        except RuntimeError as e:  # a tiling beyond the LDS limit is refused, never run
            assert "GLV_EINVAL_TILING" in str(e), e
            continue
        _check_forward(off, p, dtype, "PtEtaPhiM", mode, *out, f"seed {seed} {mode} {tiling}")
    po = oracle.pair_offsets(off)
    gt = synth.upstream(g, ne, 4)
    gem = g.standard_normal(ne)
    gpr = g.standard_normal(int(po[-1]))
    want = oracle.event_reduce_vjp("PtEtaPhiM", off, p, gt, gem, gpr)
    bt = tiling
    try:
        got = glv.glv_event_reduce_bwd(gpu(p, torch.float64), go, grad_total=gpu(gt, torch.float64),
                                       grad_event_m=gpu([gem], torch.float64)[0],
                                       grad_pair_m=gpu([gpr], torch.float64)[0], tiling=bt)
    except RuntimeError as e:
        assert "GLV_EINVAL_TILING" in str(e), e
        bt = (64, tiling[1], min(tiling[2], 256), tiling[3])
        got = glv.glv_event_reduce_bwd(gpu(p, torch.float64), go, grad_total=gpu(gt, torch.float64),
                                       grad_event_m=gpu([gem], torch.float64)[0],
                                       grad_pair_m=gpu([gpr], torch.float64)[0], tiling=bt)
    _check_bwd(off, p, torch.float64, "PtEtaPhiM", [host(c) for c in got], want, f"seed {seed} bwd {bt}")


def _signature(off):
    """The documented dataset signature, recomputed from the offsets: order of
    magnitude of the event count; share of sampled events per size class in
    5 % steps (all events up to 65,536, else 32 evenly spread runs of 2,048)."""
    ne = off.size - 1
    sizes = np.diff(off)
    if ne > 65536:
        ln = 2048
        sizes = np.concatenate([sizes[r * (ne - ln) // 31: r * (ne - ln) // 31 + ln] for r in range(32)])
    cls = np.array([int(n).bit_length() for n in sizes])
    parts = []
    for b in range(41):
        steps = (int(np.sum(cls == b)) * 20 + sizes.size // 2) // sizes.size
        if steps:
            parts.append(f"{b}:{steps * 5}")
    return f"e{int(ne).bit_length() - 1};" + ",".join(parts)


def test_autotune_cache_retunes_per_dataset_signature(tmp_path, monkeypatch):
    """Two datasets with different multiplicity distributions get their own
    entries in the GLV_AUTOTUNE_CACHE file; after forgetting, the lookup finds
    each one's choice without timing; tuning a dataset again adds nothing."""
    import json
    path = tmp_path / "tune.json"
    monkeypatch.setenv("GLV_AUTOTUNE_CACHE", str(path))
    glv.glv_autotune_forget()
    try:
        off_a, p_a = _events(1 << 14, 740)
        off_b, p_b = _events(1 << 17, 741, mean=3.0)
        ka, kb = glv.glv_autotune_key(_off(off_a)), glv.glv_autotune_key(_off(off_b))
        assert ka.split("|")[4] == _signature(off_a) and kb.split("|")[4] == _signature(off_b)
        assert ka != kb
        ta = glv.glv_autotune_event_reduce(gpu(p_a, torch.float64), _off(off_a))
        assert [e["key"] for e in json.loads(path.read_text())["entries"]] == [ka]
        tb = glv.glv_autotune_event_reduce(gpu(p_b, torch.float64), _off(off_b))
        entries = json.loads(path.read_text())["entries"]
        assert [e["key"] for e in entries] == [ka, kb]
        assert [tuple(e["tiling"]) for e in entries] == [ta, tb]
        glv.glv_autotune_forget()
        assert glv.glv_autotune_lookup(_off(off_a)) == (ta, True)
        assert glv.glv_current_tiling(torch.float64, "PtEtaPhiM", "plain") == ta
        assert glv.glv_autotune_lookup(_off(off_b)) == (tb, True)
        assert glv.glv_autotune_event_reduce(gpu(p_a, torch.float64), _off(off_a)) == ta
        assert len(json.loads(path.read_text())["entries"]) == 2
        # the backward has keys of its own
        kbw = glv.glv_autotune_key(_off(off_a), backward=True)
        assert kbw.split("|")[3] == "bwd"
        glv.glv_autotune_event_reduce_bwd(gpu(p_a, torch.float64), _off(off_a),
                                          grad_pair_m=torch.ones(int(oracle.pair_offsets(off_a)[-1]),
                                                                 dtype=torch.float64, device=DEV))
        assert [e["key"] for e in json.loads(path.read_text())["entries"]] == [ka, kb, kbw]
    finally:
        glv.glv_autotune_forget()
