"""GPU parity of the analysis step fused into the kernels (not in the paper;
its Sec. 6 places GenVector inside ROOT, whose analyses histogram pair masses
and pick pairs near a resonance):

  * glv_invariant_mass_histogram -- pair masses binned as they are computed,
    never stored;
  * glv_event_reduce_best_pair -- each jagged event's pair closest to a target
    mass, chosen inside the reduction without writing pair masses.

Against the oracle: its masses (plain or accurate, binary64) carry the
stated per-mass tolerance t, so a mass may legitimately fall on either side
of a bin edge or swap places with a near-equal competitor.  The histogram is
held to the cumulative band that this allows (bin slots are monotone in the
mass): for every slot b,
    #{slot(m_or + t) <= b}  <=  sum of the GPU counts up to b  <=  #{slot(m_or - t) <= b},
and the best pair to the set of pairs whose oracle distance could be the
smallest within the tolerances, with its mass within the tolerance of the
oracle's mass of that pair.  Beside that, the fused results must equal, bit
for bit, the unfused kernels' (the mass kernel then glv_mass_histogram, the
reduction then glv_event_best_pair) on the same inputs: the fusion changes
where masses go, never their values."""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import DEV, gpu, host, widened
from tolerances import U64, mass_tol_comp_f32, mass_tol_f32, mass_tol_f64

pytestmark = pytest.mark.gpu
glv = pytest.importorskip("paper_2312_02756_amd.glv")

TARGET = 91.1876


def _pair_tol(a, b, dtype, mode):
    """Oracle masses of the pairs (a_i, b_i) and their per-mass tolerance."""
    if mode == "compensated":
        m = oracle.mass_accurate(a, b)
        t = mass_tol_comp_f32(m) if dtype == torch.float32 else 64 * U64 * m + 1e-300
        return m, t
    m, s = oracle.mass_plain("PtEtaPhiM", a, b, scale=True)
    return m, (mass_tol_f64(m, s) if dtype == torch.float64 else mass_tol_f32(m, s))


def _check_hist_band(counts, m_or, tol, lo, hi, nb):
    c = np.cumsum(counts.astype(np.int64))
    upper = np.cumsum(oracle.histogram(m_or - tol, lo, hi, nb).astype(np.int64))
    lower = np.cumsum(oracle.histogram(m_or + tol, lo, hi, nb).astype(np.int64))
    bad = np.nonzero((c < lower) | (c > upper))[0]
    assert bad.size == 0, (bad[:5], c[bad[:5]], lower[bad[:5]], upper[bad[:5]])
    assert c[-1] == np.count_nonzero(~np.isnan(m_or))


def _legs(dtype, mode, n, seed):
    if mode == "compensated":
        a, b, _ = synth.pairs_stress(synth.rng(seed), n)
    else:
        a, b = synth.pairs_generic(synth.rng(seed), n)
    return a, b


@pytest.mark.parametrize("dtype,mode", [(torch.float64, "plain"), (torch.float32, "plain"),
                                        (torch.float32, "compensated"), (torch.float64, "compensated")])
@pytest.mark.parametrize("bins", [(0.0, 400.0, 1000), (50.0, 150.0, 7), (0.0, 400.0, 20000)])
def test_fused_histogram(dtype, mode, bins):
    """65,536 pairs plus ragged and misaligned views; LDS counters (up to 8,190
    bins) and global counters (20,000 bins)."""
    lo, hi, nb = bins
    n = 65536 + 37
    a, b = _legs(dtype, mode, n, 970)
    ga, gb = gpu(a, dtype), gpu(b, dtype)
    wa, wb = widened(a, dtype), widened(b, dtype)
    m_or, tol = _pair_tol(wa, wb, dtype, mode)
    for sl in (slice(None), slice(1, None), slice(0, 1), slice(5, 4100)):
        sa, sb = tuple(c[sl] for c in ga), tuple(c[sl] for c in gb)
        fb = torch.zeros(1, dtype=torch.int64, device=DEV)
        got = glv.glv_invariant_mass_histogram(sa, sb, lo, hi, nb, mode=mode, fallback_count=fb)
        _check_hist_band(host(got), m_or[sl], tol[sl], lo, hi, nb)
        # bitwise the unfused kernels' histogram, and the same redo count
        fb2 = torch.zeros(1, dtype=torch.int64, device=DEV)
        m = glv.glv_invariant_mass(sa, sb, mode=mode, fallback_count=fb2)
        assert torch.equal(got, glv.glv_mass_histogram(m, lo, hi, nb)), sl
        assert int(fb.item()) == int(fb2.item())


def test_fused_histogram_other_coords_accumulates_and_counts_redos():
    """PxPyPzE legs (plain); counts added to a given histogram; FP32
    compensated legs that force the FP64 redo (heavy, slow particles at
    opposite large |eta|) count it as the stored-mass kernel does."""
    n = 50000
    a, b = synth.pairs_generic(synth.rng(971), n)
    ca, cb = oracle.to_cartesian("PtEtaPhiM", a), oracle.to_cartesian("PtEtaPhiM", b)
    ga, gb = gpu(ca, torch.float64), gpu(cb, torch.float64)
    m_or, s = oracle.mass_plain("PxPyPzE", ca, cb, scale=True)
    c = glv.glv_invariant_mass_histogram(ga, gb, 0.0, 400.0, 500, coords="PxPyPzE")
    _check_hist_band(host(c), m_or, mass_tol_f64(m_or, s), 0.0, 400.0, 500)
    c0 = host(c).copy()
    glv.glv_invariant_mass_histogram(ga, gb, 0.0, 400.0, 500, coords="PxPyPzE", counts=c)
    assert np.array_equal(host(c), 2 * c0)
    g = synth.rng(972)
    p = [np.exp(g.uniform(np.log(0.01), np.log(10.0), n)), g.uniform(-4, 4, n), g.uniform(-np.pi, np.pi, n),
         g.uniform(5.0, 20.0, n)]
    q = [np.exp(g.uniform(np.log(0.01), np.log(10.0), n)), -p[1] + g.uniform(-0.5, 0.5, n),
         g.uniform(-np.pi, np.pi, n), g.uniform(5.0, 20.0, n)]
    gp, gq = gpu(p, torch.float32), gpu(q, torch.float32)
    fb = torch.zeros(1, dtype=torch.int64, device=DEV)
    c = glv.glv_invariant_mass_histogram(gp, gq, 0.0, 200.0, 800, mode="compensated", fallback_count=fb)
    assert 0 < int(fb.item()) < n
    m_or = oracle.mass_accurate(widened(p, torch.float32), widened(q, torch.float32))
    _check_hist_band(host(c), m_or, mass_tol_comp_f32(m_or), 0.0, 200.0, 800)


# ------------------------------------------------------------ best pair

def _best_band(po, pm_or, tol, target, rank, best_m, label):
    """The GPU's choice lies in each event's set of possible winners."""
    ne = po.size - 1
    d = np.abs(pm_or - target)
    for e in range(ne):
        lo, hi = int(po[e]), int(po[e + 1])
        de, te = d[lo:hi], tol[lo:hi]
        ok = ~np.isnan(de)
        if not ok.any():
            assert rank[e] == -1 and np.isnan(best_m[e]), (label, e)
            continue
        bound = np.min((de + te)[ok])
        cand = np.nonzero(ok & (de - te <= bound))[0]
        r = int(rank[e])
        assert r in cand, (label, e, r, cand[:8])
        assert abs(float(best_m[e]) - pm_or[lo + r]) <= tol[lo + r], (label, e, r)


def _events_with_big(seed, ne=3000):
    g = synth.rng(seed)
    counts = np.minimum(g.poisson(8, ne), 64)
    counts[[7, 500, 2999]] = [300, 0, 129]  # one event past every staging capacity, one empty
    counts[[11, 12]] = [1, 2]
    off = np.zeros(ne + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    p, _ = synth.pairs_generic(g, int(off[-1]))
    return off, p


@pytest.mark.parametrize("dtype,mode", [(torch.float64, "plain"), (torch.float32, "plain"),
                                        (torch.float32, "compensated")])
@pytest.mark.parametrize("tiling", [None, (64, 16, 64, 128), (128, 64, 256, 512)])
def test_fused_best_pair(dtype, mode, tiling):
    off, p = _events_with_big(973)
    go, gp = torch.from_numpy(off).to(DEV), gpu(p, dtype)
    po = glv.glv_pair_offsets(go)
    rank, bm = glv.glv_event_reduce_best_pair(gp, go, TARGET, pair_offsets=po, mode=mode, tiling=tiling)
    rank, bm = host(rank), host(bm).astype(np.float64)
    wp = widened(p, dtype)
    _, _, pm_or, po_or = oracle.event_reduce("PtEtaPhiM", off, wp,
                                              mode=oracle.ACCURATE if mode == "compensated" else oracle.PLAIN)
    ii, jj = [], []
    for e in range(off.size - 1):
        r, c = np.triu_indices(int(off[e + 1] - off[e]), 1)
        ii.append(off[e] + r)
        jj.append(off[e] + c)
    ii, jj = np.concatenate(ii), np.concatenate(jj)
    _, tol = _pair_tol(tuple(c[ii] for c in wp), tuple(c[jj] for c in wp), dtype, mode)
    _best_band(po_or, pm_or, tol, TARGET, rank, bm, f"{dtype} {mode} {tiling}")
    # bitwise the unfused path: the reduction's pair masses, then the selection
    _, _, pm = glv.glv_event_reduce(gp, go, pair_offsets=po, mode=mode, tiling=tiling, want_total=False,
                                    want_event_m=False)
    r2, m2 = glv.glv_event_best_pair(po, pm, TARGET)
    assert np.array_equal(rank, host(r2))
    assert np.array_equal(bm, host(m2).astype(np.float64), equal_nan=True)


def test_fused_best_pair_fp64_redo_events():
    """FP32 compensated events whose pairs need the FP64 redo (heavy, slow
    particles at opposite large |eta|): the reduction marks them in the best
    mass and the second launch recomputes them."""
    g = synth.rng(974)
    counts = np.concatenate([np.minimum(g.poisson(6, 1500), 40), [0, 1, 2]]).astype(np.int64)
    off = np.zeros(counts.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    n = int(off[-1])
    p = (np.exp(g.uniform(np.log(0.01), np.log(10.0), n)), g.uniform(-4, 4, n), g.uniform(-np.pi, np.pi, n),
         g.uniform(5.0, 20.0, n))
    go, gp = torch.from_numpy(off).to(DEV), gpu(p, torch.float32)
    fb = torch.zeros(1, dtype=torch.int64, device=DEV)
    target = 30.0
    rank, bm = glv.glv_event_reduce_best_pair(gp, go, target, mode="compensated", fallback_count=fb)
    assert int(fb.item()) > 0
    wp = widened(p, torch.float32)
    _, _, pm_or, po_or = oracle.event_reduce("PtEtaPhiM", off, wp, mode=oracle.ACCURATE)
    _best_band(po_or, pm_or, mass_tol_comp_f32(pm_or), target, host(rank), host(bm).astype(np.float64), "redo")
    _, _, pm = glv.glv_event_reduce(gp, go, mode="compensated", want_total=False, want_event_m=False)
    r2, m2 = glv.glv_event_best_pair(glv.glv_pair_offsets(go), pm, target)
    assert np.array_equal(host(rank), host(r2))
    assert np.array_equal(host(bm), host(m2), equal_nan=True)


def test_fused_best_pair_full_size():
    """2^20 Poisson(8) events in the benchmark's launch shape: every event
    against the unfused path, a sample against the oracle."""
    off, p = synth.jagged_events(synth.rng(synth.JAGGED), 1 << 20)
    go, gp = torch.from_numpy(off).to(DEV), gpu(p, torch.float64)
    po = glv.glv_pair_offsets(go)
    rank, bm = glv.glv_event_reduce_best_pair(gp, go, TARGET, pair_offsets=po)
    _, _, pm = glv.glv_event_reduce(gp, go, pair_offsets=po, want_total=False, want_event_m=False)
    r2, m2 = glv.glv_event_best_pair(po, pm, TARGET)
    assert torch.equal(rank, r2) and torch.equal(torch.nan_to_num(bm, nan=-1.0), torch.nan_to_num(m2, nan=-1.0))
    sel = np.sort(np.random.default_rng(15).choice(off.size - 1, 4000, replace=False))
    cnt = off[sel + 1] - off[sel]
    soff = np.zeros(sel.size + 1, dtype=np.int64)
    soff[1:] = np.cumsum(cnt)
    pidx = np.concatenate([np.arange(off[e], off[e + 1]) for e in sel])
    sp = tuple(c[pidx] for c in p)
    _, _, pm_or, po_or = oracle.event_reduce("PtEtaPhiM", soff, sp)
    ii, jj = [], []
    for e in range(sel.size):
        r, c = np.triu_indices(int(cnt[e]), 1)
        ii.append(soff[e] + r)
        jj.append(soff[e] + c)
    ii, jj = np.concatenate(ii), np.concatenate(jj)
    _, tol = _pair_tol(tuple(c[ii] for c in sp), tuple(c[jj] for c in sp), torch.float64, "plain")
    _best_band(po_or, pm_or, tol, TARGET, host(rank)[sel], host(bm)[sel], "full size")


def test_fused_empty_inputs():
    e64 = torch.empty(0, dtype=torch.float64, device=DEV)
    c = glv.glv_invariant_mass_histogram((e64,) * 4, (e64,) * 4, 0.0, 1.0, 5)
    assert host(c).tolist() == [0] * 7
    z = torch.zeros(1, dtype=torch.int64, device=DEV)
    r, m = glv.glv_event_reduce_best_pair((e64,) * 4, z, TARGET, pair_offsets=z)
    assert r.numel() == 0 and m.numel() == 0


def _spanning_layout(seed):
    """Events laid out so that the lanes' runs of pairs cross many events and
    events cross many runs and rounds: blocks of one-pair events (n = 2),
    events of 12 to 20 particles (66 to 190 pairs: several 64-pair rounds on
    their own), one- and zero-particle events, and Poisson(8) events."""
    g = np.random.default_rng(seed)
    counts = []
    for _ in range(60):
        kind = int(g.integers(0, 4))
        if kind == 0:
            counts += [2] * int(g.integers(1, 50))
        elif kind == 1:
            counts += [int(g.integers(12, 21))]
        elif kind == 2:
            counts += [int(c) for c in g.integers(0, 2, int(g.integers(1, 6)))]
        else:
            counts += [int(c) for c in np.minimum(g.poisson(8, int(g.integers(1, 20))), 64)]
    counts = np.array(counts, dtype=np.int64)
    off = np.zeros(counts.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    return off, g


@pytest.mark.parametrize("tiling", [(64, 64, 128, 64), (64, 16, 64, 128), (256, 32, 256, 192),
                                    (64, 64, 128, 1024)])
def test_cross_run_combines(tiling):
    """The compensated event mass and the fused best pair combine each event's
    partial results across the lanes' runs of pairs (a segmented scan over the
    lanes plus the run where the event ends) and across rounds.  On layouts
    that make runs cross many events and events cross many runs and rounds:
    compensated event masses against the oracle's accurate masses (FP32 and
    FP64), reproducible bit for bit for the tiling, with pair masses
    independent of it; the fused best pair bitwise the unfused selection."""
    off, g = _spanning_layout(977 + tiling[3])
    a, _, _ = synth.pairs_stress(synth.rng(977), int(off[-1]))
    go = torch.from_numpy(off).to(DEV)
    po = glv.glv_pair_offsets(go)
    for dtype in (torch.float32, torch.float64):
        gp = gpu(a, dtype)
        try:
            _, em, pm = glv.glv_event_reduce(gp, go, pair_offsets=po, mode="compensated", tiling=tiling)
        except RuntimeError as e:  # a tiling beyond the LDS limit is refused, never run
            assert "GLV_EINVAL_TILING" in str(e), e
            continue
        _, em2, pm2 = glv.glv_event_reduce(gp, go, pair_offsets=po, mode="compensated", tiling=tiling)
        assert torch.equal(em, em2) and torch.equal(pm, pm2)
        _, _, pm_d = glv.glv_event_reduce(gp, go, pair_offsets=po, mode="compensated")
        assert torch.equal(pm, pm_d), "pair masses do not depend on the tiling"
        wa = widened(a, dtype)
        _, em_or, _, _ = oracle.event_reduce("PtEtaPhiM", off, wa, mode=oracle.ACCURATE)
        got = host(em).astype(np.float64)
        tol = mass_tol_comp_f32(em_or) if dtype == torch.float32 else 64 * U64 * np.abs(em_or) + 1e-300
        bad = np.nonzero(~(np.abs(got - em_or) <= tol))[0]
        assert bad.size == 0, (dtype, tiling, bad[:5], got[bad[:5]], em_or[bad[:5]])
    for dtype, mode in ((torch.float64, "plain"), (torch.float32, "compensated")):
        gp = gpu(a, dtype)
        try:
            rank, bm = glv.glv_event_reduce_best_pair(gp, go, TARGET, pair_offsets=po, mode=mode, tiling=tiling)
        except RuntimeError as e:
            assert "GLV_EINVAL_TILING" in str(e), e
            continue
        _, _, pm = glv.glv_event_reduce(gp, go, pair_offsets=po, mode=mode, tiling=tiling, want_total=False,
                                        want_event_m=False)
        r2, m2 = glv.glv_event_best_pair(po, pm, TARGET)
        assert np.array_equal(host(rank), host(r2)), (dtype, mode, tiling)
        assert np.array_equal(host(bm), host(m2), equal_nan=True), (dtype, mode, tiling)
