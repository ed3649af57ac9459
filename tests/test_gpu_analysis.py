"""GPU parity of the analysis step after the mass (not in the paper): the
mass histogram and the per-event pair closest to a target mass, bit for bit
against the oracle (both take the bin and the argmin in binary64)."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import DEV, host

pytestmark = pytest.mark.gpu
glv = pytest.importorskip("paper_2312_02756_amd.glv")

SPECIAL = [math.nan, math.inf, -math.inf, -1.0, 0.0, 20.0, 160.0, 200.0, 199.99999999999997, 1e-300, 91.1876]


def _masses(n, seed):
    """A falling continuum with a resonance peak (the shape of a pair-mass
    spectrum), plus the special values."""
    g = synth.rng(seed)
    m = np.concatenate([g.exponential(40.0, n - n // 4), g.normal(91.1876, 2.5, n // 4)])
    return np.concatenate([m, SPECIAL])


@pytest.mark.parametrize("bins", [(0.0, 200.0, 1000), (20.0, 160.0, 7), (0.0, 200.0, 8190), (0.0, 200.0, 8191),
                                  (0.0, 200.0, 20000), (-3.0, 1e4, 1)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_histogram_against_oracle(bins, dtype):
    lo, hi, nb = bins
    m = _masses(65536, 960)
    mt = torch.from_numpy(m).to(DEV).to(dtype)
    wide = host(mt).astype(np.float64)
    c = host(glv.glv_mass_histogram(mt, lo, hi, nb)).astype(np.uint64)
    assert np.array_equal(c, oracle.histogram(wide, lo, hi, nb))
    # one element in (not 16-byte aligned) and ragged lengths
    for sl in (slice(1, None), slice(0, 1), slice(3, 260), slice(0, 4097)):
        c = host(glv.glv_mass_histogram(mt[sl], lo, hi, nb)).astype(np.uint64)
        assert np.array_equal(c, oracle.histogram(wide[sl], lo, hi, nb)), sl


def test_histogram_accumulates_and_full_size():
    n = 1 << 24
    m = _masses(n - len(SPECIAL), synth.LARGE)
    mt = torch.from_numpy(m).to(DEV)
    c = glv.glv_mass_histogram(mt, 0.0, 200.0, 1000)
    want = oracle.histogram(m, 0.0, 200.0, 1000)
    assert np.array_equal(host(c).astype(np.uint64), want)
    glv.glv_mass_histogram(mt[: n // 2], 0.0, 200.0, 1000, counts=c)  # adds
    assert np.array_equal(host(c).astype(np.uint64), want + oracle.histogram(m[: n // 2], 0.0, 200.0, 1000))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_histogram_mostly_outside_the_range(dtype):
    """Nearly every value under- or overflows (their counts are kept per lane
    and added once per thread): sizes past several full rounds of four packs
    per thread of the whole grid, a ragged tail and a misaligned start."""
    n = 5 * (1 << 20) + 37
    m = _masses(n - len(SPECIAL), 961)
    mt = torch.from_numpy(m).to(DEV).to(dtype)
    wide = host(mt).astype(np.float64)
    for lo, hi, nb in ((100.0, 101.0, 10), (0.0, 1.0, 1000), (150.0, 1e9, 3)):
        for sl in (slice(None), slice(1, None), slice(5, n - 11)):
            c = host(glv.glv_mass_histogram(mt[sl], lo, hi, nb)).astype(np.uint64)
            want = oracle.histogram(wide[sl], lo, hi, nb)
            assert np.array_equal(c, want), (lo, hi, nb, sl)
            assert want[0] + want[-1] > 0.5 * want.sum()


def _events(n_events, seed, nan_frac=0.01):
    g = synth.rng(seed)
    counts = np.minimum(g.poisson(8, n_events), 64)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    po = oracle.pair_offsets(off)
    npair = int(po[-1])
    pm = g.uniform(0.0, 200.0, npair)
    pm[g.random(npair) < nan_frac] = math.nan
    pm[:: 97] = 91.0  # equal distances inside events: the lowest rank must win
    return po, pm


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_best_pair_against_oracle(dtype):
    po, pm = _events(5000, 961)
    po = np.concatenate([po, [po[-1], po[-1]]])  # two trailing empty events
    pmt = torch.from_numpy(pm).to(DEV).to(dtype)
    rank, bm = glv.glv_event_best_pair(torch.from_numpy(po).to(DEV), pmt, 91.1876)
    wr, wm = oracle.best_pair(po, host(pmt).astype(np.float64), 91.1876)
    assert np.array_equal(host(rank), wr)
    assert np.array_equal(host(bm).astype(np.float64), wm, equal_nan=True)
    assert host(rank)[-1] == -1


def test_best_pair_full_size():
    """2^20 Poisson(8) events (the jagged workload's shape), every event."""
    po, pm = _events(1 << 20, synth.JAGGED)
    rank, bm = glv.glv_event_best_pair(torch.from_numpy(po).to(DEV), torch.from_numpy(pm).to(DEV), 91.1876)
    wr, wm = oracle.best_pair(po, pm, 91.1876)
    assert np.array_equal(host(rank), wr)
    assert np.array_equal(host(bm), wm, equal_nan=True)


def test_edge_cases_empty_and_giant_event():
    """Empty inputs launch nothing; one event of 2,000 particles (1,999,000
    pairs) among small ones is walked by its lane group to the end."""
    e64 = torch.empty(0, dtype=torch.float64, device=DEV)
    c = glv.glv_mass_histogram(e64, 0.0, 1.0, 5)
    assert host(c).tolist() == [0] * 7
    r, m = glv.glv_event_best_pair(torch.zeros(1, dtype=torch.int64, device=DEV), e64, 91.0)
    assert r.numel() == 0 and m.numel() == 0
    counts = np.array([3, 2000, 0, 5], dtype=np.int64)
    po = oracle.pair_offsets(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64))
    pm = synth.rng(962).uniform(0.0, 200.0, int(po[-1]))
    pm[int(po[1]) + 1_500_000] = 91.0  # the closest pair deep inside the large event
    rank, bm = glv.glv_event_best_pair(torch.from_numpy(po).to(DEV), torch.from_numpy(pm).to(DEV), 91.0)
    wr, wm = oracle.best_pair(po, pm, 91.0)
    assert np.array_equal(host(rank), wr) and wr[1] == 1_500_000
    assert np.array_equal(host(bm), wm, equal_nan=True)
