"""Pins of the oracle's analysis step after the mass (not in the paper): the
mass histogram and the per-event pair closest to a target mass.  CPU only."""
import itertools
import math

import numpy as np

import oracle
import synth


def test_histogram_exact_cases():
    v = np.array([0.0, 0.5, 1.0, 9.999, 10.0, -1e-300, -5.0, 1e300, math.nan, 3.0, 3.0, 7.25, -math.inf, math.inf])
    c = oracle.histogram(v, 0.0, 10.0, 10)
    want = np.zeros(12, dtype=np.uint64)
    want[0] = 3          # -1e-300, -5, -inf
    want[11] = 3         # 10, 1e300, inf
    want[1 + 0] = 2      # 0, 0.5
    want[1 + 1] = 1      # 1
    want[1 + 9] = 1      # 9.999
    want[1 + 3] = 2      # 3, 3
    want[1 + 7] = 1      # 7.25
    assert np.array_equal(c, want)


def test_histogram_against_numpy_on_exact_bins():
    """Bins of width 2 (a power of two): every bin edge and index is exact, so
    numpy's histogram and the brute-force edge test agree with it bit for bit."""
    m = np.concatenate([synth.rng(990).exponential(40.0, 200000), [128.0, 0.0, 127.99999999999999, 64.0]])
    c = oracle.histogram(m, 0.0, 128.0, 64)
    h, _ = np.histogram(m[m < 128.0], bins=64, range=(0.0, 128.0))
    assert np.array_equal(c[1:65], h.astype(np.uint64))
    assert c[0] == 0 and c[65] == np.sum(m >= 128.0)
    small = m[:2000]
    brute = np.zeros(66, dtype=np.uint64)
    for x in small:
        if x >= 128.0:
            brute[65] += 1
        else:
            b = next(b for b in range(64) if 2.0 * b <= x < 2.0 * (b + 1))
            brute[1 + b] += 1
    assert np.array_equal(oracle.histogram(small, 0.0, 128.0, 64), brute)


def test_histogram_totals_and_accumulation():
    m = synth.rng(991).normal(90.0, 30.0, 100000)
    c = oracle.histogram(m, 20.0, 160.0, 1000)
    assert int(c.sum()) == m.size
    assert c[0] == np.sum(m < 20.0) and c[-1] == np.sum(m >= 160.0)
    # counts are added to what the array holds: two halves give the whole
    v = oracle._f64(m)
    counts = np.zeros(1002, dtype=np.uint64)
    for part in (v[:40000], v[40000:]):
        oracle._load().orc_histogram(oracle.ctypes.c_int64(part.size), oracle._p(np.ascontiguousarray(part)),
                                     oracle.ctypes.c_double(20.0), oracle.ctypes.c_double(160.0),
                                     oracle.ctypes.c_int64(1000), oracle._p(counts))
    assert np.array_equal(counts, c)


def _brute_best(counts, masses, target):
    """itertools over each event's pairs in lexicographic order, min by (distance, rank)."""
    ranks, bms, k = [], [], 0
    for n in counts:
        cand = []
        for r, (i, j) in enumerate(itertools.combinations(range(n), 2)):
            m = masses[k + r]
            if not math.isnan(m):
                cand.append((abs(m - target), r, m))
        k += n * (n - 1) // 2
        if cand:
            d, r, m = min(cand)
            ranks.append(r)
            bms.append(m)
        else:
            ranks.append(-1)
            bms.append(math.nan)
    return np.array(ranks), np.array(bms)


def test_best_pair_against_brute_force():
    g = synth.rng(992)
    counts = np.minimum(g.poisson(6, 3000), 40)
    po = oracle.pair_offsets(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64))
    npair = int(po[-1])
    masses = g.uniform(0.0, 200.0, npair)
    masses[g.random(npair) < 0.01] = math.nan
    masses[:50] = 91.0  # ties inside the first events: the lowest rank wins
    r, m = oracle.best_pair(po, masses, 91.1876)
    br, bm = _brute_best(counts, masses, 91.1876)
    assert np.array_equal(r, br)
    assert np.array_equal(m, bm, equal_nan=True)


def test_best_pair_special_events():
    # events: no particles, one particle, one pair, three equal-distance pairs, all NaN
    counts = [0, 1, 2, 3, 2]
    po = oracle.pair_offsets(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64))
    masses = np.array([80.0, 95.0, 87.0, 95.0, math.nan])
    r, m = oracle.best_pair(po, masses, 91.0)
    assert r.tolist() == [-1, -1, 0, 0, -1]
    assert m[2] == 80.0 and m[3] == 95.0 and math.isnan(m[0]) and math.isnan(m[4])
