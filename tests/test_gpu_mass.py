"""GPU parity of the pair invariant mass (plain and compensated) against the
CPU oracle, element by element, through the C ABI (via the binding)."""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import gpu, host, widened
from tolerances import U64, mass_tol_comp_f32, mass_tol_f32, mass_tol_f64, worst

pytestmark = pytest.mark.gpu

glv = pytest.importorskip("paper_2312_02756_amd.glv")

COORDS = ["PtEtaPhiM", "PtEtaPhiE", "PxPyPzE", "PxPyPzM"]


def _legs(coords, n, seed):
    a, b = synth.pairs_generic(synth.rng(seed), n)
    if coords == "PtEtaPhiM":
        return a, b
    ca, cb = oracle.to_cartesian("PtEtaPhiM", a), oracle.to_cartesian("PtEtaPhiM", b)
    if coords == "PxPyPzE":
        return ca, cb
    if coords == "PxPyPzM":
        return (ca[0], ca[1], ca[2], a[3]), (cb[0], cb[1], cb[2], b[3])
    return (a[0], a[1], a[2], ca[3]), (b[0], b[1], b[2], cb[3])


def _check_plain(coords, a, b, dtype, m_gpu, label=""):
    wa, wb = widened(a, dtype), widened(b, dtype)
    m_or, s = oracle.mass_plain(coords, wa, wb, scale=True)
    tol = mass_tol_f64(m_or, s) if dtype == torch.float64 else mass_tol_f32(m_or, s)
    r, i = worst(np.abs(host(m_gpu) - m_or), tol)
    assert r <= 1.0, f"{label} worst item {i}: gpu {host(m_gpu)[i]!r} oracle {m_or[i]!r} ratio {r}"


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("coords", COORDS)
def test_plain_small_workload(coords, dtype):
    """65,536 generic pairs (the correctness workload), every element."""
    a, b = _legs(coords, 65536, synth.SMALL_PAIRS)
    m = glv.glv_invariant_mass(gpu(a, dtype), gpu(b, dtype), coords=coords)
    torch.cuda.synchronize()
    _check_plain(coords, a, b, dtype, m, f"{coords} {dtype}")


@pytest.mark.parametrize("n", [0, 1, 2, 3, 63, 64, 65, 255, 257, 1000, 4097])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_plain_ragged_sizes_and_misaligned(n, dtype):
    a, b = _legs("PtEtaPhiM", n + 1, 500 + n)
    ga, gb = gpu(a, dtype), gpu(b, dtype)
    m = glv.glv_invariant_mass(tuple(t[:n] for t in ga), tuple(t[:n] for t in gb))
    # views starting one element in: not 16-byte aligned -> one element per lane
    m1 = glv.glv_invariant_mass(tuple(t[1:] for t in ga), tuple(t[1:] for t in gb))
    torch.cuda.synchronize()
    assert m.numel() == n and m1.numel() == n
    _check_plain("PtEtaPhiM", tuple(c[:n] for c in a), tuple(c[:n] for c in b), dtype, m)
    _check_plain("PtEtaPhiM", tuple(c[1:] for c in a), tuple(c[1:] for c in b), dtype, m1)


@pytest.mark.parametrize("n", [1, 3, 5, 63, 65, 257, 4097])
def test_compensated_ragged_sizes_and_misaligned(n):
    """The FP32 compensated mass on ragged sizes (four pairs per lane plus a
    tail) and on views one element in (one pair per lane), against the
    accurate oracle of the widened inputs; the two runs agree bitwise."""
    a, b, _ = synth.pairs_stress(synth.rng(540 + n), n + 1)
    a, b = synth.as_dtype(a, np.float32), synth.as_dtype(b, np.float32)
    ga, gb = gpu(a, torch.float32), gpu(b, torch.float32)
    m = host(glv.glv_invariant_mass(tuple(t[:n] for t in ga), tuple(t[:n] for t in gb), mode="compensated"))
    m1 = host(glv.glv_invariant_mass(tuple(t[1:] for t in ga), tuple(t[1:] for t in gb), mode="compensated"))
    for got, sl in ((m, slice(0, n)), (m1, slice(1, n + 1))):
        wa, wb = widened(tuple(c[sl] for c in a), torch.float32), widened(tuple(c[sl] for c in b), torch.float32)
        m_or = oracle.mass_accurate(wa, wb)
        r, i = worst(np.abs(got.astype(np.float64) - m_or), mass_tol_comp_f32(m_or))
        assert r <= 1.0, (n, i, got[i], m_or[i])
    assert np.array_equal(m[1:], m1[:-1])


def test_back_to_back_is_exactly_2E_and_swap_is_bitwise():
    x, _ = synth.boost_items(synth.rng(501), 10000)
    a = gpu(x, torch.float64)
    b = gpu((-x[0], -x[1], -x[2], x[3]), torch.float64)
    m = host(glv.glv_invariant_mass(a, b, coords="PxPyPzE"))
    assert np.array_equal(m, 2 * x[3])
    pa, pb = _legs("PtEtaPhiM", 20000, 502)
    ga, gb = gpu(pa, torch.float64), gpu(pb, torch.float64)
    m1 = glv.glv_invariant_mass(ga, gb)
    m2 = glv.glv_invariant_mass(gb, ga)
    m3 = glv.glv_invariant_mass(ga, gb)
    torch.cuda.synchronize()
    assert torch.equal(m1, m2) and torch.equal(m1, m3)


def test_fp64_square_root_is_correctly_rounded():
    """Sums w = (p, 0, 0, E) with p and E of at most 26 significant bits: E^2
    and p^2 are exact in binary64, so q = E^2 - p^2 is rounded once in any
    evaluation order, and m must be the correctly rounded square root of that
    q (Python's math.sqrt is IEEE-correct), with the sign convention for q < 0."""
    import math

    rng = synth.rng(503)
    n = 100000
    ke = rng.integers(1 << 25, 1 << 26, size=n)
    kp = rng.integers(0, 1 << 26, size=n)
    kp[: n // 4] = ke[: n // 4] - rng.integers(0, 1 << 12, size=n // 4)  # near-lightlike sums
    sc = rng.integers(-40, 20, size=n)
    e = np.ldexp(ke.astype(np.float64), sc)
    pz = np.ldexp(kp.astype(np.float64), sc)
    want = np.empty(n)
    for t in range(n):
        q = math.ldexp(float(int(ke[t]) ** 2 - int(kp[t]) ** 2), 2 * int(sc[t]))  # one rounding
        want[t] = math.sqrt(q) if q >= 0 else -math.sqrt(-q)
    zero = np.zeros(n)
    a = gpu((pz, zero, zero, e), torch.float64)
    b = gpu((zero, zero, zero, zero), torch.float64)
    m = host(glv.glv_invariant_mass(a, b, coords="PxPyPzE"))
    bad = np.flatnonzero(m != want)
    assert bad.size == 0, f"{bad.size} items differ, first {bad[:4]}: gpu {m[bad[:4]]} want {want[bad[:4]]}"


def test_plain_full_size():
    """2^24 FP64 pairs in the benchmark's launch shape, every item against the
    oracle (on all host cores)."""
    n = 1 << 24
    a, b = synth.pairs_generic(synth.rng(synth.LARGE), n)
    m = host(glv.glv_invariant_mass(gpu(a, torch.float64), gpu(b, torch.float64)))
    m_or, s = oracle.mass_plain("PtEtaPhiM", a, b, scale=True)
    r, i = worst(np.abs(m - m_or), mass_tol_f64(m_or, s))
    assert r <= 1.0, (i, m[i], m_or[i])
    assert np.all(np.isfinite(m)) and np.all(m > 0)


# --------------------------------------------------------------- compensated

def _stress(n, seed):
    a, b, mask = synth.pairs_stress(synth.rng(seed), n)
    return synth.as_dtype(a, np.float32), synth.as_dtype(b, np.float32), mask


def test_compensated_fp32_stress_workload():
    """Light, wide-pt pairs with 10% nearly collinear, FP32 compensated,
    every element against the accurate FP64 oracle of the same FP32 inputs:
    |m - m_or| <= 4e-6 m_or + 1e-6 GeV."""
    n = 1 << 20
    a, b, mask = _stress(n, synth.STRESS)
    fb = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    m = host(glv.glv_invariant_mass(gpu(a, torch.float32), gpu(b, torch.float32), mode="compensated",
                                    fallback_count=fb))
    m_or = oracle.mass_accurate(a, b)
    err = np.abs(m.astype(np.float64) - m_or)
    r, i = worst(err, mass_tol_comp_f32(m_or))
    assert r <= 1.0, (i, bool(mask[i]), m[i], m_or[i])
    nfb = int(fb.item())
    assert 0 <= nfb < n // 100  # the FP64 redo stays rare
    # the plain FP32 form fails here, which is the point of the compensated one
    mp = host(glv.glv_invariant_mass(gpu(a, torch.float32), gpu(b, torch.float32)))
    assert np.max(np.abs(mp - m_or) / m_or) > 1e-3


def _heavy_slow_pairs(n, seed):
    """Heavy, slow legs (M ~ U[5, 20] GeV, pt ~ LogUniform[0.01, 10] GeV,
    eta ~ U[-4, 4]): pairs at opposite large |eta| exceed the FP32 error
    bound of the compensated form (its rapidity shifts are large there)."""
    g = synth.rng(seed)

    def leg():
        return (np.exp(g.uniform(np.log(0.01), np.log(10.0), n)), g.uniform(-4.0, 4.0, n),
                g.uniform(-np.pi, np.pi, n), g.uniform(5.0, 20.0, n))

    a = leg()
    b = leg()
    return synth.as_dtype(a, np.float32), synth.as_dtype(b, np.float32)


@pytest.mark.parametrize("n", [4097, 1 << 16])
def test_compensated_fp64_redo_elementwise(n):
    """Pairs that force the FP64 redo of the element-wise FP32 compensated
    mass: some but not all items are recomputed, every element lies within
    4e-6 m + 1e-6 GeV of the accurate oracle, and the aligned launch (four
    pairs per lane) and the launch on views one element in (one pair per lane)
    agree bitwise, redo count included."""
    a, b = _heavy_slow_pairs(n + 1, 760)
    ga, gb = gpu(a, torch.float32), gpu(b, torch.float32)
    fb = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    fb1 = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    m = host(glv.glv_invariant_mass(tuple(t[1:] for t in ga), tuple(t[1:] for t in gb), mode="compensated",
                                    fallback_count=fb1))
    ca, cb = tuple(t[1:].clone() for t in ga), tuple(t[1:].clone() for t in gb)
    assert all(t.data_ptr() % 16 == 0 for t in ca + cb)
    mal = host(glv.glv_invariant_mass(ca, cb, mode="compensated", fallback_count=fb))
    nfb, nfb1 = int(fb.item()), int(fb1.item())
    assert 0 < nfb < n, nfb
    assert nfb == nfb1
    assert np.array_equal(m.view(np.uint32), mal.view(np.uint32))
    wa, wb = widened(tuple(c[1:] for c in a), torch.float32), widened(tuple(c[1:] for c in b), torch.float32)
    m_or = oracle.mass_accurate(wa, wb)
    r, i = worst(np.abs(m.astype(np.float64) - m_or), mass_tol_comp_f32(m_or))
    assert r <= 1.0, (i, m[i], m_or[i])


def test_compensated_fp64_is_accurate():
    n = 1 << 18
    a, b, _ = synth.pairs_stress(synth.rng(503), n)
    m = host(glv.glv_invariant_mass(gpu(a, torch.float64), gpu(b, torch.float64), mode="compensated"))
    mq = oracle.mass_plain_q("PtEtaPhiM", a, b)
    # device libm differs from glibc by an ulp or so per function
    r, i = worst(np.abs(m - mq), 64 * U64 * mq)
    assert r <= 1.0, (i, m[i], mq[i])


def test_compensated_seam_and_degenerate():
    pt = np.array([50.0, 900.0, 10.0, 3.0, 7.0, 0.0])
    eta = np.array([0.3, -1.2, 2.0, 0.0, -3.9, 1.0])
    phia = np.array([np.pi - 1e-4, -np.pi + 3e-5, 0.1, 1.0, -2.0, 0.5])
    phib = np.array([-np.pi + 2e-4, np.pi - 5e-5, 0.1, 1.0, -2.0, 0.5])
    ma = np.array([0.0, 0.1, 0.105, 0.0, 0.13, 0.0])
    mb = np.array([0.0, 0.0, 0.105, 0.0, 0.13, 0.0])
    a = synth.as_dtype((pt, eta, phia, ma), np.float32)
    b = synth.as_dtype((pt * 1.5, eta, phib, mb), np.float32)
    m = host(glv.glv_invariant_mass(gpu(a, torch.float32), gpu(b, torch.float32), mode="compensated"))
    m_or = oracle.mass_accurate(a, b)
    assert np.all(np.abs(m - m_or) <= mass_tol_comp_f32(m_or))
    # identical massless legs: exactly zero; zero leg: the other leg's mass
    assert m[3] == 0.0


def test_compensated_azimuths_beyond_pi():
    """Azimuths shifted by whole turns (|phi| up to 5 pi): the half azimuth
    difference then leaves [-pi/2, pi/2] and the reduced sine takes over.
    Pairs at least 0.3 rad apart in azimuth, where the FP32 rounding of the
    shifted inputs' difference stays within the tolerance."""
    g = synth.rng(713)
    n = 4096
    a, b = synth.pairs_generic(g, n)
    ka, kb = g.integers(-2, 3, n), g.integers(-2, 3, n)
    a = (a[0], a[1], a[2] + 2 * np.pi * ka, a[3])
    b = (b[0], b[1], b[2] + 2 * np.pi * kb, b[3])
    a, b = synth.as_dtype(a, np.float32), synth.as_dtype(b, np.float32)
    d = np.angle(np.exp(1j * (a[2].astype(np.float64) - b[2].astype(np.float64))))
    keep = np.abs(d) >= 0.3
    assert np.count_nonzero(keep) > n // 2 and np.count_nonzero(np.abs(a[2] - b[2]) > np.pi) > n // 4
    m = host(glv.glv_invariant_mass(gpu(a, torch.float32), gpu(b, torch.float32), mode="compensated"))
    m_or = oracle.mass_accurate(widened(a, torch.float32), widened(b, torch.float32))
    r, i = worst(np.abs(m[keep].astype(np.float64) - m_or[keep]), mass_tol_comp_f32(m_or[keep]))
    assert r <= 1.0, (i, m[keep][i], m_or[keep][i])


def test_compensated_full_size():
    """2^26 FP32 stress pairs (the precision-stress workload) in the
    benchmark's launch shape, every item against the accurate oracle."""
    n = 1 << 26
    a, b, mask = _stress(n, synth.STRESS)
    fb = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    m = host(glv.glv_invariant_mass(gpu(a, torch.float32), gpu(b, torch.float32), mode="compensated",
                                    fallback_count=fb))
    m_or = oracle.mass_accurate(widened(a, torch.float32), widened(b, torch.float32))
    r, i = worst(np.abs(m.astype(np.float64) - m_or), mass_tol_comp_f32(m_or))
    assert r <= 1.0, (i, m[i], m_or[i])
    assert np.all(np.isfinite(m))
    assert int(fb.item()) < n // 100


def test_golden_pair_masses():
    """The fixed cases of tests/golden/pair_masses.txt (generic, Z-like,
    collinear, identical, zero leg, azimuth seam, large |eta|, heavy and slow,
    high pt, back to back) against their stored binary128 masses: plain FP64
    within its bound, the FP64 cancellation-free mode within 64 u64, and
    identical massless legs exactly 0 in that mode."""
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_fixtures.py")
    spec = importlib.util.spec_from_file_location("make_fixtures", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    labels, a, b, m_q, _ = mod.load()
    _, s = oracle.mass_plain("PtEtaPhiM", a, b, scale=True)
    m = host(glv.glv_invariant_mass(gpu(a, torch.float64), gpu(b, torch.float64)))
    r, i = worst(np.abs(m - m_q), mass_tol_f64(m_q, s))
    assert r <= 1.0, (labels[i], m[i], m_q[i])
    mc = host(glv.glv_invariant_mass(gpu(a, torch.float64), gpu(b, torch.float64), mode="compensated"))
    keep = np.array([lab != "identical_massless" for lab in labels])
    assert np.all(np.abs(mc - m_q)[keep] <= 64 * U64 * m_q[keep]), [(l, x, y) for l, x, y in zip(labels, mc, m_q)]
    assert mc[labels.index("identical_massless")] == 0.0
