"""Precision of the GPU's coordinate conversion (its own sincos / exp-based
sinh and cosh) against binary128: single-particle events make the per-event
totals equal to the particle's Cartesian components."""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import gpu, host, widened
from tolerances import U32, U64, worst

pytestmark = pytest.mark.gpu

glv = pytest.importorskip("paper_2312_02756_amd.glv")


def _particles(n, seed, wide_phi):
    g = synth.rng(seed)
    pt = 5.0 + g.exponential(30.0, n)
    eta = g.uniform(-5.0, 5.0, n)
    phi = g.uniform(-np.pi, np.pi, n)
    # a quarter of the angles far outside [-pi, pi): the reduction's range,
    # and beyond it the library path
    k = n // 4
    phi[:k] = g.uniform(-wide_phi, wide_phi, k)
    eta[:16] = [0.0, 0.49, -0.49, 0.5, -0.5, 0.51, 1e-300, -1e-12, 20.0, -20.0, 3.9, -3.9, 1e-8, 0.25, 2.0, -2.0]
    phi[:16] = [0.0, np.pi / 2, -np.pi / 2, np.pi, -np.pi, np.pi / 4, 3 * np.pi / 4, 1e-300, 2.0, -2.0,
                1.5707963267948966, 3.141592653589793, 6.283185307179586, -1e-9, 0.785, -0.7854]
    m = g.uniform(0.0, 0.2, n)
    return pt, eta, phi, m


@pytest.mark.parametrize("dtype,wide", [(torch.float64, 2e5), (torch.float32, 2e4)])
def test_conversion_against_binary128(dtype, wide):
    n = 1 << 18
    p = _particles(n, 800, wide)
    wp = widened(p, dtype)
    off = np.arange(n + 1, dtype=np.int64)
    total, _, _ = glv.glv_event_reduce(gpu(p, dtype), torch.from_numpy(off).to("cuda:0"), want_event_m=False,
                                       want_pair_m=False)
    got = [host(t).astype(np.float64) for t in total]
    want, _ = oracle.event_reduce_q("PtEtaPhiM", off, wp)
    u = U64 if dtype == torch.float64 else U32
    pt, eta = wp[0], wp[1]
    scales = [pt, pt, pt * np.cosh(eta), np.abs(want[3])]
    for k, c in enumerate(("px", "py", "pz", "E")):
        r, i = worst(np.abs(got[k] - want[k]), 6 * u * scales[k])
        assert r <= 1.0, (c, i, wp[1][i], wp[2][i], got[k][i], want[k][i])
