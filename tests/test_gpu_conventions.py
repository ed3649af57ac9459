"""The documented value conventions on the GPU, against the oracle where it
defines them: spacelike sums give -sqrt(-q), NaN propagates, the mass
gradient is zero where m = 0, |beta| >= 1 is not checked (inf/NaN out), and
empty inputs launch nothing."""

import math

import numpy as np
import pytest
import torch

import oracle
from gpu_util import gpu, host

pytestmark = pytest.mark.gpu

glv = pytest.importorskip("paper_2312_02756_amd.glv")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_spacelike_and_lightlike_sums(dtype):
    a = (np.array([3.0, 0.0, 5.0, 1.0]), np.array([0.0, 4.0, 0.0, 2.0]), np.array([0.0, 0.0, 0.0, 2.0]),
         np.array([1.0, 1.0, 4.0, 3.0]))
    b = (np.array([0.0, 0.0, 0.0, 1.0]), np.array([0.0, 0.0, 12.0, 2.0]), np.array([0.0, 0.0, 0.0, 2.0]),
         np.array([1.0, 2.0, 9.0, 3.0]))
    m = host(glv.glv_invariant_mass(gpu(a, dtype), gpu(b, dtype), coords="PxPyPzE"))
    want = oracle.mass_plain("PxPyPzE", a, b)
    assert want[0] == -math.sqrt(5.0) and want[2] == 0.0 and want[3] == 0.0
    assert np.allclose(m, want, rtol=1e-6 if dtype == torch.float32 else 1e-15, atol=0)
    assert m[2] == 0.0 and m[3] == 0.0


def test_nan_propagates_and_zero_mass_gradient_is_zero():
    a = (np.array([np.nan, 3.0]), np.array([0.0, 4.0]), np.array([0.0, 0.0]), np.array([1.0, 5.0]))
    b = (np.array([1.0, 3.0]), np.array([0.0, 4.0]), np.array([0.0, 0.0]), np.array([2.0, 5.0]))
    ga, gb = gpu(a, torch.float64), gpu(b, torch.float64)
    m = host(glv.glv_invariant_mass(ga, gb, coords="PxPyPzE"))
    assert np.isnan(m[0]) and m[1] == 0.0  # second pair: two identical lightlike vectors
    da, db = glv.glv_invariant_mass_bwd(ga, gb, torch.ones(2, dtype=torch.float64, device="cuda:0"),
                                        coords="PxPyPzE")
    assert all(host(t)[1] == 0.0 for t in da + db)


def test_superluminal_velocity_is_not_checked():
    x = (np.array([1.0]), np.array([0.0]), np.array([0.0]), np.array([2.0]))
    beta = (np.array([1.0]), np.array([0.0]), np.array([0.0]))
    y = host(glv.glv_boost(gpu(x, torch.float64), gpu(beta, torch.float64)))
    assert all(not np.isfinite(c[0]) for c in (y[0], y[3]))
    beta = (np.array([0.8]), np.array([0.8]), np.array([0.0]))  # |beta| > 1: sqrt of a negative
    y = host(glv.glv_boost(gpu(x, torch.float64), gpu(beta, torch.float64)))
    assert np.isnan(y[3][0])


def test_empty_inputs():
    e = torch.empty(0, dtype=torch.float64, device="cuda:0")
    m = glv.glv_invariant_mass((e,) * 4, (e,) * 4)
    assert m.numel() == 0
    y = glv.glv_boost((e,) * 4, (e,) * 3)
    assert all(t.numel() == 0 for t in y)
    off = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    po = glv.glv_pair_offsets(off)
    assert po.numel() == 1 and int(po.item()) == 0
    total, em, pm = glv.glv_event_reduce((e,) * 4, off, po)
    assert em.numel() == 0 and pm.numel() == 0
