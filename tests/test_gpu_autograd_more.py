"""torch.autograd.gradcheck of the wrappers around the conversion and the
general transformations: their backward (the library's _bwd kernels)
against central differences of their forward (FP64)."""
import itertools

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import gpu

pytestmark = pytest.mark.gpu
ag = pytest.importorskip("paper_2312_02756_amd.autograd")

SYSTEMS = ["PxPyPzE", "PtEtaPhiM", "PtEtaPhiE", "PxPyPzM"]


@pytest.mark.parametrize("src,dst", [p for p in itertools.permutations(SYSTEMS, 2)])
def test_gradcheck_convert(src, dst):
    a, _ = synth.pairs_generic(synth.rng(970), 24)
    a = (a[0], a[1], a[2], a[3] + 20.0)  # masses well above the rounding of E^2 - |p|^2
    cols = tuple(t.requires_grad_(True) for t in gpu(oracle.convert("PtEtaPhiM", src, a), torch.float64))
    assert torch.autograd.gradcheck(lambda *c: ag.Convert.apply(src, dst, *c), cols, eps=1e-6, atol=1e-5,
                                    rtol=1e-4)


@pytest.mark.parametrize("kind,k", [("lorentz", 16), ("rotate", 9)])
def test_gradcheck_matrices(kind, k):
    x, _ = synth.boost_items(synth.rng(971), 16)
    m = [synth.rng(972 + i).normal(size=16) for i in range(k)]
    cols = tuple(t.requires_grad_(True) for t in gpu(tuple(x) + tuple(m), torch.float64))
    assert torch.autograd.gradcheck(lambda *c: ag.LorentzTransform.apply(kind, *c), cols, eps=1e-6, atol=1e-6,
                                    rtol=1e-5)


def test_gradcheck_axis_angle_and_broadcast():
    x, _ = synth.boost_items(synth.rng(975), 16)
    xs = tuple(t.requires_grad_(True) for t in gpu(x, torch.float64))
    aa = gpu((np.array([0.3]), np.array([-1.2]), np.array([0.5]), np.array([2.1])), torch.float64)
    assert torch.autograd.gradcheck(lambda *c: ag.RotateAxisAngle.apply(*c, *aa), xs, eps=1e-6, atol=1e-6,
                                    rtol=1e-5)
    one = gpu([np.array([v]) for v in synth.rng(976).normal(size=16)], torch.float64)
    assert torch.autograd.gradcheck(lambda *c: ag.LorentzTransform.apply("lorentz", *c, *one), xs, eps=1e-6,
                                    atol=1e-6, rtol=1e-5)
    y = ag.lorentz_transform(xs, one)
    sum(t.sum() for t in y).backward()
    assert all(t.grad is not None for t in xs)
