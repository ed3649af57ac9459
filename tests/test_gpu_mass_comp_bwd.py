"""GPU parity of the reverse mode of the cancellation-free pair mass against
the binary128 chain rule of the oracle: FP32 keeps its digits on nearly
collinear light pairs, where the plain FP32 reverse mode loses them."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import gpu, host, widened

pytestmark = pytest.mark.gpu
glv = pytest.importorskip("paper_2312_02756_amd.glv")
ag = pytest.importorskip("paper_2312_02756_amd.autograd")


def _ratio(got, want, rel):
    """Largest |got - want| / (rel * max_k |want_k|) over items and components."""
    w = np.stack(want)
    g = np.stack([host(c).astype(np.float64) for c in got])
    ref = np.max(np.abs(w), axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(np.abs(g - w) == 0, 0.0, np.abs(g - w) / (rel * ref))
    r = np.where(np.isnan(r), np.inf, r)  # a NaN gradient fails
    return float(np.max(r)) if r.size else 0.0


@pytest.mark.parametrize("dtype,rel", [(torch.float32, 2.0 ** -15), (torch.float64, 1e-12)])
def test_comp_bwd_against_binary128(dtype, rel):
    n = 40000
    sa, sb, collinear = synth.pairs_stress(synth.rng(980), n)
    gm = synth.upstream(synth.rng(981), n, 1)[0]
    a, b, g = gpu(sa, dtype), gpu(sb, dtype), gpu([gm], dtype)[0]
    ga, gb = glv.glv_invariant_mass_comp_bwd(a, b, g)
    wa, wb, wg = widened(sa, dtype), widened(sb, dtype), widened([gm], dtype)[0]
    qa, qb = oracle.mass_vjp_q(wa, wb, wg)
    assert _ratio(list(ga) + list(gb), list(qa) + list(qb), rel) <= 1.0
    if dtype == torch.float32:
        # the plain reverse mode of the same FP32 pairs misses this bar on the collinear ones
        pa, pb = glv.glv_invariant_mass_bwd(a, b, g)
        idx = np.nonzero(collinear)[0]
        sel = lambda cols: [c[idx] for c in cols]  # noqa: E731
        plain = [torch.from_numpy(host(c)[idx]) for c in list(pa) + list(pb)]
        assert _ratio(plain, sel(list(qa) + list(qb)), rel) > 10.0


def test_comp_bwd_generic_and_misaligned():
    n = 1001
    a, b = synth.pairs_generic(synth.rng(982), n + 1)
    gm = synth.upstream(synth.rng(983), n + 1, 1)[0]
    ga_, gb_, gg = gpu(a, torch.float32), gpu(b, torch.float32), gpu([gm], torch.float32)[0]
    full = glv.glv_invariant_mass_comp_bwd(ga_, gb_, gg)
    wa, wb, wg = widened(a, torch.float32), widened(b, torch.float32), widened([gm], torch.float32)[0]
    qa, qb = oracle.mass_vjp_q(wa, wb, wg)
    assert _ratio(list(full[0]) + list(full[1]), list(qa) + list(qb), 2.0 ** -15) <= 1.0
    # views one element in (one item per lane) give the same bits as the aligned packs
    mis = glv.glv_invariant_mass_comp_bwd(tuple(t[1:] for t in ga_), tuple(t[1:] for t in gb_), gg[1:])
    for u, v in zip(list(full[0]) + list(full[1]), list(mis[0]) + list(mis[1])):
        assert torch.equal(u[1:], v)


def test_autograd_compensated_uses_it():
    a, b, _ = synth.pairs_stress(synth.rng(984), 257)
    ca = tuple(t.requires_grad_(True) for t in gpu(a, torch.float32))
    cb = tuple(t.requires_grad_(True) for t in gpu(b, torch.float32))
    m = ag.invariant_mass(ca, cb, mode="compensated")
    m.sum().backward()
    ga, gb = glv.glv_invariant_mass_comp_bwd(tuple(t.detach() for t in ca), tuple(t.detach() for t in cb),
                                             torch.ones_like(m))
    assert all(torch.equal(t.grad, g) for t, g in zip(ca + cb, ga + gb))


def test_comp_bwd_full_size_sampled():
    """2^24 FP32 stress pairs (the compensated workload), 65,536 samples."""
    n = 1 << 24
    sa, sb, _ = synth.pairs_stress(synth.rng(synth.STRESS), n)
    sa, sb = synth.as_dtype(sa, np.float32), synth.as_dtype(sb, np.float32)
    gm = np.ones(n, dtype=np.float32)
    ga, gb = glv.glv_invariant_mass_comp_bwd(gpu(sa, torch.float32), gpu(sb, torch.float32),
                                             gpu([gm], torch.float32)[0])
    idx = np.sort(np.random.default_rng(16).choice(n, 65536, replace=False))
    ws = lambda cols: [np.asarray(c[idx], dtype=np.float64) for c in cols]  # noqa: E731
    qa, qb = oracle.mass_vjp_q(ws(sa), ws(sb), np.ones(idx.size))
    got = [torch.from_numpy(host(c)[idx]) for c in list(ga) + list(gb)]
    assert _ratio(got, list(qa) + list(qb), 2.0 ** -15) <= 1.0
