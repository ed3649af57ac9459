"""GPU parity of the general transformations (Sec. 3.1: Lorentz
transformations held as a 4x4 matrix, rotations as a 3x3 matrix or an axis
and angle) and their reverse modes against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import gpu, host, widened
from tolerances import U32, U64, worst

pytestmark = pytest.mark.gpu
glv = pytest.importorskip("paper_2312_02756_amd.glv")

KINDS = {"lorentz": 16, "rotate": 9, "axis_angle": 4}
FWD = {"lorentz": ("glv_lorentz_transform", oracle.lorentz_transform),
       "rotate": ("glv_rotate", oracle.rotate),
       "axis_angle": ("glv_rotate_axis_angle", oracle.rotate_axis_angle)}


def _params(kind, n, seed):
    g = synth.rng(seed)
    if kind == "axis_angle":
        return [g.normal(size=n), g.normal(size=n), g.normal(size=n), g.uniform(-7.0, 7.0, n)]
    return [g.normal(size=n) for _ in range(KINDS[kind])]


def _abs_apply(kind, m, x):
    """(|M| |x|) per output component: the rounding scale of each sum."""
    ax = [np.abs(c) for c in x]
    if kind == "lorentz":
        return [sum(np.abs(m[4 * a + c]) * ax[c] for c in range(4)) for a in range(4)]
    if kind == "rotate":
        return [sum(np.abs(m[3 * a + c]) * ax[c] for c in range(3)) for a in range(3)] + [ax[3]]
    p1 = ax[0] + ax[1] + ax[2]  # |R| <= 1 entrywise
    return [p1, p1, p1, ax[3]]


def _check(kind, got, want, scale, u, label):
    units = 16 if kind == "axis_angle" else 8  # the axis-angle matrix itself carries a few rounding units
    for k in range(4):
        r, i = worst(np.abs(host(got[k]).astype(np.float64) - want[k]), units * u * scale[k] + 1e-300)
        assert r <= 1.0, (label, k, i, host(got[k])[i], want[k][i])


@pytest.mark.parametrize("stride", [1, 0])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind", list(KINDS))
def test_forward_against_oracle(kind, dtype, stride):
    n = 4097
    x, _ = synth.boost_items(synth.rng(950), n + 1)
    m = _params(kind, n + 1 if stride else 1, 951)
    u = U64 if dtype == torch.float64 else U32
    gx, gm = gpu(x, dtype), gpu(m, dtype)
    fn = getattr(glv, FWD[kind][0])
    for sl in (slice(0, n), slice(1, n + 1)):  # aligned, and one element in (one item per lane)
        xs = tuple(t[sl] for t in gx)
        ms = tuple(t[sl] for t in gm) if stride else gm
        y = fn(xs, ms)
        wx = widened(tuple(c[sl] for c in x), dtype)
        wm = widened(tuple(c[sl] for c in m) if stride else m, dtype)
        want = FWD[kind][1](wx, wm, stride)
        _check(kind, y, want, _abs_apply(kind, wm, wx), u, (kind, str(dtype), stride, sl.start))


@pytest.mark.parametrize("kind", list(KINDS))
def test_in_place_equals_out_of_place(kind):
    x, _ = synth.boost_items(synth.rng(952), 1000)
    m = gpu(_params(kind, 1000, 953), torch.float64)
    fn = getattr(glv, FWD[kind][0])
    gx = gpu(x, torch.float64)
    ref = fn(gx, m)
    same = fn(gx, m, out=gx)
    assert all(torch.equal(a, b) for a, b in zip(ref, same)) and same[0].data_ptr() == gx[0].data_ptr()


def test_exact_cases():
    """Permutation matrices, the identity and a zero axis are exact on the GPU too."""
    x, _ = synth.boost_items(synth.rng(954), 999)
    gx = gpu(x, torch.float64)
    one = lambda vals: tuple(torch.tensor([float(v)], dtype=torch.float64, device="cuda:0") for v in vals)  # noqa
    y = [host(c) for c in glv.glv_rotate(gx, one((0, -1, 0, 1, 0, 0, 0, 0, 1)))]
    assert np.array_equal(y[0], -x[1]) and np.array_equal(y[1], x[0]) and np.array_equal(y[2], x[2])
    assert np.array_equal(y[3], x[3])
    eye = one([1.0 if a == c else 0.0 for a in range(4) for c in range(4)])
    assert all(np.array_equal(host(a), b) for a, b in zip(glv.glv_lorentz_transform(gx, eye), x))
    z = [host(c) for c in glv.glv_rotate_axis_angle(gx, one((0, 0, 0, 2.0)))]
    assert all(np.array_equal(a, b) for a, b in zip(z, x))


@pytest.mark.parametrize("stride", [1, 0])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind", list(KINDS))
def test_reverse_against_oracle(kind, dtype, stride):
    n = 2049
    x, _ = synth.boost_items(synth.rng(955), n)
    m = _params(kind, n if stride else 1, 956)
    gy = synth.upstream(synth.rng(957), n, 4)
    u = U64 if dtype == torch.float64 else U32
    wx, wm, wg = widened(x, dtype), widened(m, dtype), widened(gy, dtype)
    if kind == "axis_angle":
        got = glv.glv_rotate_axis_angle_bwd(gpu(m, dtype), gpu(gy, dtype))
        want = oracle.rotate_axis_angle_vjp(wm, wg, stride)
        _check(kind, got, want, _abs_apply(kind, wm, wg), u, (kind, "bwd"))
        return
    want_m = stride == 1
    fn = glv.glv_lorentz_transform_bwd if kind == "lorentz" else glv.glv_rotate_bwd
    gxx, gmm = fn(gpu(x, dtype), gpu(m, dtype), gpu(gy, dtype), want_matrix=want_m)
    ofn = oracle.lorentz_transform_vjp if kind == "lorentz" else oracle.rotate_vjp
    wgx, wgm = ofn(wx, wm, wg, stride, want_m)
    N = 4 if kind == "lorentz" else 3
    # grad_x = M^T g: the scale of each sum is (|M|^T |g|)
    scale = [sum(np.abs(wm[N * a + c]) * np.abs(wg[a]) for a in range(N)) for c in range(N)]
    if N == 3:
        scale.append(np.abs(wg[3]))
    for k in range(4):
        r, i = worst(np.abs(host(gxx[k]).astype(np.float64) - wgx[k]), 8 * u * scale[k] + 1e-300)
        assert r <= 1.0, (kind, "grad_x", k, i)
    if want_m:
        for k in range(N * N):  # one rounded product each
            r, i = worst(np.abs(host(gmm[k]).astype(np.float64) - wgm[k]), u * np.abs(wgm[k]) + 1e-300)
            assert r <= 1.0, (kind, "grad_m", k, i)
    else:
        assert gmm is None


def test_lorentz_full_size_sampled():
    """2^24 FP64 vectors with one matrix each, forward and reverse mode (with
    the matrix gradient), in the measured launch shape; 65,536 samples."""
    n = 1 << 24
    g = synth.rng(synth.LARGE)
    x, _ = synth.boost_items(g, n)
    m = [g.normal(size=n) for _ in range(16)]
    gy = synth.upstream(synth.rng(synth.GRADS), n, 4)
    gx_, gm_, gg_ = gpu(x, torch.float64), gpu(m, torch.float64), gpu(gy, torch.float64)
    y = [host(c) for c in glv.glv_lorentz_transform(gx_, gm_)]
    rgx, rgm = glv.glv_lorentz_transform_bwd(gx_, gm_, gg_)
    rgx, rgm = [host(c) for c in rgx], [host(c) for c in rgm]
    idx = np.sort(np.random.default_rng(14).choice(n, 65536, replace=False))
    xs, ms, gs = [c[idx] for c in x], [c[idx] for c in m], [c[idx] for c in gy]
    want = oracle.lorentz_transform(xs, ms, 1)
    _check("lorentz", [torch.from_numpy(c[idx]) for c in y], want, _abs_apply("lorentz", ms, xs), U64, "full fwd")
    wgx, wgm = oracle.lorentz_transform_vjp(xs, ms, gs, 1)
    scale = [sum(np.abs(ms[4 * a + c]) * np.abs(gs[a]) for a in range(4)) for c in range(4)]
    for k in range(4):
        r, _ = worst(np.abs(rgx[k][idx] - wgx[k]), 8 * U64 * scale[k] + 1e-300)
        assert r <= 1.0
    for k in range(16):
        r, _ = worst(np.abs(rgm[k][idx] - wgm[k]), U64 * np.abs(wgm[k]) + 1e-300)
        assert r <= 1.0


def test_empty_inputs():
    e = tuple(torch.empty(0, dtype=torch.float64, device="cuda:0") for _ in range(4))
    one = lambda k: tuple(torch.ones(1, dtype=torch.float64, device="cuda:0") for _ in range(k))  # noqa: E731
    assert all(t.numel() == 0 for t in glv.glv_lorentz_transform(e, one(16)))
    assert all(t.numel() == 0 for t in glv.glv_rotate(e, one(9)))
    assert all(t.numel() == 0 for t in glv.glv_rotate_axis_angle(e, one(4)))
    assert all(t.numel() == 0 for t in glv.glv_convert(e, "PxPyPzE", "PtEtaPhiM"))
