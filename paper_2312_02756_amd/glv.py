"""Python binding of the C ABI (include/glv.h), one function per entry point
with the same name.  Argument marshalling only: tensors are checked (same GPU,
dtype, contiguous) and their device pointers handed to the library together
with torch's current HIP stream; every step of the computation runs in the
library's gfx950 kernels.  Outputs are allocated here with torch (the
library itself never allocates).

Coordinates are given as "PxPyPzE", "PtEtaPhiM", "PtEtaPhiE" or "PxPyPzM"; modes as
"plain" or "compensated".
"""

import ctypes

import torch

from . import _lib
from ._lib import P3, P4, check, glv_tiling

COORDS = {"PxPyPzE": _lib.GLV_PXPYPZE, "PtEtaPhiM": _lib.GLV_PTETAPHIM, "PtEtaPhiE": _lib.GLV_PTETAPHIE,
          "PxPyPzM": _lib.GLV_PXPYPZM}
MODES = {"plain": _lib.GLV_PLAIN, "compensated": _lib.GLV_COMPENSATED}
DTYPES = {torch.float32: _lib.GLV_F32, torch.float64: _lib.GLV_F64}


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _cols(ts, n_expected, dtype, device, name):
    ts = tuple(ts)
    for t in ts:
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name}: expected tensors")
        if t.device != device or t.dtype != dtype:
            raise ValueError(f"{name}: all columns must be {dtype} on {device}")
        if not t.is_contiguous() or t.dim() != 1:
            raise ValueError(f"{name}: columns must be contiguous 1-D tensors")
        if n_expected is not None and t.numel() != n_expected:
            raise ValueError(f"{name}: expected {n_expected} elements, got {t.numel()}")
    return ts


def _dtype_code(dtype):
    if dtype not in DTYPES:
        raise ValueError(f"unsupported dtype {dtype}")
    return DTYPES[dtype]


def _coords_code(coords):
    return COORDS[coords] if isinstance(coords, str) else int(coords)


def _mode_code(mode):
    return MODES[mode] if isinstance(mode, str) else int(mode)


def _check_device(t):
    if t.device.type != "cuda":
        raise ValueError("inputs must be GPU tensors")


# ---------------------------------------------------------------- pair mass

def glv_invariant_mass(a, b, coords="PtEtaPhiM", mode="plain", out=None, fallback_count=None):
    """m[i] = mass(conv(a_i) + conv(b_i)).  ``fallback_count``: optional int64
    GPU tensor of one element, incremented by the number of FP32 items the
    compensated mode recomputed in FP64."""
    dev, dt = a[0].device, a[0].dtype
    _check_device(a[0])
    n = a[0].numel()
    a = _cols(a, n, dt, dev, "a")
    b = _cols(b, n, dt, dev, "b")
    m = torch.empty(n, dtype=dt, device=dev) if out is None else _cols([out], n, dt, dev, "out")[0]
    fb = None
    if fallback_count is not None:
        if fallback_count.dtype != torch.int64 or fallback_count.device != dev or fallback_count.numel() != 1:
            raise ValueError("fallback_count must be one int64 element on the inputs' device")
        fb = fallback_count
    lib = _lib.load()
    check("glv_invariant_mass",
          lib.glv_invariant_mass(_dtype_code(dt), _coords_code(coords), _mode_code(mode), n,
                                 P4(*[t.data_ptr() for t in a]), P4(*[t.data_ptr() for t in b]), _ptr(m), _ptr(fb),
                                 _stream(dev)))
    return m


def glv_invariant_mass_comp_bwd(a, b, grad_m):
    """Gradients of the cancellation-free pair mass of PtEtaPhiM legs (the
    reverse mode that keeps its digits for nearly collinear light pairs)."""
    dev, dt = a[0].device, a[0].dtype
    _check_device(a[0])
    n = a[0].numel()
    a = _cols(a, n, dt, dev, "a")
    b = _cols(b, n, dt, dev, "b")
    (grad_m,) = _cols([grad_m], n, dt, dev, "grad_m")
    ga = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(4))
    gb = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(4))
    check("glv_invariant_mass_comp_bwd",
          _lib.load().glv_invariant_mass_comp_bwd(_dtype_code(dt), n, P4(*[t.data_ptr() for t in a]),
                                                  P4(*[t.data_ptr() for t in b]), _ptr(grad_m),
                                                  P4(*[t.data_ptr() for t in ga]), P4(*[t.data_ptr() for t in gb]),
                                                  _stream(dev)))
    return ga, gb


def glv_invariant_mass_bwd(a, b, grad_m, coords="PtEtaPhiM"):
    dev, dt = a[0].device, a[0].dtype
    _check_device(a[0])
    n = a[0].numel()
    a = _cols(a, n, dt, dev, "a")
    b = _cols(b, n, dt, dev, "b")
    (grad_m,) = _cols([grad_m], n, dt, dev, "grad_m")
    ga = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(4))
    gb = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(4))
    lib = _lib.load()
    check("glv_invariant_mass_bwd",
          lib.glv_invariant_mass_bwd(_dtype_code(dt), _coords_code(coords), n, P4(*[t.data_ptr() for t in a]),
                                     P4(*[t.data_ptr() for t in b]), _ptr(grad_m),
                                     P4(*[t.data_ptr() for t in ga]), P4(*[t.data_ptr() for t in gb]),
                                     _stream(dev)))
    return ga, gb


# -------------------------------------------------------------------- boost

def glv_boost(x, beta, out=None):
    """Active boost of Cartesian (px, py, pz, E) columns by beta (3 columns of
    n items, or of 1 element = one velocity for all).  ``out`` may be ``x``
    itself (in place)."""
    dev, dt = x[0].device, x[0].dtype
    _check_device(x[0])
    n = x[0].numel()
    x = _cols(x, n, dt, dev, "x")
    bs = 1 if beta[0].numel() == n else 0
    beta = _cols(beta, n if bs else 1, dt, dev, "beta")
    y = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(4)) if out is None else _cols(out, n, dt, dev, "out")
    lib = _lib.load()
    check("glv_boost", lib.glv_boost(_dtype_code(dt), n, P4(*[t.data_ptr() for t in x]),
                                     P3(*[t.data_ptr() for t in beta]), bs, P4(*[t.data_ptr() for t in y]),
                                     _stream(dev)))
    return y


def glv_boost_bwd(x, beta, grad_y, want_beta=True):
    dev, dt = x[0].device, x[0].dtype
    _check_device(x[0])
    n = x[0].numel()
    x = _cols(x, n, dt, dev, "x")
    bs = 1 if beta[0].numel() == n else 0
    beta = _cols(beta, n if bs else 1, dt, dev, "beta")
    gy = _cols(grad_y, n, dt, dev, "grad_y")
    gx = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(4))
    gbeta = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(3)) if want_beta else None
    lib = _lib.load()
    gb_arg = P3(*[t.data_ptr() for t in gbeta]) if want_beta else None
    check("glv_boost_bwd", lib.glv_boost_bwd(_dtype_code(dt), n, P4(*[t.data_ptr() for t in x]),
                                             P3(*[t.data_ptr() for t in beta]), bs, P4(*[t.data_ptr() for t in gy]),
                                             P4(*[t.data_ptr() for t in gx]), gb_arg, _stream(dev)))
    return gx, gbeta


# ---------------------------------------------------- general transformations

_TF = {"lorentz": ("glv_lorentz_transform", 16, 16), "rotate": ("glv_rotate", 9, 9),
       "axis_angle": ("glv_rotate_axis_angle", 4, None)}


def _params(m, n, k, dt, dev, name):
    if len(m) != k:
        raise ValueError(f"{name}: expected {k} columns, got {len(m)}")
    stride = 1 if m[0].numel() == n else 0
    return _cols(m, n if stride else 1, dt, dev, name), stride


def _transform(kind, x, m, out):
    fn, k, _ = _TF[kind]
    dev, dt = x[0].device, x[0].dtype
    _check_device(x[0])
    n = x[0].numel()
    x = _cols(x, n, dt, dev, "x")
    m, stride = _params(m, n, k, dt, dev, "matrix" if k > 4 else "axis_angle")
    y = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(4)) if out is None else _cols(out, n, dt, dev, "out")
    arr = ctypes.c_void_p * k
    check(fn, getattr(_lib.load(), fn)(_dtype_code(dt), n, P4(*[t.data_ptr() for t in x]),
                                       arr(*[t.data_ptr() for t in m]), stride, P4(*[t.data_ptr() for t in y]),
                                       _stream(dev)))
    return y


def glv_lorentz_transform(x, L, out=None):
    """y = L x for Cartesian (px, py, pz, E) columns; L = 16 row-major columns
    of n items, or of 1 element = one matrix for all.  ``out`` may be ``x``."""
    return _transform("lorentz", x, L, out)


def glv_rotate(x, R, out=None):
    """Rotation3D: R = 9 row-major columns (n items or 1 element) applied to
    (px, py, pz); E passes through."""
    return _transform("rotate", x, R, out)


def glv_rotate_axis_angle(x, axis_angle, out=None):
    """AxisAngle: axis_angle = (ax, ay, az, angle) columns (n items or 1 element)."""
    return _transform("axis_angle", x, axis_angle, out)


def _transform_bwd(kind, x, m, grad_y, want_matrix):
    fn, k, nn = _TF[kind]
    dev, dt = grad_y[0].device, grad_y[0].dtype
    _check_device(grad_y[0])
    n = grad_y[0].numel()
    gy = _cols(grad_y, n, dt, dev, "grad_y")
    m, stride = _params(m, n, k, dt, dev, "matrix" if k > 4 else "axis_angle")
    gx = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(4))
    lib = _lib.load()
    arr = ctypes.c_void_p * k
    if kind == "axis_angle":
        check(fn + "_bwd", lib.glv_rotate_axis_angle_bwd(_dtype_code(dt), n, arr(*[t.data_ptr() for t in m]), stride,
                                                        P4(*[t.data_ptr() for t in gy]),
                                                        P4(*[t.data_ptr() for t in gx]), _stream(dev)))
        return gx
    gm = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(nn)) if want_matrix else None
    xp = P4(*[t.data_ptr() for t in _cols(x, n, dt, dev, "x")]) if x is not None else None
    gm_arg = (ctypes.c_void_p * nn)(*[t.data_ptr() for t in gm]) if gm else None
    check(fn + "_bwd", getattr(lib, fn + "_bwd")(_dtype_code(dt), n, xp, arr(*[t.data_ptr() for t in m]), stride,
                                                 P4(*[t.data_ptr() for t in gy]), P4(*[t.data_ptr() for t in gx]),
                                                 gm_arg, _stream(dev)))
    return gx, gm


def glv_lorentz_transform_bwd(x, L, grad_y, want_matrix=True):
    """(grad_x, grad_L): L^T grad_y and the per-item grad_y x^T (16 columns;
    needs one matrix per item)."""
    return _transform_bwd("lorentz", x, L, grad_y, want_matrix)


def glv_rotate_bwd(x, R, grad_y, want_matrix=True):
    """(grad_x, grad_R) of glv_rotate."""
    return _transform_bwd("rotate", x, R, grad_y, want_matrix)


def glv_rotate_axis_angle_bwd(axis_angle, grad_y):
    """grad_x of glv_rotate_axis_angle (the rotation by the opposite angle)."""
    return _transform_bwd("axis_angle", None, axis_angle, grad_y, False)


# ------------------------------------------------------------ jagged events

def glv_convert(cols, from_coords, to_coords, out=None):
    """The ``to_coords`` coordinates of vectors given in ``from_coords`` (4
    columns each).  ``out`` may be ``cols`` itself (in place)."""
    dev, dt = cols[0].device, cols[0].dtype
    _check_device(cols[0])
    n = cols[0].numel()
    cols = _cols(cols, n, dt, dev, "cols")
    y = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(4)) if out is None else _cols(out, n, dt, dev, "out")
    check("glv_convert", _lib.load().glv_convert(_dtype_code(dt), _coords_code(from_coords), _coords_code(to_coords),
                                                 n, P4(*[t.data_ptr() for t in cols]), P4(*[t.data_ptr() for t in y]),
                                                 _stream(dev)))
    return y


def glv_convert_bwd(cols, grad_out, from_coords, to_coords):
    """(d convert / d cols)^T grad_out, 4 columns."""
    dev, dt = cols[0].device, cols[0].dtype
    _check_device(cols[0])
    n = cols[0].numel()
    cols = _cols(cols, n, dt, dev, "cols")
    grad_out = _cols(grad_out, n, dt, dev, "grad_out")
    g = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(4))
    check("glv_convert_bwd",
          _lib.load().glv_convert_bwd(_dtype_code(dt), _coords_code(from_coords), _coords_code(to_coords), n,
                                      P4(*[t.data_ptr() for t in cols]), P4(*[t.data_ptr() for t in grad_out]),
                                      P4(*[t.data_ptr() for t in g]), _stream(dev)))
    return g


def glv_mass_histogram(m, lo, hi, n_bins, counts=None):
    """Counts (n_bins + 2 uint64 as int64: underflow, the bins, overflow) of the
    masses ``m`` in n_bins equal bins of [lo, hi).  ``counts``, if given, is
    added to (accumulate several batches)."""
    dev, dt = m.device, m.dtype
    _check_device(m)
    (m,) = _cols((m,), m.numel(), dt, dev, "m")
    if counts is None:
        counts = torch.zeros(int(n_bins) + 2, dtype=torch.int64, device=dev)
    elif counts.dtype != torch.int64 or counts.numel() != int(n_bins) + 2 or not counts.is_contiguous():
        raise ValueError("counts must be a contiguous int64 tensor of n_bins + 2 elements")
    check("glv_mass_histogram", _lib.load().glv_mass_histogram(_dtype_code(dt), m.numel(), _ptr(m), float(lo),
                                                               float(hi), int(n_bins), _ptr(counts), _stream(dev)))
    return counts


def glv_event_best_pair(pair_offsets, pair_m, target):
    """(rank, mass) per event of its pair closest to ``target`` (rank -1 and
    NaN for an event without one)."""
    _check_device(pair_m)
    dev, dt = pair_m.device, pair_m.dtype
    po = _offsets(pair_offsets, dev)
    ne = po.numel() - 1
    rank = torch.empty(ne, dtype=torch.int64, device=dev)
    bm = torch.empty(ne, dtype=dt, device=dev)
    check("glv_event_best_pair", _lib.load().glv_event_best_pair(_dtype_code(dt), ne, _ptr(po), _ptr(pair_m),
                                                                 float(target), _ptr(rank), _ptr(bm), _stream(dev)))
    return rank, bm


def glv_invariant_mass_histogram(a, b, lo, hi, n_bins, coords="PtEtaPhiM", mode="plain", counts=None,
                                 fallback_count=None):
    """The pair masses of glv_invariant_mass(a, b, coords, mode) counted into
    n_bins equal bins of [lo, hi) plus under- and overflow (n_bins + 2 int64)
    without being stored; ``counts``, if given, is added to."""
    dev, dt = a[0].device, a[0].dtype
    _check_device(a[0])
    n = a[0].numel()
    a = _cols(a, n, dt, dev, "a")
    b = _cols(b, n, dt, dev, "b")
    if counts is None:
        counts = torch.zeros(int(n_bins) + 2, dtype=torch.int64, device=dev)
    elif counts.dtype != torch.int64 or counts.numel() != int(n_bins) + 2 or not counts.is_contiguous():
        raise ValueError("counts must be a contiguous int64 tensor of n_bins + 2 elements")
    check("glv_invariant_mass_histogram",
          _lib.load().glv_invariant_mass_histogram(_dtype_code(dt), _coords_code(coords), _mode_code(mode), n,
                                                   P4(*[t.data_ptr() for t in a]), P4(*[t.data_ptr() for t in b]),
                                                   float(lo), float(hi), int(n_bins), _ptr(counts),
                                                   _ptr(fallback_count), _stream(dev)))
    return counts


def glv_event_reduce_best_pair(p, offsets, target, pair_offsets=None, coords="PtEtaPhiM", mode="plain", tiling=None,
                               fallback_count=None):
    """(rank, mass) per event of its pair closest to ``target``, chosen inside
    the jagged reduction without writing pair masses (rank -1 and NaN for an
    event without one)."""
    dev, dt = p[0].device, p[0].dtype
    _check_device(p[0])
    offsets = _offsets(offsets, dev)
    ne = offsets.numel() - 1
    p = _cols(p, p[0].numel(), dt, dev, "p")
    if pair_offsets is None:
        pair_offsets = glv_pair_offsets(offsets)
    pair_offsets = _offsets(pair_offsets, dev)
    rank = torch.empty(ne, dtype=torch.int64, device=dev)
    bm = torch.empty(ne, dtype=dt, device=dev)
    check("glv_event_reduce_best_pair",
          _lib.load().glv_event_reduce_best_pair(_dtype_code(dt), _coords_code(coords), _mode_code(mode), ne,
                                                 _ptr(offsets), _ptr(pair_offsets), P4(*[t.data_ptr() for t in p]),
                                                 float(target), _ptr(rank), _ptr(bm), _ptr(fallback_count),
                                                 _tiling(tiling), _stream(dev)))
    return rank, bm


def _offsets(offsets, dev):
    if offsets.dtype != torch.int64 or offsets.device != dev or not offsets.is_contiguous() or offsets.dim() != 1:
        raise ValueError("offsets must be a contiguous 1-D int64 tensor on the particles' device")
    return offsets


def glv_pair_offsets(offsets):
    _check_device(offsets)
    offsets = _offsets(offsets, offsets.device)
    ne = offsets.numel() - 1
    po = torch.empty(ne + 1, dtype=torch.int64, device=offsets.device)
    check("glv_pair_offsets", _lib.load().glv_pair_offsets(ne, _ptr(offsets), _ptr(po), _stream(offsets.device)))
    return po


def glv_validate_offsets(offsets, n_particles):
    """Number of violations (GPU int64 tensor of one element; 0 = valid)."""
    _check_device(offsets)
    offsets = _offsets(offsets, offsets.device)
    bad = torch.zeros(1, dtype=torch.int64, device=offsets.device)
    check("glv_validate_offsets",
          _lib.load().glv_validate_offsets(offsets.numel() - 1, _ptr(offsets), int(n_particles), _ptr(bad),
                                           _stream(offsets.device)))
    return bad


def _tiling(t):
    """A glv_tiling from (block, events_per_tile, lds_particles[, pairs_per_round]);
    0 or a missing pairs_per_round = the library's choice."""
    if t is None:
        return None
    if isinstance(t, glv_tiling):
        return ctypes.byref(t)
    t = tuple(t) + (0,) * (4 - len(t))
    return ctypes.byref(glv_tiling(*t))


def _as_tuple(t):
    return (t.block, t.events_per_tile, t.lds_particles, t.pairs_per_round)


def glv_event_reduce(p, offsets, pair_offsets=None, coords="PtEtaPhiM", mode="plain", want_total=True,
                     want_event_m=True, want_pair_m=True, tiling=None, fallback_count=None, n_pairs=None):
    """Returns (total (4 tensors) or None, event_m or None, pair_m or None).
    ``n_pairs`` (the last pair offset) avoids a device-to-host read when given."""
    dev, dt = p[0].device, p[0].dtype
    _check_device(p[0])
    offsets = _offsets(offsets, dev)
    ne = offsets.numel() - 1
    p = _cols(p, p[0].numel(), dt, dev, "p")
    need_po = want_pair_m or (_mode_code(mode) == _lib.GLV_COMPENSATED and want_event_m)
    if need_po and pair_offsets is None:
        pair_offsets = glv_pair_offsets(offsets)
    if pair_offsets is not None:
        pair_offsets = _offsets(pair_offsets, dev)
    total = tuple(torch.empty(ne, dtype=dt, device=dev) for _ in range(4)) if want_total else None
    em = torch.empty(ne, dtype=dt, device=dev) if want_event_m else None
    pm = None
    if want_pair_m:
        if n_pairs is None:
            n_pairs = int(pair_offsets[-1].item()) if ne > 0 else 0
        pm = torch.empty(int(n_pairs), dtype=dt, device=dev)
    lib = _lib.load()
    check("glv_event_reduce",
          lib.glv_event_reduce(_dtype_code(dt), _coords_code(coords), _mode_code(mode), ne, _ptr(offsets),
                               _ptr(pair_offsets), P4(*[t.data_ptr() for t in p]),
                               P4(*[t.data_ptr() for t in total]) if total else None, _ptr(em), _ptr(pm),
                               _ptr(fallback_count), _tiling(tiling), _stream(dev)))
    return total, em, pm


def glv_event_reduce_bwd(p, offsets, pair_offsets=None, grad_total=None, grad_event_m=None, grad_pair_m=None,
                         coords="PtEtaPhiM", tiling=None, total=None):
    """Reverse mode of glv_event_reduce (plain).  `total`: the forward's event
    totals (4 columns), if at hand -- then glv_event_reduce_bwd_totals, which
    takes the event-mass term's V from them instead of summing it again."""
    dev, dt = p[0].device, p[0].dtype
    _check_device(p[0])
    offsets = _offsets(offsets, dev)
    ne = offsets.numel() - 1
    n = p[0].numel()
    p = _cols(p, n, dt, dev, "p")
    if grad_pair_m is not None and pair_offsets is None:
        pair_offsets = glv_pair_offsets(offsets)
    gt = _cols(grad_total, ne, dt, dev, "grad_total") if grad_total is not None else None
    gem = _cols([grad_event_m], ne, dt, dev, "grad_event_m")[0] if grad_event_m is not None else None
    gpm = _cols([grad_pair_m], None, dt, dev, "grad_pair_m")[0] if grad_pair_m is not None else None
    gp = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(4))
    lib = _lib.load()
    gtp = P4(*[t.data_ptr() for t in gt]) if gt else None
    if total is not None:
        tot = _cols(total, ne, dt, dev, "total")
        check("glv_event_reduce_bwd_totals",
              lib.glv_event_reduce_bwd_totals(_dtype_code(dt), _coords_code(coords), ne, _ptr(offsets),
                                              _ptr(pair_offsets), P4(*[t.data_ptr() for t in p]),
                                              P4(*[t.data_ptr() for t in tot]), gtp, _ptr(gem), _ptr(gpm),
                                              P4(*[t.data_ptr() for t in gp]), _tiling(tiling), _stream(dev)))
        return gp
    check("glv_event_reduce_bwd",
          lib.glv_event_reduce_bwd(_dtype_code(dt), _coords_code(coords), ne, _ptr(offsets), _ptr(pair_offsets),
                                   P4(*[t.data_ptr() for t in p]), gtp, _ptr(gem), _ptr(gpm),
                                   P4(*[t.data_ptr() for t in gp]), _tiling(tiling), _stream(dev)))
    return gp


def glv_autotune_event_reduce(p, offsets, pair_offsets=None, coords="PtEtaPhiM", mode="plain"):
    """Times candidate tilings on these inputs, keeps the fastest for this
    process (device, dtype, coords, mode) and returns it as (block,
    events_per_tile, lds_particles, pairs_per_round)."""
    dev, dt = p[0].device, p[0].dtype
    _check_device(p[0])
    offsets = _offsets(offsets, dev)
    ne = offsets.numel() - 1
    if pair_offsets is None:
        pair_offsets = glv_pair_offsets(offsets)
    n_pairs = int(pair_offsets[-1].item()) if ne > 0 else 0
    total = tuple(torch.empty(ne, dtype=dt, device=dev) for _ in range(4))
    em = torch.empty(ne, dtype=dt, device=dev)
    pm = torch.empty(n_pairs, dtype=dt, device=dev)
    best = glv_tiling()
    check("glv_autotune_event_reduce",
          _lib.load().glv_autotune_event_reduce(_dtype_code(dt), _coords_code(coords), _mode_code(mode), ne,
                                                _ptr(offsets), _ptr(pair_offsets), P4(*[t.data_ptr() for t in p]),
                                                P4(*[t.data_ptr() for t in total]), _ptr(em), _ptr(pm),
                                                ctypes.byref(best), _stream(dev)))
    return _as_tuple(best)


def glv_current_tiling(dtype=torch.float64, coords="PtEtaPhiM", mode="plain"):
    t = glv_tiling()
    check("glv_current_tiling", _lib.load().glv_current_tiling(_dtype_code(dtype), _coords_code(coords),
                                                               _mode_code(mode), ctypes.byref(t)))
    return _as_tuple(t)


def glv_autotune_event_reduce_bwd(p, offsets, pair_offsets=None, grad_total=None, grad_event_m=None,
                                  grad_pair_m=None, coords="PtEtaPhiM"):
    """Times the backward's candidate tilings on these inputs and upstreams,
    keeps the fastest for this process (device, dtype, coords) and returns
    it as (block, events_per_tile, lds_particles, pairs_per_round)."""
    dev, dt = p[0].device, p[0].dtype
    _check_device(p[0])
    offsets = _offsets(offsets, dev)
    ne = offsets.numel() - 1
    n = p[0].numel()
    p = _cols(p, n, dt, dev, "p")
    if grad_pair_m is not None and pair_offsets is None:
        pair_offsets = glv_pair_offsets(offsets)
    gt = _cols(grad_total, ne, dt, dev, "grad_total") if grad_total is not None else None
    gem = _cols([grad_event_m], ne, dt, dev, "grad_event_m")[0] if grad_event_m is not None else None
    gpm = _cols([grad_pair_m], None, dt, dev, "grad_pair_m")[0] if grad_pair_m is not None else None
    gp = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(4))
    best = glv_tiling()
    check("glv_autotune_event_reduce_bwd",
          _lib.load().glv_autotune_event_reduce_bwd(
              _dtype_code(dt), _coords_code(coords), ne, _ptr(offsets), _ptr(pair_offsets),
              P4(*[t.data_ptr() for t in p]), P4(*[t.data_ptr() for t in gt]) if gt else None, _ptr(gem),
              _ptr(gpm), P4(*[t.data_ptr() for t in gp]), ctypes.byref(best), _stream(dev)))
    return _as_tuple(best)


def glv_current_tiling_bwd(dtype=torch.float64, coords="PtEtaPhiM"):
    t = glv_tiling()
    check("glv_current_tiling_bwd", _lib.load().glv_current_tiling_bwd(_dtype_code(dtype), _coords_code(coords),
                                                                       ctypes.byref(t)))
    return _as_tuple(t)


def _key_args(dtype, coords, mode, backward, offsets):
    if offsets is None:
        return _dtype_code(dtype), _coords_code(coords), _mode_code(mode), int(bool(backward)), 0, None, None
    offsets = _offsets(offsets, offsets.device)
    return (_dtype_code(dtype), _coords_code(coords), _mode_code(mode), int(bool(backward)), offsets.numel() - 1,
            _ptr(offsets), _stream(offsets.device))


def glv_autotune_key(offsets, dtype=torch.float64, coords="PtEtaPhiM", mode="plain", backward=False):
    """The autotuning cache key of a CSR dataset (``offsets`` on the GPU, or
    None for an empty dataset)."""
    buf = ctypes.create_string_buffer(512)
    dt, co, mo, bw, ne, po, st = _key_args(dtype, coords, mode, backward, offsets)
    check("glv_autotune_key", _lib.load().glv_autotune_key(dt, co, mo, bw, ne, po, buf, len(buf), st))
    return buf.value.decode()


def glv_autotune_lookup(offsets, dtype=torch.float64, coords="PtEtaPhiM", mode="plain", backward=False):
    """The tuned tiling of this dataset from this process's choices or the
    GLV_AUTOTUNE_CACHE file, without timing: (tiling, found); not found gives
    the default tiling (and a warning on stderr).  Either becomes the current
    choice."""
    t = glv_tiling()
    found = ctypes.c_int32(0)
    dt, co, mo, bw, ne, po, st = _key_args(dtype, coords, mode, backward, offsets)
    check("glv_autotune_lookup", _lib.load().glv_autotune_lookup(dt, co, mo, bw, ne, po, ctypes.byref(t),
                                                                 ctypes.byref(found), st))
    return _as_tuple(t), bool(found.value)


def glv_autotune_forget():
    """Forget this process's tuned choices (the cache file stays)."""
    _lib.load().glv_autotune_forget()


def glv_abi_version():
    return _lib.load().glv_abi_version()
