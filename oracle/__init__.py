"""CPU oracle for the batched Lorentz-vector path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The GPU library never does, and
this package imports nothing from it.

Thin ctypes wrapper around ``liborc.so`` (built from ``glv_oracle.c`` by
``oracle/build.py``).  Inputs are numpy arrays; FP32 inputs are widened to
float64 first (exactly), so every result is the exact-input result computed
in binary64 (or binary128 for the ``*_q`` functions).

Coordinate codes: 0 = PxPyPzE, 1 = PtEtaPhiM, 2 = PtEtaPhiE, 3 = PxPyPzM.
"""

import ctypes
import os

import numpy as np

from . import build as _build

PXPYPZE, PTETAPHIM, PTETAPHIE, PXPYPZM = 0, 1, 2, 3
PLAIN, ACCURATE = 0, 1
COORDS = {"PxPyPzE": PXPYPZE, "PtEtaPhiM": PTETAPHIM, "PtEtaPhiE": PTETAPHIE, "PxPyPzM": PXPYPZM}

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.library_path()
        if not os.path.exists(path):
            _build.build()
        _lib = ctypes.CDLL(path)
        _lib.orc_get_threads.restype = ctypes.c_int
    return _lib


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _p(x):
    return x.ctypes.data_as(ctypes.c_void_p) if x is not None else None


def _coords(c):
    return COORDS[c] if isinstance(c, str) else int(c)


def set_threads(k: int) -> None:
    _load().orc_set_threads(ctypes.c_int(int(k)))


def get_threads() -> int:
    return int(_load().orc_get_threads())


def to_cartesian(coords, cols):
    c = [_f64(x) for x in cols]
    n = c[0].size
    out = [np.empty(n) for _ in range(4)]
    _load().orc_to_cartesian(ctypes.c_int(_coords(coords)), ctypes.c_int64(n), *map(_p, c), *map(_p, out))
    return tuple(out)


def convert(src, dst, cols):
    """Coordinates in system ``dst`` of vectors given in ``src`` (through the
    Cartesian components; src == dst copies)."""
    c = [_f64(x) for x in cols]
    n = c[0].size
    out = [np.empty(n) for _ in range(4)]
    _load().orc_convert(ctypes.c_int(_coords(src)), ctypes.c_int(_coords(dst)), ctypes.c_int64(n), *map(_p, c),
                        *map(_p, out))
    return tuple(out)


def convert_vjp(src, dst, cols, g):
    """(d convert / d cols)^T g for upstream gradients ``g`` of the 4 outputs."""
    c = [_f64(x) for x in cols]
    gg = [_f64(x) for x in g]
    n = c[0].size
    out = [np.empty(n) for _ in range(4)]
    _load().orc_convert_vjp(ctypes.c_int(_coords(src)), ctypes.c_int(_coords(dst)), ctypes.c_int64(n),
                            *map(_p, c), *map(_p, gg), *map(_p, out))
    return tuple(out)


def mass_plain(coords, a, b, scale=False):
    """Pair mass by the definition (binary64); optionally S = E^2 + |P|^2."""
    a = [_f64(x) for x in a]
    b = [_f64(x) for x in b]
    n = a[0].size
    m = np.empty(n)
    s = np.empty(n) if scale else None
    _load().orc_mass_plain(ctypes.c_int(_coords(coords)), ctypes.c_int64(n), *map(_p, a), *map(_p, b), _p(m), _p(s))
    return (m, s) if scale else m


def mass_plain_q(coords, a, b, lo=False):
    """Pair mass by the definition in binary128, rounded to binary64.
    With ``lo=True`` also the rounding remainder (m + lo ~ 106 bits)."""
    a = [_f64(x) for x in a]
    b = [_f64(x) for x in b]
    n = a[0].size
    m = np.empty(n)
    ml = np.empty(n) if lo else None
    _load().orc_mass_plain_q(ctypes.c_int(_coords(coords)), ctypes.c_int64(n), *map(_p, a), *map(_p, b), _p(m),
                             _p(ml))
    return (m, ml) if lo else m


def mass_accurate(a, b):
    """Pair mass of PtEtaPhiM legs by the cancellation-free form (binary64)."""
    a = [_f64(x) for x in a]
    b = [_f64(x) for x in b]
    n = a[0].size
    m = np.empty(n)
    _load().orc_mass_accurate(ctypes.c_int64(n), *map(_p, a), *map(_p, b), _p(m))
    return m


def _boost_call(fn, x, beta, beta_stride, extra=()):
    x = [_f64(v) for v in x]
    beta = [_f64(v) for v in beta]
    n = x[0].size
    if beta_stride == 1:
        assert beta[0].size == n
    out = [np.empty(n) for _ in range(4)]
    fn(ctypes.c_int64(n), *map(_p, x), *map(_p, beta), ctypes.c_int64(beta_stride), *map(_p, out), *extra)
    return tuple(out)


def boost(x, beta, beta_stride=1):
    return _boost_call(_load().orc_boost, x, beta, beta_stride)


def boost_q(x, beta, beta_stride=1, lo=False):
    """Boost in binary128; with ``lo=True`` also the rounding remainders."""
    if not lo:
        return _boost_call(_load().orc_boost_q, x, beta, beta_stride, (None,))
    n = np.asarray(x[0]).size
    rem = [np.empty(n) for _ in range(4)]
    arr = (ctypes.c_void_p * 4)(*[r.ctypes.data for r in rem])
    y = _boost_call(_load().orc_boost_q, x, beta, beta_stride, (arr,))
    return y, tuple(rem)


def boost_scale(x, beta, beta_stride=1):
    return _boost_call(_load().orc_boost_scale, x, beta, beta_stride)


def mass_vjp(coords, a, b, gm):
    a = [_f64(x) for x in a]
    b = [_f64(x) for x in b]
    gm = _f64(gm)
    n = a[0].size
    ga = [np.empty(n) for _ in range(4)]
    gb = [np.empty(n) for _ in range(4)]
    _load().orc_mass_vjp(ctypes.c_int(_coords(coords)), ctypes.c_int64(n), *map(_p, a), *map(_p, b), _p(gm),
                         *map(_p, ga), *map(_p, gb))
    return tuple(ga), tuple(gb)


def mass_vjp_scale(coords, a, b, gm):
    """Absolute-value evaluation of the mass VJP's chain rule (rounding scale
    of each gradient component)."""
    a = [_f64(x) for x in a]
    b = [_f64(x) for x in b]
    gm = _f64(gm)
    n = a[0].size
    ga = [np.empty(n) for _ in range(4)]
    gb = [np.empty(n) for _ in range(4)]
    _load().orc_mass_vjp_scale(ctypes.c_int(_coords(coords)), ctypes.c_int64(n), *map(_p, a), *map(_p, b),
                               _p(gm), *map(_p, ga), *map(_p, gb))
    return tuple(ga), tuple(gb)


def boost_vjp(x, beta, gy):
    x = [_f64(v) for v in x]
    beta = [_f64(v) for v in beta]
    gy = [_f64(v) for v in gy]
    n = x[0].size
    gx = [np.empty(n) for _ in range(4)]
    gbeta = [np.empty(n) for _ in range(3)]
    _load().orc_boost_vjp(ctypes.c_int64(n), *map(_p, x), *map(_p, beta), *map(_p, gy), *map(_p, gx),
                          *map(_p, gbeta))
    return tuple(gx), tuple(gbeta)


def _i64(x):
    return np.ascontiguousarray(x, dtype=np.int64)


def pair_offsets(offsets):
    offsets = _i64(offsets)
    ne = offsets.size - 1
    po = np.empty(ne + 1, dtype=np.int64)
    _load().orc_pair_offsets(ctypes.c_int64(ne), _p(offsets), _p(po))
    return po


def event_reduce(coords, offsets, p, mode=PLAIN):
    """Returns (total (4 arrays), event_m, pair_m, pair_offsets)."""
    offsets = _i64(offsets)
    p = [_f64(x) for x in p]
    ne = offsets.size - 1
    po = pair_offsets(offsets)
    tot = [np.empty(ne) for _ in range(4)]
    em = np.empty(ne)
    pm = np.empty(int(po[-1]))
    _load().orc_event_reduce(ctypes.c_int(_coords(coords)), ctypes.c_int(int(mode)), ctypes.c_int64(ne),
                             _p(offsets), _p(po), *map(_p, p), *map(_p, tot), _p(em), _p(pm))
    return tuple(tot), em, pm, po


def event_reduce_q(coords, offsets, p):
    """Totals and event masses of the plain definition in binary128."""
    offsets = _i64(offsets)
    p = [_f64(x) for x in p]
    ne = offsets.size - 1
    tot = [np.empty(ne) for _ in range(4)]
    em = np.empty(ne)
    _load().orc_event_reduce_q(ctypes.c_int(_coords(coords)), ctypes.c_int64(ne), _p(offsets), *map(_p, p),
                               *map(_p, tot), _p(em))
    return tuple(tot), em


def event_reduce_vjp(coords, offsets, p, g_total=None, g_em=None, g_pair=None):
    offsets = _i64(offsets)
    p = [_f64(x) for x in p]
    ne = offsets.size - 1
    po = pair_offsets(offsets)
    gt = [None] * 4 if g_total is None else [_f64(x) for x in g_total]
    gem = None if g_em is None else _f64(g_em)
    gpr = None if g_pair is None else _f64(g_pair)
    n = p[0].size
    gp = [np.empty(n) for _ in range(4)]
    _load().orc_event_reduce_vjp(ctypes.c_int(_coords(coords)), ctypes.c_int64(ne), _p(offsets), _p(po),
                                 *map(_p, p), *map(_p, gt), _p(gem), _p(gpr), *map(_p, gp))
    return tuple(gp)


# ------------------------------------------------- general transformations

def _ptrs(cols):
    arr = (ctypes.c_void_p * len(cols))(*[c.ctypes.data for c in cols])
    return arr


def _transform(fn, x, mats, stride, n_out=4):
    x = [_f64(c) for c in x]
    mats = [_f64(c) for c in mats]
    n = x[0].size
    y = [np.empty(n) for _ in range(n_out)]
    fn(ctypes.c_int64(n), _ptrs(x), _ptrs(mats), ctypes.c_int64(int(stride)), _ptrs(y))
    return tuple(y)


def lorentz_transform(x, m, stride=1):
    """y = L x per item; ``m`` = 16 row-major columns (stride 1) or 16 scalars /
    one-element arrays (stride 0)."""
    return _transform(_load().orc_lorentz_transform, x, m, stride)


def lorentz_transform_vjp(x, m, gy, stride=1, want_gm=True):
    x, m, gy = [_f64(c) for c in x], [_f64(c) for c in m], [_f64(c) for c in gy]
    n = x[0].size
    gx = [np.empty(n) for _ in range(4)]
    gm = [np.empty(n) for _ in range(16)] if want_gm else None
    _load().orc_lorentz_transform_vjp(ctypes.c_int64(n), _ptrs(x), _ptrs(m), ctypes.c_int64(int(stride)),
                                      _ptrs(gy), _ptrs(gx), _ptrs(gm) if gm else None)
    return tuple(gx), (tuple(gm) if gm else None)


def rotate(x, r, stride=1):
    """Rotation3D: 9 row-major columns (or scalars with stride 0) applied to
    (px, py, pz); E passes through."""
    return _transform(_load().orc_rotate, x, r, stride)


def rotate_vjp(x, r, gy, stride=1, want_gr=True):
    x, r, gy = [_f64(c) for c in x], [_f64(c) for c in r], [_f64(c) for c in gy]
    n = x[0].size
    gx = [np.empty(n) for _ in range(4)]
    gr = [np.empty(n) for _ in range(9)] if want_gr else None
    _load().orc_rotate_vjp(ctypes.c_int64(n), _ptrs(x), _ptrs(r), ctypes.c_int64(int(stride)), _ptrs(gy),
                           _ptrs(gx), _ptrs(gr) if gr else None)
    return tuple(gx), (tuple(gr) if gr else None)


def rotate_axis_angle(x, aa, stride=1):
    """AxisAngle: aa = (ax, ay, az, angle) columns (or scalars with stride 0)."""
    return _transform(_load().orc_rotate_axis_angle, x, aa, stride)


def rotate_axis_angle_vjp(aa, gy, stride=1):
    aa, gy = [_f64(c) for c in aa], [_f64(c) for c in gy]
    n = gy[0].size
    gx = [np.empty(n) for _ in range(4)]
    _load().orc_rotate_axis_angle_vjp(ctypes.c_int64(n), _ptrs(aa), ctypes.c_int64(int(stride)), _ptrs(gy),
                                      _ptrs(gx))
    return tuple(gx)


# ------------------------------------------------------------ analysis step

def histogram(v, lo, hi, n_bins):
    """Counts of n_bins equal bins of [lo, hi) with an underflow bin first and
    an overflow bin last (n_bins + 2 uint64)."""
    v = _f64(v)
    counts = np.zeros(int(n_bins) + 2, dtype=np.uint64)
    _load().orc_histogram(ctypes.c_int64(v.size), _p(v), ctypes.c_double(lo), ctypes.c_double(hi),
                          ctypes.c_int64(int(n_bins)), _p(counts))
    return counts


def best_pair(pair_offsets, pm, target):
    """(rank, mass) per event of its pair closest to ``target``."""
    po = np.ascontiguousarray(pair_offsets, dtype=np.int64)
    pm = _f64(pm)
    ne = po.size - 1
    rank = np.empty(ne, dtype=np.int64)
    bm = np.empty(ne)
    _load().orc_best_pair(ctypes.c_int64(ne), _p(po), _p(pm), ctypes.c_double(target), _p(rank), _p(bm))
    return rank, bm


def mass_vjp_q(a, b, gm):
    """Pair-mass VJP of PtEtaPhiM legs by the chain rule in binary128."""
    a, b = [_f64(c) for c in a], [_f64(c) for c in b]
    gm = _f64(gm)
    n = a[0].size
    ga = [np.empty(n) for _ in range(4)]
    gb = [np.empty(n) for _ in range(4)]
    _load().orc_mass_vjp_q(ctypes.c_int64(n), _ptrs(a), _ptrs(b), _p(gm), _ptrs(ga), _ptrs(gb))
    return tuple(ga), tuple(gb)
