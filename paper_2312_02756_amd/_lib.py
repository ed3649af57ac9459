"""ctypes loader for libglv.so (the C ABI of include/glv.h).

torch is imported first so that the library's HIP runtime dependency binds to
the runtime torch already loaded (one runtime per process).  There is no
fallback: if the library is missing the import of this module fails.
"""

import ctypes
import os

import torch  # noqa: F401  (load order: torch's HIP runtime first)

from . import build as _build

GLV_OK = 0
STATUS_NAMES = {
    0: "GLV_OK", 1: "GLV_EINVAL_NULL", 2: "GLV_EINVAL_SIZE", 3: "GLV_EINVAL_DTYPE",
    4: "GLV_EINVAL_COORDS", 5: "GLV_EINVAL_MODE", 6: "GLV_EINVAL_ALIAS", 7: "GLV_EINVAL_STRIDE",
    8: "GLV_EINVAL_OFFSETS", 9: "GLV_EINVAL_TILING", 10: "GLV_EHIP",
}
GLV_F32, GLV_F64 = 1, 2
GLV_PXPYPZE, GLV_PTETAPHIM, GLV_PTETAPHIE, GLV_PXPYPZM = 0, 1, 2, 3
GLV_PLAIN, GLV_COMPENSATED = 0, 1

# Every symbol include/glv.h declares.
EXPORTS = (
    "glv_invariant_mass", "glv_invariant_mass_bwd", "glv_boost", "glv_boost_bwd", "glv_pair_offsets",
    "glv_event_reduce", "glv_event_reduce_bwd", "glv_event_reduce_bwd_totals", "glv_validate_offsets", "glv_autotune_event_reduce",
    "glv_current_tiling", "glv_autotune_event_reduce_bwd", "glv_current_tiling_bwd", "glv_status_str",
    "glv_abi_version", "glv_last_hip_error", "glv_convert", "glv_convert_bwd", "glv_lorentz_transform",
    "glv_lorentz_transform_bwd", "glv_rotate", "glv_rotate_bwd", "glv_rotate_axis_angle",
    "glv_rotate_axis_angle_bwd", "glv_mass_histogram", "glv_event_best_pair", "glv_invariant_mass_comp_bwd",
    "glv_autotune_key", "glv_autotune_lookup", "glv_autotune_forget", "glv_invariant_mass_histogram",
    "glv_event_reduce_best_pair",
)


class glv_tiling(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("events_per_tile", ctypes.c_int32),
                ("lds_particles", ctypes.c_int32), ("pairs_per_round", ctypes.c_int32)]


P4 = ctypes.c_void_p * 4
P3 = ctypes.c_void_p * 3
P9 = ctypes.c_void_p * 9
P16 = ctypes.c_void_p * 16
_vp = ctypes.c_void_p
_i = ctypes.c_int
_i64 = ctypes.c_int64

# Column-pointer arrays (P4 / P3 instances, or None for NULL) pass as void*.
_SIGS = {
    "glv_invariant_mass": [_i, _i, _i, _i64, _vp, _vp, _vp, _vp, _vp],
    "glv_invariant_mass_bwd": [_i, _i, _i64, _vp, _vp, _vp, _vp, _vp, _vp],
    "glv_invariant_mass_comp_bwd": [_i, _i64, _vp, _vp, _vp, _vp, _vp, _vp],
    "glv_boost": [_i, _i64, _vp, _vp, _i64, _vp, _vp],
    "glv_boost_bwd": [_i, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp],
    "glv_pair_offsets": [_i64, _vp, _vp, _vp],
    "glv_event_reduce": [_i, _i, _i, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "glv_event_reduce_bwd": [_i, _i, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "glv_event_reduce_bwd_totals": [_i, _i, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "glv_validate_offsets": [_i64, _vp, _i64, _vp, _vp],
    "glv_autotune_event_reduce": [_i, _i, _i, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "glv_current_tiling": [_i, _i, _i, _vp],
    "glv_autotune_event_reduce_bwd": [_i, _i, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "glv_convert": [_i, _i, _i, _i64, _vp, _vp, _vp],
    "glv_convert_bwd": [_i, _i, _i, _i64, _vp, _vp, _vp, _vp],
    "glv_lorentz_transform": [_i, _i64, _vp, _vp, _i64, _vp, _vp],
    "glv_lorentz_transform_bwd": [_i, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp],
    "glv_rotate": [_i, _i64, _vp, _vp, _i64, _vp, _vp],
    "glv_rotate_bwd": [_i, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp],
    "glv_rotate_axis_angle": [_i, _i64, _vp, _vp, _i64, _vp, _vp],
    "glv_rotate_axis_angle_bwd": [_i, _i64, _vp, _i64, _vp, _vp, _vp],
    "glv_mass_histogram": [_i, _i64, _vp, ctypes.c_double, ctypes.c_double, _i64, _vp, _vp],
    "glv_event_best_pair": [_i, _i64, _vp, _vp, ctypes.c_double, _vp, _vp, _vp],
    "glv_invariant_mass_histogram": [_i, _i, _i, _i64, _vp, _vp, ctypes.c_double, ctypes.c_double, _i64, _vp, _vp,
                                     _vp],
    "glv_event_reduce_best_pair": [_i, _i, _i, _i64, _vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp],
    "glv_current_tiling_bwd": [_i, _i, _vp],
    "glv_autotune_key": [_i, _i, _i, ctypes.c_int32, _i64, _vp, ctypes.c_char_p, _i64, _vp],
    "glv_autotune_lookup": [_i, _i, _i, ctypes.c_int32, _i64, _vp, _vp, _vp, _vp],
    "glv_autotune_forget": [],
    "glv_status_str": [_i],
    "glv_abi_version": [],
    "glv_last_hip_error": [],
}

_lib = None


def library_path() -> str:
    return _build.library_path()


def load():
    """Load libglv.so (built by paper_2312_02756_amd.build)."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2312_02756_amd.build` "
                               "(or __graft_entry__.build()); there is no fallback path")
        lib = ctypes.CDLL(path)
        for name, args in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.glv_status_str.restype = ctypes.c_char_p
        lib.glv_autotune_forget.restype = None
        _lib = lib
    return _lib


class GlvError(RuntimeError):
    def __init__(self, fn, code):
        lib = load()
        msg = lib.glv_status_str(code).decode()
        extra = f" (hip error {lib.glv_last_hip_error()})" if code == 10 else ""
        super().__init__(f"{fn}: {STATUS_NAMES.get(code, code)}: {msg}{extra}")
        self.code = code


def check(fn, code):
    if code != GLV_OK:
        raise GlvError(fn, code)
