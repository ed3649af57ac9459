"""The C ABI on the host (no GPU needed): the library loads, exports every
symbol include/glv.h declares, and rejects invalid arguments with the
documented status before any kernel could be launched.  Pointers here are
fake addresses; no call below reaches a launch."""

import ctypes
import os
import re

import pytest

from paper_2312_02756_amd import _lib, build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "glv.h")

OK, NULL, SIZE, DTYPE, COORDS, MODE, ALIAS, STRIDE, OFFSETS, TILING = range(10)
GiB = 1 << 30


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(build.library_path()):
        build.build()
    return _lib.load()


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(glv_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_strings(lib):
    assert lib.glv_abi_version() == 2
    for code in range(11):
        assert lib.glv_status_str(code)
    assert lib.glv_status_str(0) == b"ok"


def cols(base, k=4):
    arr = _lib.P4 if k == 4 else _lib.P3
    return arr(*[base + i * GiB for i in range(k)])


A, B, M = 16 * GiB, 32 * GiB, 48 * GiB
N = 1000


def test_mass_validation(lib):
    f = lib.glv_invariant_mass
    assert f(7, 1, 0, N, cols(A), cols(B), M, None, None) == DTYPE
    assert f(2, 9, 0, N, cols(A), cols(B), M, None, None) == COORDS
    assert f(2, 0, 1, N, cols(A), cols(B), M, None, None) == MODE   # compensated needs PtEtaPhiM
    assert f(2, 2, 1, N, cols(A), cols(B), M, None, None) == MODE
    assert f(2, 1, 5, N, cols(A), cols(B), M, None, None) == MODE
    assert f(2, 1, 0, -1, cols(A), cols(B), M, None, None) == SIZE
    bad = cols(A)
    bad[2] = None
    assert f(2, 1, 0, N, bad, cols(B), M, None, None) == NULL
    assert f(2, 1, 0, N, cols(A), cols(B), None, None, None) == NULL
    assert f(2, 1, 0, N, cols(A), cols(B), A + 8 * (N - 1), None, None) == ALIAS  # m overlaps a[0]
    assert f(2, 1, 0, 0, cols(A), cols(B), M, None, None) == OK                    # empty: nothing to do


def test_mass_bwd_validation(lib):
    f = lib.glv_invariant_mass_bwd
    G = 64 * GiB
    assert f(2, 1, -3, cols(A), cols(B), M, cols(G), cols(G + 8 * GiB), None) == SIZE
    assert f(2, 1, N, cols(A), cols(B), None, cols(G), cols(G + 8 * GiB), None) == NULL
    assert f(2, 1, N, cols(A), cols(B), M, cols(G), cols(G), None) == ALIAS          # grad_a = grad_b
    assert f(2, 1, N, cols(A), cols(B), M, cols(A), cols(G), None) == ALIAS          # grad over input
    assert f(2, 1, 0, cols(A), cols(B), M, cols(G), cols(G + 8 * GiB), None) == OK


def test_boost_validation(lib):
    f = lib.glv_boost
    X, BETA, Y = A, B, 80 * GiB
    assert f(2, N, cols(X), cols(BETA, 3), 2, cols(Y), None) == STRIDE
    assert f(2, N, cols(X), cols(BETA, 3), -1, cols(Y), None) == STRIDE
    y = cols(X)
    y[0], y[1] = y[1], y[0]
    assert f(2, N, cols(X), cols(BETA, 3), 1, y, None) == ALIAS                      # permuted in place
    assert f(2, N, cols(X), cols(X, 3), 1, cols(X), None) == ALIAS                   # beta inside y
    assert f(2, 0, cols(X), cols(BETA, 3), 1, cols(X), None) == OK                   # in place, empty
    g = lib.glv_boost_bwd
    assert g(2, N, cols(X), cols(BETA, 3), 0, cols(Y), cols(Y + 8 * GiB), cols(Y + 16 * GiB, 3), None) == STRIDE
    assert g(2, N, None, cols(BETA, 3), 1, cols(Y), cols(Y + 8 * GiB), cols(Y + 16 * GiB, 3), None) == NULL
    assert g(2, 0, None, cols(BETA, 3), 0, cols(Y), cols(Y + 8 * GiB), None, None) == OK


def test_convert_validation(lib):
    f = lib.glv_convert
    Y = 80 * GiB
    assert f(7, 0, 1, N, cols(A), cols(Y), None) == DTYPE
    assert f(2, 4, 1, N, cols(A), cols(Y), None) == COORDS
    assert f(2, 0, -1, N, cols(A), cols(Y), None) == COORDS
    assert f(2, 0, 1, -1, cols(A), cols(Y), None) == SIZE
    bad = cols(Y)
    bad[3] = None
    assert f(2, 0, 1, N, cols(A), bad, None) == NULL
    assert f(2, 0, 1, 0, None, None, None) == OK                                    # empty: nothing to do
    y = cols(A)
    y[0], y[1] = y[1], y[0]
    assert f(1, 1, 0, N, cols(A), y, None) == ALIAS                                  # permuted in place
    part = cols(Y)
    part[2] = A + 2 * GiB
    assert f(1, 1, 0, N, cols(A), part, None) == ALIAS                               # one column in place
    assert f(2, 1, 0, N, cols(A), cols(A + 4 * (N - 1)), None) == ALIAS              # shifted overlap
    g = lib.glv_convert_bwd
    G = 64 * GiB
    assert g(2, 1, 0, N, cols(A), cols(G), cols(A), None) == ALIAS                   # grad_in over the vectors
    assert g(2, 1, 0, N, cols(A), cols(G), cols(G + 8), None) == ALIAS               # shifted over grad_out
    assert g(2, 1, 0, N, cols(A), None, cols(Y), None) == NULL
    assert g(2, 1, 9, N, cols(A), cols(G), cols(Y), None) == COORDS


def test_transform_validation(lib):
    X, L, Y, G = A, 40 * GiB, 80 * GiB, 100 * GiB
    P16, P9 = _lib.P16, _lib.P9

    def mat(base, k):
        return (P16 if k == 16 else (P9 if k == 9 else _lib.P4))(*[base + i * GiB for i in range(k)])

    f = lib.glv_lorentz_transform
    assert f(7, N, cols(X), mat(L, 16), 1, cols(Y), None) == DTYPE
    assert f(2, -1, cols(X), mat(L, 16), 1, cols(Y), None) == SIZE
    assert f(2, N, cols(X), mat(L, 16), 2, cols(Y), None) == STRIDE
    assert f(2, 0, None, None, 0, None, None) == OK                                   # empty
    m = mat(L, 16)
    m[11] = None
    assert f(2, N, cols(X), m, 1, cols(Y), None) == NULL
    assert f(2, N, cols(X), mat(L, 16), 1, None, None) == NULL
    assert f(2, N, cols(X), mat(L, 16), 1, cols(L + 3 * GiB), None) == ALIAS         # y over the matrix
    assert f(2, N, cols(X), mat(L, 16), 0, cols(L + 15 * GiB - 4 * 8), None) == ALIAS  # over a broadcast entry
    y = cols(X)
    y[2], y[3] = y[3], y[2]
    assert f(1, N, cols(X), mat(L, 16), 1, y, None) == ALIAS                        # permuted in place
    g = lib.glv_lorentz_transform_bwd
    assert g(2, N, cols(X), mat(L, 16), 0, cols(G), cols(Y), mat(Y + 8 * GiB, 16), None) == STRIDE  # grad_L: per item
    assert g(2, N, None, mat(L, 16), 1, cols(G), cols(Y), mat(Y + 8 * GiB, 16), None) == NULL      # grad_L needs x
    assert g(2, N, cols(X), mat(L, 16), 1, cols(G), cols(G), None, None) == ALIAS                 # grad_x over grad_y
    assert g(2, N, cols(X), mat(L, 16), 1, cols(G), cols(Y), mat(X, 16), None) == ALIAS           # grad_L over x
    r = lib.glv_rotate
    assert r(2, N, cols(X), mat(L, 9), 3, cols(Y), None) == STRIDE
    assert r(2, N, cols(X), None, 1, cols(Y), None) == NULL
    assert r(2, N, cols(X), mat(L, 9), 1, cols(L + 8 * GiB), None) == ALIAS
    rb = lib.glv_rotate_bwd
    assert rb(2, N, cols(X), mat(L, 9), 0, cols(G), cols(Y), mat(Y + 8 * GiB, 9), None) == STRIDE
    assert rb(9, N, cols(X), mat(L, 9), 1, cols(G), cols(Y), None, None) == DTYPE
    a = lib.glv_rotate_axis_angle
    assert a(2, N, cols(X), mat(L, 4), -1, cols(Y), None) == STRIDE
    assert a(2, N, cols(X), mat(L, 4), 1, cols(L), None) == ALIAS
    ab = lib.glv_rotate_axis_angle_bwd
    assert ab(2, N, mat(L, 4), 1, cols(G), cols(L + 2 * GiB), None) == ALIAS             # grad_x over the angles
    assert ab(2, N, mat(L, 4), 1, None, cols(Y), None) == NULL
    assert ab(2, 0, None, 0, None, None, None) == OK


def test_analysis_validation(lib):
    C, R, BM = 40 * GiB, 60 * GiB, 70 * GiB
    h = lib.glv_mass_histogram
    assert h(7, N, A, 0.0, 1.0, 10, C, None) == DTYPE
    assert h(2, -1, A, 0.0, 1.0, 10, C, None) == SIZE
    assert h(2, N, A, 0.0, 1.0, 0, C, None) == SIZE                       # no bins
    assert h(2, N, A, 1.0, 1.0, 10, C, None) == SIZE                      # empty range
    assert h(2, N, A, 2.0, 1.0, 10, C, None) == SIZE                      # reversed
    assert h(2, N, A, float("nan"), 1.0, 10, C, None) == SIZE
    assert h(2, N, A, -1e308, 1e308, 10, C, None) == SIZE                 # hi - lo overflows
    assert h(2, N, A, 0.0, 1e-320, 1 << 40, C, None) == SIZE              # n_bins / (hi - lo) overflows
    assert h(2, N, None, 0.0, 1.0, 10, C, None) == NULL
    assert h(2, N, A, 0.0, 1.0, 10, None, None) == NULL
    assert h(2, N, A, 0.0, 1.0, 10, A + 8 * (N - 1), None) == ALIAS         # counts over the masses
    assert h(2, 0, None, 0.0, 1.0, 10, None, None) == OK                    # empty
    b = lib.glv_event_best_pair
    assert b(5, N, B, M, 91.0, R, BM, None) == DTYPE
    assert b(2, -2, B, M, 91.0, R, BM, None) == SIZE
    assert b(2, N, None, M, 91.0, R, BM, None) == NULL
    assert b(2, N, B, M, 91.0, R, None, None) == NULL
    assert b(2, N, B, M, 91.0, R, R + 8, None) == ALIAS                    # the two outputs overlap
    assert b(2, N, B, M, 91.0, B + 8 * N, BM, None) == ALIAS               # rank over the offsets' last entry
    assert b(2, 0, None, None, 91.0, None, None, None) == OK


def test_fused_analysis_validation(lib):
    """The fused entry points reject what their unfused halves reject."""
    C, R, BM = 40 * GiB, 60 * GiB, 70 * GiB
    h = lib.glv_invariant_mass_histogram
    a, b = cols(A), cols(B)
    assert h(7, 1, 0, N, a, b, 0.0, 1.0, 10, C, None, None) == DTYPE
    assert h(2, 9, 0, N, a, b, 0.0, 1.0, 10, C, None, None) == COORDS
    assert h(2, 0, 1, N, a, b, 0.0, 1.0, 10, C, None, None) == MODE        # compensated needs PtEtaPhiM
    assert h(2, 1, 0, -1, a, b, 0.0, 1.0, 10, C, None, None) == SIZE
    assert h(2, 1, 0, N, a, b, 0.0, 1.0, 0, C, None, None) == SIZE          # no bins
    assert h(2, 1, 0, N, a, b, 1.0, 0.0, 10, C, None, None) == SIZE         # reversed range
    assert h(2, 1, 0, N, a, b, 0.0, float("inf"), 10, C, None, None) == SIZE
    assert h(2, 1, 0, N, None, b, 0.0, 1.0, 10, C, None, None) == NULL
    assert h(2, 1, 0, N, a, b, 0.0, 1.0, 10, None, None, None) == NULL
    assert h(2, 1, 0, N, a, b, 0.0, 1.0, 10, B + 8 * (N - 1), None, None) == ALIAS  # counts over leg b's column 0
    assert h(2, 1, 1, N, a, b, 0.0, 1.0, 10, C, A, None) == ALIAS          # fallback counter over a leg
    assert h(2, 1, 1, N, a, b, 0.0, 1.0, 10, C, C + 16, None) == ALIAS     # fallback counter inside counts
    assert h(2, 1, 0, 0, None, None, 0.0, 1.0, 10, None, None, None) == OK  # empty
    OFF, PO, P = 80 * GiB, 90 * GiB, 100 * GiB
    f = lib.glv_event_reduce_best_pair
    assert f(7, 1, 0, 10, OFF, PO, cols(P), 91.0, R, BM, None, None, None) == DTYPE
    assert f(2, 0, 1, 10, OFF, PO, cols(P), 91.0, R, BM, None, None, None) == MODE
    assert f(2, 1, 0, -3, OFF, PO, cols(P), 91.0, R, BM, None, None, None) == SIZE
    assert f(2, 1, 0, 10, None, PO, cols(P), 91.0, R, BM, None, None, None) == OFFSETS
    assert f(2, 1, 0, 10, OFF, None, cols(P), 91.0, R, BM, None, None, None) == OFFSETS   # pair offsets required
    assert f(2, 1, 0, 10, OFF, PO, None, 91.0, R, BM, None, None, None) == NULL
    assert f(2, 1, 0, 10, OFF, PO, cols(P), 91.0, None, BM, None, None, None) == NULL
    assert f(2, 1, 0, 10, OFF, PO, cols(P), 91.0, R, R + 8, None, None, None) == ALIAS    # outputs overlap
    assert f(2, 1, 0, 10, OFF, PO, cols(P), 91.0, PO + 8, BM, None, None, None) == ALIAS  # rank over pair offsets
    assert f(2, 1, 0, 10, OFF, PO, cols(P), 91.0, R, P, None, None, None) == ALIAS        # mass over a column
    assert f(2, 1, 1, 10, OFF, PO, cols(P), 91.0, R, BM, R + 8, None, None) == ALIAS      # counter inside rank
    for bad in ((100, 0, 0, 0), (256, 65, 128, 512), (256, 32, 128, 100), (512, 64, 4096, 4096)):
        t = _lib.glv_tiling(*bad)
        assert f(2, 1, 0, 10, OFF, PO, cols(P), 91.0, R, BM, None, ctypes.byref(t), None) == TILING, bad
    assert f(2, 1, 0, 0, None, None, None, 91.0, None, None, None, None, None) == OK


def test_jagged_validation(lib):
    OFF, PO, P, T, EM, PM = A, B, 100 * GiB, 140 * GiB, 180 * GiB, 190 * GiB
    f = lib.glv_event_reduce
    assert f(2, 1, 0, 10, None, PO, cols(P), cols(T), EM, PM, None, None, None) == OFFSETS
    assert f(2, 1, 0, 10, OFF, None, cols(P), cols(T), EM, PM, None, None, None) == OFFSETS  # pairs need po
    assert f(2, 1, 1, 10, OFF, None, cols(P), None, EM, None, None, None, None) == OFFSETS   # comp event mass
    assert f(2, 0, 1, 10, OFF, PO, cols(P), cols(T), EM, PM, None, None, None) == MODE
    assert f(2, 1, 0, -2, OFF, PO, cols(P), cols(T), EM, PM, None, None, None) == SIZE
    assert f(2, 1, 0, 10, OFF, PO, cols(P), cols(T), OFF, PM, None, None, None) == ALIAS    # event_m over offsets
    for bad in ((100, 0, 0, 0), (256, 512, 0, 0), (256, 128, 32, 0), (256, 128, 8192, 0), (256, 128, 1024, 1),
                (1024, 16, 256, 0), (512, 512, 4096, 0), (256, 65, 128, 512), (256, 32, 128, 100),
                (256, 32, 128, 8192), (256, 32, 128, 32), (256, 32, 4096, 512), (512, 32, 1024, 1024)):
        t = _lib.glv_tiling(*bad)
        assert f(2, 1, 0, 10, OFF, PO, cols(P), cols(T), EM, PM, None, ctypes.byref(t), None) == TILING, bad
    g = lib.glv_pair_offsets
    assert g(-1, OFF, PO, None) == SIZE
    assert g(10, None, PO, None) == NULL
    assert g(10, OFF, OFF + 8, None) == ALIAS
    h = lib.glv_event_reduce_bwd
    assert h(2, 1, 10, OFF, None, cols(P), None, None, PM, cols(T), None, None) == OFFSETS
    for bad in ((128, 16, 128, 100), (128, 65, 128, 512), (128, 16, 32, 512), (512, 64, 512, 4160)):
        t = _lib.glv_tiling(*bad)
        assert h(2, 1, 10, OFF, PO, cols(P), None, None, PM, cols(T), ctypes.byref(t), None) == TILING, bad
    assert h(2, 1, 10, OFF, PO, cols(P), None, None, None, cols(P), None, None) == ALIAS
    # the reverse mode given the forward's totals: 4 columns required, not over grad_p
    b = lib.glv_event_reduce_bwd_totals
    G = 200 * GiB
    assert b(2, 1, 10, OFF, PO, cols(P), None, None, EM, None, cols(G), None, None) == NULL
    assert b(2, 1, 10, OFF, PO, cols(P), _lib.P4(T, T + GiB, T + 2 * GiB, None), None, EM, None, cols(G), None,
             None) == NULL
    assert b(2, 1, 10, OFF, PO, cols(P), cols(G), None, EM, None, cols(G), None, None) == ALIAS
    assert b(2, 1, 10, OFF, None, cols(P), cols(T), None, EM, PM, cols(G), None, None) == OFFSETS
    assert b(2, 1, 10, OFF, PO, cols(P), cols(T), None, EM, None, cols(P), None, None) == ALIAS
    v = lib.glv_validate_offsets
    assert v(10, OFF, -1, EM, None) == SIZE
    assert v(10, OFF, 5, None, None) == NULL


def test_current_tiling_default(lib):
    t = _lib.glv_tiling()
    assert lib.glv_current_tiling(2, 1, 0, ctypes.byref(t)) == OK
    assert t.block in (64, 128, 256, 512) and 1 <= t.events_per_tile <= t.block
    assert 64 <= t.lds_particles <= 4096
    assert lib.glv_current_tiling(2, 0, 1, ctypes.byref(t)) == MODE


def test_default_tilings_valid_for_every_combination(lib):
    """The default tiling of every dtype, coordinate system and mode passes
    the library's own validation (the FP64 compensated wavefront stages the
    most LDS)."""
    t = _lib.glv_tiling()
    for dt in (1, 2):
        for co in (0, 1, 2, 3):
            assert lib.glv_current_tiling(dt, co, 0, ctypes.byref(t)) == OK, (dt, co)
            assert lib.glv_current_tiling_bwd(dt, co, ctypes.byref(t)) == OK, (dt, co)
        assert lib.glv_current_tiling(dt, 1, 1, ctypes.byref(t)) == OK, (dt, "compensated")


def test_current_tiling_bwd_default_and_autotune_validation(lib):
    t = _lib.glv_tiling()
    assert lib.glv_current_tiling_bwd(2, 1, ctypes.byref(t)) == OK
    assert (t.block, t.events_per_tile, t.lds_particles, t.pairs_per_round) == (128, 64, 128, 512)
    assert lib.glv_current_tiling_bwd(3, 1, ctypes.byref(t)) == DTYPE
    assert lib.glv_current_tiling_bwd(2, 1, None) == NULL
    # host-side validation, before any device work: missing gradient outputs
    P4 = _lib.P4
    cols = P4(*[0x1000 * (k + 1) for k in range(4)])
    assert lib.glv_autotune_event_reduce_bwd(2, 1, 10, 0x100, None, cols, None, None, None, None, None,
                                             None) == NULL


@pytest.mark.parametrize("lang", ["c", "c++"])
def test_header_compiles_standalone(lang, tmp_path):
    """include/glv.h is a plain C header: it compiles on its own as C and as
    C++ with warnings as errors (no torch or HIP types needed)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc" if lang == "c" else "g++")
    if gcc is None:
        pytest.skip("no host compiler")
    header = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "glv.h")
    src = tmp_path / ("use." + ("c" if lang == "c" else "cpp"))
    src.write_text('#include "glv.h"\nint probe(void) { return (int)GLV_OK + (int)sizeof(glv_tiling); }\n')
    r = subprocess.run([gcc, "-fsyntax-only", "-Wall", "-Wextra", "-Werror", "-I", os.path.dirname(header),
                        str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
