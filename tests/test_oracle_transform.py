"""Pins of the oracle's general transformations (Sec. 3.1: Lorentz
transformations and rotations, each a matrix or an axis and angle; Sec. 4.1:
ApplyBoost applies a 4x4 Lorentz matrix): LorentzRotation (4x4), Rotation3D
(3x3) and AxisAngle applied to batches of 4-vectors, and their reverse
modes.  CPU only."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth

U = 2.0 ** -53


def _vectors(n, seed):
    x, _ = synth.boost_items(synth.rng(seed), n)
    return x


def _cols(mats):
    """(n, r, c) matrices -> r*c row-major columns."""
    n, r, c = mats.shape
    return [np.ascontiguousarray(mats[:, a, b]) for a in range(r) for b in range(c)]


def _boost_matrix(beta):
    """The textbook 4x4 boost in (px, py, pz, E) order, per item."""
    b = np.stack(beta, axis=1)
    b2 = np.sum(b * b, axis=1)
    g = 1.0 / np.sqrt(1.0 - b2)
    k = g * g / (1.0 + g)
    n = b.shape[0]
    m = np.zeros((n, 4, 4))
    m[:, :3, :3] = np.eye(3) + k[:, None, None] * b[:, :, None] * b[:, None, :]
    m[:, :3, 3] = g[:, None] * b
    m[:, 3, :3] = g[:, None] * b
    m[:, 3, 3] = g
    return m


def _random_lorentz(n, seed):
    """Proper orthochronous transformations: rotation, boost, rotation."""
    g = synth.rng(seed)
    r1 = Rotation.random(n, random_state=int(g.integers(1 << 30))).as_matrix()
    r2 = Rotation.random(n, random_state=int(g.integers(1 << 30))).as_matrix()
    beta = tuple(0.5 * c for c in synth.boost_items(g, n)[1])
    e1, e2 = np.zeros((n, 4, 4)), np.zeros((n, 4, 4))
    e1[:, :3, :3], e2[:, :3, :3] = r1, r2
    e1[:, 3, 3] = e2[:, 3, 3] = 1.0
    return e2 @ _boost_matrix(beta) @ e1


def test_identity_is_exact():
    x = _vectors(1000, 901)
    eye4 = [np.array([1.0 if a == c else 0.0]) for a in range(4) for c in range(4)]
    assert all(np.array_equal(a, b) for a, b in zip(oracle.lorentz_transform(x, eye4, 0), x))
    eye3 = [np.array([1.0 if a == c else 0.0]) for a in range(3) for c in range(3)]
    assert all(np.array_equal(a, b) for a, b in zip(oracle.rotate(x, eye3, 0), x))
    for aa in ([0.0, 0.0, 0.0, 1.3], [0.3, -2.0, 0.7, 0.0]):  # zero axis, zero angle
        y = oracle.rotate_axis_angle(x, [np.array([v]) for v in aa], 0)
        assert all(np.array_equal(a, b) for a, b in zip(y, x))


def test_permutation_matrices_exact():
    """A quarter turn about z as an exact matrix: (px, py) -> (-py, px)."""
    x = _vectors(1000, 902)
    rz = [np.array([v]) for v in (0.0, -1.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 1.0)]
    y = oracle.rotate(x, rz, 0)
    assert np.array_equal(y[0], -x[1]) and np.array_equal(y[1], x[0])
    assert np.array_equal(y[2], x[2]) and np.array_equal(y[3], x[3])
    # the same as a 4x4 matrix with E untouched: bitwise the same (zeros add exactly)
    l4 = [np.array([v]) for v in (0, -1, 0, 0, 1, 0, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1.0)]
    assert all(np.array_equal(a, b) for a, b in zip(oracle.lorentz_transform(x, l4, 0), y))
    # a time reversal and a parity flip
    tp = [np.array([v]) for v in (-1, 0, 0, 0, 0, -1, 0, 0, 0, 0, -1, 0, 0, 0, 0, -1.0)]
    assert all(np.array_equal(a, -b) for a, b in zip(oracle.lorentz_transform(x, tp, 0), x))


def test_rotation_as_lorentz_is_bitwise_the_same():
    x = _vectors(2000, 903)
    r = Rotation.random(2000, random_state=5).as_matrix()
    m = np.zeros((2000, 4, 4))
    m[:, :3, :3] = r
    m[:, 3, 3] = 1.0
    a = oracle.rotate(x, _cols(r), 1)
    b = oracle.lorentz_transform(x, _cols(m), 1)
    assert all(np.array_equal(u, v) for u, v in zip(a, b))


def test_boost_matrix_matches_the_boost():
    x, beta = synth.boost_items(synth.rng(904), 3000)
    y = oracle.lorentz_transform(x, _cols(_boost_matrix(beta)), 1)
    ref = oracle.boost_q(x, beta)
    scale = oracle.boost_scale(x, beta)
    for k in range(4):
        assert np.all(np.abs(y[k] - ref[k]) <= 16 * U * scale[k]), k


def test_composition_and_minkowski_norm():
    x = _vectors(3000, 905)
    l1, l2 = _random_lorentz(3000, 906), _random_lorentz(3000, 907)
    two = oracle.lorentz_transform(oracle.lorentz_transform(x, _cols(l1), 1), _cols(l2), 1)
    one = oracle.lorentz_transform(x, _cols(l2 @ l1), 1)
    absl = np.abs(l2) @ np.abs(l1)
    xa = np.abs(np.stack(x, axis=1))
    scale = np.einsum("nij,nj->ni", absl, xa)
    for k in range(4):
        assert np.all(np.abs(two[k] - one[k]) <= 64 * U * scale[:, k]), k
    y = oracle.lorentz_transform(x, _cols(l1), 1)
    q0 = x[3] ** 2 - x[0] ** 2 - x[1] ** 2 - x[2] ** 2
    q1 = y[3] ** 2 - y[0] ** 2 - y[1] ** 2 - y[2] ** 2
    s = np.sum(np.stack(y) ** 2, axis=0) + np.sum(np.stack(x) ** 2, axis=0)
    assert np.all(np.abs(q1 - q0) <= 1e-13 * s)


def test_axis_angle_against_scipy():
    g = synth.rng(908)
    n = 3000
    x = _vectors(n, 909)
    axis = g.normal(size=(n, 3)) * g.uniform(0.1, 10.0, (n, 1))  # not unit: normalised by the rotation
    angle = g.uniform(-7.0, 7.0, n)
    y = oracle.rotate_axis_angle(x, [axis[:, 0], axis[:, 1], axis[:, 2], angle], 1)
    u = axis / np.linalg.norm(axis, axis=1, keepdims=True)
    ref = Rotation.from_rotvec(u * angle[:, None]).apply(np.stack(x[:3], axis=1))
    pn = np.linalg.norm(ref, axis=1)
    for k in range(3):
        assert np.all(np.abs(y[k] - ref[:, k]) <= 32 * U * pn), k
    assert np.array_equal(y[3], x[3])
    # the same rotation as a matrix through orc_rotate
    r = Rotation.from_rotvec(u * angle[:, None]).as_matrix()
    yr = oracle.rotate(x, _cols(r), 1)
    for k in range(3):
        assert np.all(np.abs(y[k] - yr[k]) <= 32 * U * pn), k
    # broadcast: a quarter turn about +z
    q = oracle.rotate_axis_angle(x, [np.array([v]) for v in (0.0, 0.0, 2.5, np.pi / 2)], 0)
    assert np.all(np.abs(q[0] + x[1]) <= 4 * U * pn) and np.all(np.abs(q[1] - x[0]) <= 4 * U * pn)
    assert np.all(np.abs(q[2] - x[2]) <= 4 * U * np.abs(x[2]))  # cos(pi/2) rounds to 6e-17, not 0


def _fd(f, cols, k, h):
    up, dn = list(cols), list(cols)
    up[k] = cols[k] + h
    dn[k] = cols[k] - h
    return (f(up) - f(dn)) / (2 * h)


def test_lorentz_and_rotation_vjps():
    n = 500
    x = _vectors(n, 910)
    g = synth.rng(911)
    m = g.normal(size=(n, 4, 4))  # not symmetric: a transposed index would show
    gy = tuple(g.standard_normal(n) for _ in range(4))
    gx, gm = oracle.lorentz_transform_vjp(x, _cols(m), gy)
    # adjoint identity <g, L x> = <L^T g, x>
    lhs = sum(a * b for a, b in zip(gy, oracle.lorentz_transform(x, _cols(m), 1)))
    rhs = sum(a * b for a, b in zip(gx, x))
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.max(np.abs(lhs)))
    # grad of each matrix entry through the forward (linear: central differences exact up to rounding)
    mc = _cols(m)
    f = lambda cols: sum(a * b for a, b in zip(gy, oracle.lorentz_transform(x, cols, 1)))  # noqa: E731
    for k in range(16):
        fd = _fd(f, mc, k, 1e-3)
        assert np.allclose(fd, gm[k], rtol=1e-9, atol=1e-9 * np.max(np.abs(gm[k]))), k
    fx = lambda cols: sum(a * b for a, b in zip(gy, oracle.lorentz_transform(cols, mc, 1)))  # noqa: E731
    for k in range(4):
        assert np.allclose(_fd(fx, list(x), k, 1e-3), gx[k], rtol=1e-9, atol=1e-9), k
    # rotation
    r = g.normal(size=(n, 3, 3))
    gx, gr = oracle.rotate_vjp(x, _cols(r), gy)
    rc = _cols(r)
    fr = lambda cols: sum(a * b for a, b in zip(gy, oracle.rotate(x, cols, 1)))  # noqa: E731
    for k in range(9):
        assert np.allclose(_fd(fr, rc, k, 1e-3), gr[k], rtol=1e-9, atol=1e-9 * np.max(np.abs(gr[k]))), k
    fx = lambda cols: sum(a * b for a, b in zip(gy, oracle.rotate(cols, rc, 1)))  # noqa: E731
    for k in range(4):
        assert np.allclose(_fd(fx, list(x), k, 1e-3), gx[k], rtol=1e-9, atol=1e-9), k
    # broadcast matrices: the same grad_x as the per-item path with copies of the matrix
    one = [np.array([v]) for v in m[0].ravel()]
    gx0, _ = oracle.lorentz_transform_vjp(x, one, gy, stride=0, want_gm=False)
    gx1, _ = oracle.lorentz_transform_vjp(x, [np.full(n, v[0]) for v in one], gy, stride=1, want_gm=False)
    assert all(np.array_equal(a, b) for a, b in zip(gx0, gx1))


def test_axis_angle_vjp():
    n = 500
    g = synth.rng(912)
    x = _vectors(n, 913)
    aa = [g.normal(size=n), g.normal(size=n), g.normal(size=n), g.uniform(-4, 4, n)]
    gy = tuple(g.standard_normal(n) for _ in range(4))
    gx = oracle.rotate_axis_angle_vjp(aa, gy)
    f = lambda cols: sum(a * b for a, b in zip(gy, oracle.rotate_axis_angle(cols, aa, 1)))  # noqa: E731
    for k in range(4):
        assert np.allclose(_fd(f, list(x), k, 1e-3), gx[k], rtol=1e-8, atol=1e-8), k
    # orthogonal: rotating the reverse-mode result forward returns the upstream
    back = oracle.rotate_axis_angle(gx, aa, 1)
    for k in range(4):
        assert np.allclose(back[k], gy[k], rtol=0, atol=1e-14 * np.max(np.abs(gy[k]))), k
