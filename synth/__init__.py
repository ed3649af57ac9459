"""Seeded synthetic inputs shaped like collider data.

This module only draws random numbers and lays them out as structure-of-arrays
(SoA) columns.  It holds none of the arithmetic of the Lorentz-vector method
(no coordinate conversion, no mass, no boost); both the GPU library's tests and
the CPU oracle consume the same arrays from here.

Every generator takes a ``numpy.random.Generator`` so a caller fixes the seed.
``rng(k)`` gives the stream used for workload ``k``: PCG64 seeded with
``SEED_BASE + k``.  Draws happen in the order the docstrings list, always in
float64; FP32 workloads are produced by casting afterwards.

Workloads (the paper has no public dataset; its inputs are arrays of particles
of varying size, Sec. 5.1-5.2):

* ``pairs_generic``  -- leg a then leg b, each pt = 5 + Exp(scale 30) GeV,
  eta ~ U[-2.5, 2.5], phi ~ U[-pi, pi), M ~ U[0, 0.2] GeV (PtEtaPhiM).
* ``boost_items``    -- px, py, pz ~ N(0, 50^2) GeV, M ~ U[0, 100] GeV, E on the
  mass shell; beta direction uniform on the sphere, |beta| ~ U[0, 0.99].
* ``pairs_stress``   -- light legs for the FP32 precision stress: pt =
  LogUniform[1, 2000] GeV, eta ~ U[-4, 4], phi ~ U[-pi, pi), M ~ U[0, 0.14]
  GeV; 10% of pairs have leg b nearly collinear with leg a (eta and phi
  offsets ~ U(-1e-3, 1e-3), eta clipped to [-4, 4], phi wrapped to [-pi, pi)).
* ``jagged_events``  -- multiplicity ~ Poisson(8) clipped to [0, 64], CSR
  offsets (int64), particles drawn as ``pairs_generic`` legs.
* ``leg_generic_device`` -- the ``pairs_generic`` leg distribution drawn
  straight into GPU memory by torch's generator (for inputs of billions of
  items, too large to draw on the host and copy); seeded like ``rng``.
"""

import numpy as np

SEED_BASE = 2312027560

# Workload indices used with ``rng``.
SMALL_PAIRS = 0   # 65,536 generic pairs, FP64
LARGE = 1         # 2^24 boost items and 2^24 generic pairs, FP64
STRESS = 2        # 2^26 light pairs, FP32
GRADS = 3         # 2^24 items, upstream gradients
JAGGED = 4        # 2^20 jagged events
JAGGED_GRADS = 5  # upstream gradients of the jagged reduction (totals, event and pair masses)


def rng(k: int) -> np.random.Generator:
    """PCG64 stream for workload ``k``."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + int(k)))


def _leg_generic(g: np.random.Generator, n: int):
    pt = 5.0 + g.exponential(30.0, n)
    eta = g.uniform(-2.5, 2.5, n)
    phi = g.uniform(-np.pi, np.pi, n)
    m = g.uniform(0.0, 0.2, n)
    return pt, eta, phi, m


def pairs_generic(g: np.random.Generator, n: int):
    """Two PtEtaPhiM legs (a, b) of ``n`` items each, float64 SoA tuples."""
    a = _leg_generic(g, n)
    b = _leg_generic(g, n)
    return a, b


def boost_items(g: np.random.Generator, n: int):
    """PxPyPzE vectors x and per-item velocities beta, float64 SoA tuples.

    Draw order: px, py, pz, M, cos(theta), azimuth, |beta|.
    """
    px = g.normal(0.0, 50.0, n)
    py = g.normal(0.0, 50.0, n)
    pz = g.normal(0.0, 50.0, n)
    m = g.uniform(0.0, 100.0, n)
    e = np.sqrt(px * px + py * py + pz * pz + m * m)
    cth = g.uniform(-1.0, 1.0, n)
    az = g.uniform(-np.pi, np.pi, n)
    bmag = g.uniform(0.0, 0.99, n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    beta = (bmag * sth * np.cos(az), bmag * sth * np.sin(az), bmag * cth)
    return (px, py, pz, e), beta


def _wrap_phi(p):
    """Wrap angles into [-pi, pi)."""
    return (p + np.pi) % (2.0 * np.pi) - np.pi


def pairs_stress(g: np.random.Generator, n: int, collinear_frac: float = 0.1):
    """Light, wide-pt legs; a fraction of pairs nearly collinear.

    Draw order: leg a (pt, eta, phi, M), leg b (pt, eta, phi, M), collinear
    mask, eta offset, phi offset.  Returns (a, b, mask) with float64 arrays.
    """
    def leg():
        pt = np.exp(g.uniform(0.0, np.log(2000.0), n))
        eta = g.uniform(-4.0, 4.0, n)
        phi = g.uniform(-np.pi, np.pi, n)
        m = g.uniform(0.0, 0.14, n)
        return pt, eta, phi, m

    a = leg()
    pt_b, eta_b, phi_b, m_b = leg()
    mask = g.random(n) < collinear_frac
    deta = g.uniform(-1e-3, 1e-3, n)
    dphi = g.uniform(-1e-3, 1e-3, n)
    eta_b = np.where(mask, np.clip(a[1] + deta, -4.0, 4.0), eta_b)
    phi_b = np.where(mask, _wrap_phi(a[2] + dphi), phi_b)
    return a, (pt_b, eta_b, phi_b, m_b), mask


def upstream(g: np.random.Generator, n: int, k: int):
    """``k`` arrays of N(0, 1) upstream gradients."""
    return tuple(g.standard_normal(n) for _ in range(k))


def jagged_events(g: np.random.Generator, n_events: int, mean: float = 8.0, cap: int = 64):
    """CSR jagged events.  Returns (offsets int64[n_events+1], particles SoA).

    Draw order: multiplicities, then the particles as one generic leg.
    """
    counts = np.minimum(g.poisson(mean, n_events), cap).astype(np.int64)
    offsets = np.zeros(n_events + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    parts = _leg_generic(g, int(offsets[-1]))
    return offsets, parts


def as_dtype(cols, dtype):
    """Cast a tuple of columns to ``dtype`` (contiguous copies)."""
    return tuple(np.ascontiguousarray(c, dtype=dtype) for c in cols)


def leg_generic_device(k: int, n: int, device, dtype):
    """One PtEtaPhiM leg of ``n`` items drawn on ``device`` (a torch device)
    with a torch generator seeded with ``SEED_BASE + k``: pt = 5 + Exp(scale
    30) GeV, eta ~ U[-2.5, 2.5], phi ~ U[-pi, pi), M ~ U[0, 0.2] GeV, in that
    order, each column drawn in ``dtype``.  Successive calls with one ``k``
    give the same columns."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(SEED_BASE + int(k))
    pt = torch.empty(n, dtype=dtype, device=device).exponential_(1.0 / 30.0, generator=g).add_(5.0)
    eta = torch.empty(n, dtype=dtype, device=device).uniform_(-2.5, 2.5, generator=g)
    phi = torch.empty(n, dtype=dtype, device=device).uniform_(-np.pi, np.pi, generator=g)
    m = torch.empty(n, dtype=dtype, device=device).uniform_(0.0, 0.2, generator=g)
    return pt, eta, phi, m


def normal_device(k: int, n: int, device, dtype):
    """``n`` N(0, 1) upstream gradients drawn on ``device`` with a torch
    generator seeded with ``SEED_BASE + k``."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(SEED_BASE + int(k))
    return torch.empty(n, dtype=dtype, device=device).normal_(generator=g)
