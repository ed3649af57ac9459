"""Pass criteria shared by the oracle pins and the GPU parity tests.

The mass of a sum is E^2 - |P|^2 under a square root: the subtraction cancels,
so a rounding error of a few units in the last place (u) of the terms moves
q = m^2 by about u * S, with S = E^2 + |P|^2, and m by u * S / (2 |m|).
Every floating-point criterion is therefore "relative part + conditioning
part".  u64 = 2^-53, u32 = 2^-24.
"""

import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24
TINY = 1e-300


def mass_tol_f64(m_ref, scale):
    """FP64 mass (plain form): 1e-12 |m| + 64 u64 S / (2 |m|)."""
    am = np.abs(m_ref)
    return 1e-12 * am + 64 * U64 * scale / (2 * np.maximum(am, TINY))


def mass_tol_f32(m_ref, scale):
    """FP32 mass (plain form): 1e-5 |m| + 64 u32 S / (2 |m|)."""
    am = np.abs(m_ref)
    return 1e-5 * am + 64 * U32 * scale / (2 * np.maximum(am, TINY))


def mass_tol_comp_f32(m_ref):
    """FP32 compensated mass, graded against an accurate FP64 reference:
    4e-6 relative + 1e-6 GeV absolute, whatever the conditioning."""
    return 4e-6 * np.abs(m_ref) + 1e-6


def mass_tol_acc_f64(m_ref):
    """FP64 cancellation-free mass against a binary128 reference: 8 u64."""
    return 8 * U64 * np.abs(m_ref) + 1e-300


def boost_tol(scale, dtype):
    """Boosted components: 1e-12 (FP64) or 2^-19 (FP32) of (|L| |x|)_i."""
    return (1e-12 if dtype == np.float64 else 2.0 ** -19) * scale


def worst(err, tol):
    """Largest err/tol ratio (<= 1 passes) and its index."""
    err = np.asarray(err, dtype=np.float64)
    tol = np.asarray(tol, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(err == 0, 0.0, err / tol)  # an exact match passes even at zero tolerance
    r = np.where(np.isnan(r), np.inf, r)
    i = int(np.argmax(r)) if r.size else 0
    return (float(r[i]) if r.size else 0.0), i
