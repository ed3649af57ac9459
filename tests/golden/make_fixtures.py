"""Writes tests/golden/pair_masses.txt: hand-picked PtEtaPhiM pairs (the pair
mass of GenVectorX Sec. 4.1 / Fig. 1) with their masses from the CPU oracle --
the definition evaluated in binary128 and rounded to binary64, and the
cancellation-free form in binary64.  The paper prints no worked numerical
example, so these are oracle values; the file guards them against drift and
gives the GPU tests fixed cases.  Run from the repository root:

    python tests/golden/make_fixtures.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle  # noqa: E402

# (label, leg a (pt, eta, phi, M), leg b) in GeV and radians
CASES = [
    ("generic", (45.0, 0.7, 1.2, 0.105), (30.0, -1.1, -2.3, 0.000511)),
    ("z_like", (45.6, 0.3, 0.4, 0.0), (45.6, -0.3, 0.4 - np.pi, 0.0)),
    ("collinear_light", (120.0, 1.5, 0.25, 0.13957), (80.0, 1.5 + 2e-4, 0.25 - 3e-4, 0.13957)),
    ("identical_massless", (50.0, 0.5, 1.0, 0.0), (50.0, 0.5, 1.0, 0.0)),
    ("identical_massive", (50.0, 0.5, 1.0, 0.1), (50.0, 0.5, 1.0, 0.1)),
    ("zero_leg", (0.0, 0.0, 0.0, 0.0), (30.0, 2.0, -1.0, 1.5)),
    ("seam_plus_minus_pi", (60.0, 0.1, np.pi - 1e-4, 0.0), (40.0, 0.1, -np.pi + 2e-4, 0.0)),
    ("large_eta", (5.0, 3.9, 0.0, 0.105), (7.0, -3.8, 0.1, 0.105)),
    ("heavy_slow", (0.5, 2.0, 0.3, 9.46), (0.7, -2.5, -2.9, 3.097)),
    ("high_pt", (1500.0, 0.05, -0.7, 0.0), (1200.0, -0.02, 2.4, 4.18)),
    ("back_to_back_equal", (25.0, 0.0, 0.0, 0.0), (25.0, 0.0, np.pi, 0.0)),
    ("nearly_collinear_massless", (300.0, 0.8, 1.0, 0.0), (20.0, 0.8 + 1e-6, 1.0 + 1e-6, 0.0)),
]


def cols(legs):
    return tuple(np.array([leg[k] for leg in legs], dtype=np.float64) for k in range(4))


def render():
    a, b = cols([c[1] for c in CASES]), cols([c[2] for c in CASES])
    m_q = oracle.mass_plain_q("PtEtaPhiM", a, b)
    m_acc = oracle.mass_accurate(a, b)
    lines = ["# Pair masses of PtEtaPhiM legs (GenVectorX Sec. 4.1, Fig. 1: convert, add, mass of the sum).",
             "# No worked example is printed in the paper: m_binary128 is the oracle's definition in binary128",
             "# rounded to binary64, m_accurate its cancellation-free form in binary64.  Written by",
             "# tests/golden/make_fixtures.py; columns: label, pt_a eta_a phi_a M_a, pt_b eta_b phi_b M_b,",
             "# m_binary128, m_accurate (all as exact binary64 hex floats)."]
    for i, (label, _, _) in enumerate(CASES):
        vals = [a[k][i] for k in range(4)] + [b[k][i] for k in range(4)] + [m_q[i], m_acc[i]]
        lines.append(label + " " + " ".join(float(v).hex() for v in vals))
    return "\n".join(lines) + "\n"


def load(path=os.path.join(HERE, "pair_masses.txt")):
    """(labels, a, b, m_binary128, m_accurate) from the fixture file."""
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    labels = [r[0] for r in rows]
    v = np.array([[float.fromhex(x) for x in r[1:]] for r in rows])
    return labels, tuple(v[:, k] for k in range(4)), tuple(v[:, 4 + k] for k in range(4)), v[:, 8], v[:, 9]


if __name__ == "__main__":
    with open(os.path.join(HERE, "pair_masses.txt"), "w") as fh:
        fh.write(render())
