"""Length of the interface phi = 0 (Sec. 3, Eq. 20-21) by Cauchy-Crofton
line-intersection counts (numpy).

TEST INFRASTRUCTURE ONLY: used by ``tests/`` to check the GPU library's
interface pass.  Nothing in the GPU package imports it.

The interface of the immiscible mixture is the curve phi = rho_A - rho_B = 0
(Sec. 3).  Its length follows from the Cauchy-Crofton formula
L = (1/2) int_0^pi int n(theta, p) dp dtheta (n: crossings of the line at
angle theta and offset p with the curve), sampled on the lattice lines in
four directions: rows (theta = 0), columns (pi/2) and the two diagonals
(pi/4, 3 pi/4, whose lines are 1/sqrt(2) apart).  A crossing is a pair of
neighbouring sites along the line with phi > 0 at exactly one of them.
With N_0, N_90, N_45, N_135 the crossing counts,

    L = (pi / 8) [N_0 + N_90 + (N_45 + N_135) / sqrt(2)].

Pairs are counted when both sites lie in the trimmed domain D (rows
[trim, ny - trim)); x is periodic.
"""
from __future__ import annotations

import numpy as np


def crossing_counts(phi, trim: int = 10) -> dict:
    """Crossing counts along the four lattice directions (integers)."""
    pos = np.asarray(phi, dtype=np.float64) > 0.0
    d = pos[trim:pos.shape[0] - trim]
    right = np.roll(d, -1, axis=1)                 # (x + 1, y)
    n0 = int(np.count_nonzero(d != right))
    n90 = int(np.count_nonzero(d[:-1] != d[1:]))   # (x, y) - (x, y + 1)
    n45 = int(np.count_nonzero(d[:-1] != right[1:]))    # (x, y) - (x + 1, y + 1)
    n135 = int(np.count_nonzero(right[:-1] != d[1:]))   # (x + 1, y) - (x, y + 1)
    return {"n0": n0, "n90": n90, "n45": n45, "n135": n135}


def crofton_length(c: dict) -> float:
    """L = (pi/8) [N_0 + N_90 + (N_45 + N_135)/sqrt(2)]."""
    return float(np.pi / 8.0 * (c["n0"] + c["n90"] + (c["n45"] + c["n135"]) / np.sqrt(2.0)))


def interface_length(rhoA, rhoB, trim: int = 10) -> dict:
    """Crossing counts and Cauchy-Crofton length of phi = rho_A - rho_B = 0."""
    phi = np.asarray(rhoA, dtype=np.float64) - np.asarray(rhoB, dtype=np.float64)
    c = crossing_counts(phi, trim)
    c["length"] = crofton_length(c)
    return c
