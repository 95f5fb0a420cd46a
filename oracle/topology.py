"""Connected components of the two phases (Sec. 3: the topology change of the
interface) (numpy + scipy).

TEST INFRASTRUCTURE ONLY: used by ``tests/`` to check the GPU library's
component count.  Nothing in the GPU package imports it.

The A-rich phase is the set phi = rho_A - rho_B > 0 and the B-rich phase its
complement, both restricted to the trimmed domain D (rows [trim, ny - trim))
with x periodic.  Two sites of the same phase are connected when they are
neighbours along a row or a column (4-connectivity); the counts are the
numbers of connected components of each phase.  scipy's labelling does the
non-periodic part; labels that meet across the x seam are then merged.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage


def _count_periodic_x(mask: np.ndarray) -> int:
    lab, n = ndimage.label(mask)   # 4-connectivity (the default cross)
    if n == 0:
        return 0
    parent = list(range(n + 1))

    def find(a):
        while parent[a] != a:
            a = parent[a]
        return a

    merged = 0
    for y in range(mask.shape[0]):
        a, b = lab[y, -1], lab[y, 0]
        if a and b:
            ra, rb = find(a), find(b)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
                merged += 1
    return n - merged


def component_counts(rhoA, rhoB, trim: int = 10) -> dict:
    """Numbers of 4-connected components of phi > 0 and of phi <= 0 in D."""
    phi = np.asarray(rhoA, dtype=np.float64) - np.asarray(rhoB, dtype=np.float64)
    d = phi[trim:phi.shape[0] - trim] > 0.0
    return {"A": _count_periodic_x(d), "B": _count_periodic_x(~d)}
