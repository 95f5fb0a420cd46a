"""Integral width of the Rayleigh-Taylor mixing layer from the row profile of
the order parameter (plain Python loops over rows).

TEST INFRASTRUCTURE ONLY: used by ``tests/`` to check the GPU library's
mixing-width reduction.  Nothing in the GPU package imports it.

The paper (Sec. 3) follows the growth of the mixing layer between the two
pure phases but defines no width; this module takes the integral reading.
With phibar(j) the mean of phi = rho_A - rho_B over row j (the profile the
oracle's diagnostics return) and phi_lo, phi_hi the values of phibar at the
first and the last row of the trimmed domain D at t = 0 (the two bulk
phases), the local fraction of the phase that starts at the top is

    c_j = clamp((phibar(j) - phi_lo) / (phi_hi - phi_lo), 0, 1)

and the width is

    h = sum over rows j of D of 6 c_j (1 - c_j).

When the bulk phases are symmetric (phi_lo = -phi_hi) this is
c_j = (1 + phibar(j)/phi_ref)/2 with phi_ref = (phi_hi - phi_lo)/2.  A pure
row adds nothing; a linear ramp of c across m rows gives m + 1/(2m); a tanh
profile of width w gives 3w.
"""
from __future__ import annotations


def bulk_reference(profile0, trim: int = 10):
    """(phi_lo, phi_hi): the row means of phi at rows trim and ny - trim - 1
    of the t = 0 profile (the bulk rows just inside D)."""
    p = [float(v) for v in profile0]
    ny = len(p)
    if ny - 2 * trim <= 0:
        raise ValueError("the trimmed domain is empty")
    return p[trim], p[ny - trim - 1]


def concentration(phibar: float, phi_lo: float, phi_hi: float) -> float:
    """Fraction of the top phase in a row, clamped to [0, 1]."""
    c = (phibar - phi_lo) / (phi_hi - phi_lo)
    if c < 0.0:
        return 0.0
    if c > 1.0:
        return 1.0
    return c


def mixing_width(profile, phi_lo: float, phi_hi: float, trim: int = 10) -> float:
    """h = sum_{j in D} 6 c_j (1 - c_j), summed over the rows of D in order."""
    p = [float(v) for v in profile]
    ny = len(p)
    if ny - 2 * trim <= 0:
        raise ValueError("the trimmed domain is empty")
    if not phi_hi != phi_lo:
        raise ValueError("the two bulk references must differ")
    h = 0.0
    for j in range(trim, ny - trim):
        c = concentration(p[j], phi_lo, phi_hi)
        h += 6.0 * c * (1.0 - c)
    return h
