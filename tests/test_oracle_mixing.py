"""Pins of the oracle's mixing-width function (oracle/mixing.py) against
closed forms of the integral width h = sum_j 6 c_j (1 - c_j)."""
import math

import numpy as np
import pytest

from oracle import mixing


def _profile_from_c(c, lo, hi):
    """Row profile phibar = lo + (hi - lo) c of a concentration profile."""
    return [lo + (hi - lo) * v for v in c]


@pytest.mark.parametrize("m", [1, 2, 7, 40, 333])
def test_linear_ramp(m):
    """c rises linearly across m rows, c_j = (j + 1/2)/m, with pure rows
    (c = 0 below, c = 1 above) around it.  Then
    sum c = m/2, sum c^2 = (4 m^2 - 1)/(12 m), so h = m + 1/(2 m)."""
    trim, below, above = 10, 25, 31
    lo, hi = -0.9, 1.0
    c = [0.0] * (trim + below) + [(j + 0.5) / m for j in range(m)] + [1.0] * (above + trim)
    h = mixing.mixing_width(_profile_from_c(c, lo, hi), lo, hi, trim)
    assert h == pytest.approx(m + 1.0 / (2 * m), rel=1e-13)
    # A on the bottom: the references swap, the width does not change
    c_down = [1.0 - v for v in c]
    h2 = mixing.mixing_width(_profile_from_c(c_down, hi, lo), hi, lo, trim)
    assert h2 == pytest.approx(m + 1.0 / (2 * m), rel=1e-13)


@pytest.mark.parametrize("w,y0", [(4.0, 0.0), (4.5, 0.37), (9.5, -0.21)])
def test_tanh_profile(w, y0):
    """c = (1 + tanh((y - y0)/w))/2 gives 6 c (1 - c) = (3/2) sech^2((y - y0)/w).
    By Poisson summation its sum over the integers is the integral 3 w times
    1 + 2 cos(2 pi y0) x / sinh(x) + ..., x = pi^2 w, i.e. 3 w to 1e-15 for
    w >= 4; the cut tails add exp(-400 / w)."""
    ny, trim = 420, 10
    y = np.arange(ny) - 0.5 * (ny - 1)
    c = 0.5 * (1.0 + np.tanh((y - y0) / w))
    lo, hi = -0.5, 0.5
    h = mixing.mixing_width(_profile_from_c(c, lo, hi), lo, hi, trim)
    assert h == pytest.approx(3.0 * w, rel=1e-13)


def test_overshoot_is_clamped_and_trim_rows_ignored():
    """Rows beyond the bulk references are pure (c clamped to 0 or 1) and add
    nothing; the trimmed rows are not summed even if they are mixed."""
    trim, lo, hi = 10, -0.6, 0.7
    prof = [0.05] * trim + [1.3 * hi] * 30 + [1.1 * lo] * 30 + [0.05] * trim
    assert mixing.mixing_width(prof, lo, hi, trim) == 0.0
    # one half-mixed row (c = 1/2) inside D adds 6/4
    prof[trim + 30] = 0.5 * (lo + hi)
    assert mixing.mixing_width(prof, lo, hi, trim) == pytest.approx(1.5, rel=1e-15)
    # the same row in the trimmed band adds nothing
    prof[trim + 30] = 1.1 * lo
    prof[trim - 1] = 0.5 * (lo + hi)
    assert mixing.mixing_width(prof, lo, hi, trim) == 0.0


def test_reference_rows_and_asymmetric_phases():
    """The references are phibar at rows trim and ny - trim - 1 of the t = 0
    profile, whatever the trimmed rows hold.  Asymmetric bulk phases
    (+1.0 on top, -0.9 below, as in the synthetic workloads) are both pure
    (h = 0); reading c as (1 + phibar/phi_ref)/2 with one phi_ref would give
    every row of the lower phase 6 c (1 - c) = 0.154."""
    trim, ny = 10, 80
    prof = [-0.9] * (ny // 2) + [1.0] * (ny // 2)
    # every trimmed row (the ones next to D included) holds another value
    for j in list(range(trim)) + list(range(ny - trim, ny)):
        prof[j] = 7.0 + j
    lo, hi = mixing.bulk_reference(prof, trim)
    assert (lo, hi) == (-0.9, 1.0)
    assert mixing.mixing_width(prof, lo, hi, trim) == 0.0
    # a quarter-mixed row: c = 1/4 -> 6 (1/4)(3/4) = 9/8
    prof[trim + 5] = lo + 0.25 * (hi - lo)
    assert mixing.mixing_width(prof, lo, hi, trim) == pytest.approx(9.0 / 8.0, rel=1e-14)


def test_rejects_empty_domain_and_equal_references():
    with pytest.raises(ValueError):
        mixing.mixing_width([0.0] * 20, -1.0, 1.0, 10)
    with pytest.raises(ValueError):
        mixing.mixing_width([0.0] * 30, 0.5, 0.5, 10)
    with pytest.raises(ValueError):
        mixing.bulk_reference([0.0] * 20, 10)


def test_width_of_the_initial_lb_interface(orc):
    """The oracle's own t = 0 state: a flat interface with
    s = (1 + tanh((j - y_int)/1.5))/2, rho_A = 0.05 + s, rho_B = 0.05 + 0.9 (1 - s),
    so phibar = 1.9 s - 0.9 is affine in s, c = s (the bulk rows have s within
    1e-21 of 0 and 1) and h = sum_j 6 s_j (1 - s_j): 3 * 1.5 = 4.5 up to the
    Poisson term 2 x/sinh(x), x = 1.5 pi^2 (2.2e-5 relative)."""
    from paper_2101_04847_amd import inputs
    nx, ny, trim = 16, 96, 10
    y_int = 0.5 * (ny - 1) + 0.3
    rA, rB = inputs.two_phase_densities(nx, ny, np.full(nx, y_int))
    p = orc.Params(nx=nx, ny=ny)
    f = orc.fill_equilibrium(p, rA, rB)
    prof = orc.diagnostics(p, f, trim=trim, profile=True)["phi_profile"]
    lo, hi = mixing.bulk_reference(prof, trim)
    assert lo == pytest.approx(-0.9, abs=1e-15) and hi == pytest.approx(1.0, abs=1e-15)
    h = mixing.mixing_width(prof, lo, hi, trim)
    x = 1.5 * math.pi ** 2
    assert abs(h - 4.5) <= 4.5 * 2 * x / math.sinh(x) * 1.01
    s = [0.5 * (1 + math.tanh((j - y_int) / 1.5)) for j in range(trim, ny - trim)]
    assert h == pytest.approx(math.fsum(6 * v * (1 - v) for v in s), rel=1e-12)
