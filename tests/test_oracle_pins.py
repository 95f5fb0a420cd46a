"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact
rational identities, conservation laws, closed forms, or a published formula
of the paper.  The slower hydrodynamic checks live in test_oracle_physics.py.
"""
from fractions import Fraction

import numpy as np
import pytest


def _det3(m):
    return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
            - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
            + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))


def test_lattice_constants_from_isotropy(orc):
    """Eq. 4 (with c_s^2 = 1/3 and sum_i w_i = 1) fixes the D2Q9 weights.

    Unknowns: w_rest, w_axis, w_diag (weights depend only on |c_i| by the
    lattice symmetry).  Conditions, in exact rationals:
      w_rest + 4 w_axis + 4 w_diag = 1             (normalisation)
      2 w_axis + 4 w_diag          = c_s^2         (sum w c_x c_x)
      4 w_diag                     = c_s^4         (sum w c_x^2 c_y^2)
    and the fourth-order xxxx condition 2 w_axis + 4 w_diag = 3 c_s^4 must then
    hold too.  Solved by Cramer's rule.
    """
    cs2 = Fraction(1, 3)
    A = [[Fraction(1), Fraction(4), Fraction(4)],
         [Fraction(0), Fraction(2), Fraction(4)],
         [Fraction(0), Fraction(0), Fraction(4)]]
    b = [Fraction(1), cs2, cs2 * cs2]
    D = _det3(A)
    sol = []
    for k in range(3):
        Ak = [row[:] for row in A]
        for r in range(3):
            Ak[r][k] = b[r]
        sol.append(_det3(Ak) / D)
    w_rest, w_axis, w_diag = sol
    assert 2 * w_axis + 4 * w_diag == 3 * cs2 * cs2
    assert (w_rest, w_axis, w_diag) == (Fraction(4, 9), Fraction(1, 9), Fraction(1, 36))

    cx, cy, opp, w = orc.constants()
    vel = set(zip(cx.tolist(), cy.tolist()))
    assert vel == {(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)}
    for i in range(9):
        expect = {0: w_rest, 1: w_axis, 2: w_diag}[abs(cx[i]) + abs(cy[i])]
        assert w[i] == float(expect)
        assert cx[opp[i]] == -cx[i] and cy[opp[i]] == -cy[i]
    # the isotropy sums, evaluated exactly with the weights the oracle holds
    wf = [Fraction(float(x)).limit_denominator(100) for x in w]
    for a in range(2):
        for b_ in range(2):
            s2 = sum(wf[i] * [cx, cy][a][i] * [cx, cy][b_][i] for i in range(9))
            assert s2 == (cs2 if a == b_ else 0)
            assert sum(wf[i] * [cx, cy][a][i] for i in range(9)) == 0


def test_equilibrium_moments(orc):
    """Eq. 3: zeroth, first and second moments of f^eq are rho, rho v and
    rho (v v + c_s^2 I), exactly up to rounding, for any rho and v."""
    cx, cy, _, _ = orc.constants()
    rng = np.random.default_rng(5)
    for _ in range(50):
        rho = rng.uniform(0.01, 2.0)
        vx, vy = rng.uniform(-0.2, 0.2, 2)
        feq = orc.equilibrium(rho, vx, vy)
        assert abs(feq.sum() - rho) <= 1e-15 * rho * 4
        assert abs((feq * cx).sum() - rho * vx) <= 1e-15 * rho * 4
        assert abs((feq * cy).sum() - rho * vy) <= 1e-15 * rho * 4
        pxx, pyy, pxy = (feq * cx * cx).sum(), (feq * cy * cy).sum(), (feq * cx * cy).sum()
        assert abs(pxx - rho * (vx * vx + 1 / 3)) <= 1e-15 * rho * 8
        assert abs(pyy - rho * (vy * vy + 1 / 3)) <= 1e-15 * rho * 8
        assert abs(pxy - rho * vx * vy) <= 1e-15 * rho * 8


def _rt_start(orc, nx, ny, G, g, forcing, periodic_y=False, amp=2.0):
    from paper_2101_04847_amd import inputs
    p = orc.Params(nx=nx, ny=ny, tau=(1.0, 1.0), G=G, g=((0.0, -g), (0.0, g)),
                   forcing=forcing, periodic_y=periodic_y)
    rA, rB = inputs.single_mode(nx, ny, amp)
    return p, orc.fill_equilibrium(p, rA, rB)


@pytest.mark.parametrize("forcing", [0, 1])
def test_mass_conserved_per_component(orc, forcing):
    """Eq. 2: streaming is a permutation, BGK keeps each rho_s, and the
    bounce-back walls return every population: each component's mass is
    constant to rounding over 1000 steps of a forced, interacting run."""
    p, f = _rt_start(orc, 128, 64, 1.5, 1e-5, forcing)
    m0 = f.sum(axis=(1, 2, 3))
    f = orc.run(p, f, 1000)
    m1 = f.sum(axis=(1, 2, 3))
    assert np.all(np.abs(m1 - m0) / m0 < 1e-13)


@pytest.mark.parametrize("forcing", [0, 1])
def test_momentum_gains_exactly_the_impulse(orc, forcing):
    """Periodic box.  The Shan-Chen forces of Eq. 5 cancel pairwise over the
    lattice (link antisymmetry), so the total momentum sum_s sum_x sum_i f c
    changes per step by exactly the external impulse sum_s M_s g_s of Eq. 7,
    under both forcing schemes."""
    from paper_2101_04847_amd import inputs
    nx, ny = 48, 40
    g = 3e-5
    p = orc.Params(nx=nx, ny=ny, tau=(0.8, 0.8), G=1.5, g=((0.0, -g), (2e-6, g)),
                   forcing=forcing, periodic_y=True)
    amps, ph = inputs.random_modes(11, 4, 2.0)
    rA, rB = inputs.two_phase_densities(nx, ny, inputs.interface_height(nx, ny, amps, ph))
    f = orc.fill_equilibrium(p, rA, rB)
    cx, cy, _, _ = orc.constants()

    def mom(f):
        return np.array([(f * cx[None, :, None, None]).sum(), (f * cy[None, :, None, None]).sum()])

    mA, mB = f[0].sum(), f[1].sum()
    impulse = np.array([0.0 * mA + 2e-6 * mB, -g * mA + g * mB])
    p0 = mom(f)
    n = 200
    f = orc.run(p, f, n)
    assert np.allclose(mom(f) - p0, n * impulse, rtol=0, atol=1e-12 * (mA + mB))

    # without gravity the momentum is conserved
    p.g = ((0.0, 0.0), (0.0, 0.0))
    q0 = mom(f)
    f = orc.run(p, f, n)
    assert np.all(np.abs(mom(f) - q0) < 1e-13 * (mA + mB))


@pytest.mark.parametrize("forcing", [0, 1])
def test_uniform_rest_state_is_a_fixed_point_between_walls(orc, forcing):
    """A uniform mixture at rest between walls feels no Shan-Chen force,
    neither in the bulk nor next to the walls (neutral wetting, Sec. 2), and
    bounce-back keeps it at rest: one step maps it onto itself."""
    nx, ny = 16, 12
    p = orc.Params(nx=nx, ny=ny, tau=(0.53, 0.53), G=0.1381, forcing=forcing)
    f = orc.fill_equilibrium(p, np.full((ny, nx), 0.6), np.full((ny, nx), 0.5))
    f1 = orc.step(p, f)
    assert np.max(np.abs(f1 - f)) < 1e-15


def test_potential_energy_mass_and_buoyancy_closed_forms(orc):
    """Sec. 3 definitions on a field with rho_A = a + b y, rho_B = c, G = 0:
    E_p = g <y phi>_D = g b <y^2>_D with <y^2>_D = (m^2 - 1)/12 for the m rows
    of D centred on the channel, M_A = a nx ny, M_B = c nx ny, and (velocity
    u_phys = F/(2 rho) from rest) B = -g^2 <phi^2 / (2 rho)>_D."""
    nx, ny, trim = 20, 50, 10
    a, b, c, g = 0.9, 0.004, 0.7, 2e-3
    yj = np.arange(ny) - 0.5 * (ny - 1)
    rA = np.repeat((a + b * yj)[:, None], nx, axis=1)
    rB = np.full((ny, nx), c)
    p = orc.Params(nx=nx, ny=ny, tau=(1.0, 1.0), G=0.0, g=((0.0, -g), (0.0, g)))
    f = orc.fill_equilibrium(p, rA, rB)
    d = orc.diagnostics(p, f, trim=trim, profile=True)
    m = ny - 2 * trim
    assert d["Ep"] == pytest.approx(g * b * (m * m - 1) / 12.0, rel=1e-12)
    # row profile of phi = rho_A - rho_B over every row (trimmed ones too)
    assert np.max(np.abs(d["phi_profile"] - (a + b * yj - c))) <= 1e-14
    assert d["mass_A"] == pytest.approx(a * nx * ny, rel=1e-14)
    assert d["mass_B"] == pytest.approx(c * nx * ny, rel=1e-14)
    phi = (a + b * yj - c)[trim:ny - trim]
    rho = (a + b * yj + c)[trim:ny - trim]
    assert d["buoyancy"] == pytest.approx(-g * g * np.mean(phi * phi / (2 * rho)), rel=1e-12)
    assert d["omega2"] == 0.0 and d["Ek"] == pytest.approx(np.mean(rho * (g * phi / (2 * rho)) ** 2 / 2), rel=1e-12)


def test_each_component_relaxes_at_its_own_rate(orc):
    """Eq. 2 with tau_A != tau_B on a uniform mixture at rest (G = 0, g = 0,
    periodic y, so streaming maps the uniform state onto itself): a
    departure from equilibrium that carries no mass and no momentum (+e on
    the two x links, -e on the two y links) leaves rho and u, hence f^eq,
    unchanged, and decays by the factor 1 - 1/tau_s per step in component s."""
    nx, ny, e = 6, 5, 1e-3
    tau = (0.8, 1.7)
    p = orc.Params(nx=nx, ny=ny, tau=tau, periodic_y=True)
    f0 = orc.fill_equilibrium(p, np.full((ny, nx), 0.7), np.full((ny, nx), 0.4))
    cx, cy, _, _ = orc.constants()
    d = np.zeros_like(f0)
    for i in range(9):
        if cx[i] != 0 and cy[i] == 0:
            d[:, i] = e
        elif cy[i] != 0 and cx[i] == 0:
            d[:, i] = -e
    f1 = orc.step(p, f0 + d)
    for s in range(2):
        want = f0[s] + (1.0 - 1.0 / tau[s]) * d[s]
        assert np.max(np.abs(f1[s] - want)) <= 1e-15, s


def test_hydrodynamic_velocity_of_a_forced_rest_state(orc):
    """A uniform mixture at rest (j_A = j_B = 0) under body accelerations with
    x and y components (G = 0, periodic y: no Shan-Chen and no wall force):
    the total force is F = rho_A g_A + rho_B g_B, the hydrodynamic velocity
    is half of it over the density, u_phys = F / (2 rho), in both
    directions, and so E_k = rho |u_phys|^2 / 2, B = -<u_phys . F> =
    -|F|^2 / (2 rho) and max |u| = |F| / (2 rho)."""
    nx, ny = 9, 14
    rA, rB = 0.7, 0.45
    gA, gB = (3e-3, -2e-3), (-1e-3, 5e-3)
    p = orc.Params(nx=nx, ny=ny, tau=(0.8, 1.1), G=0.0, g=(gA, gB), periodic_y=True)
    f = orc.fill_equilibrium(p, np.full((ny, nx), rA), np.full((ny, nx), rB))
    m = orc.macro(p, f)
    rho = rA + rB
    Fx, Fy = rA * gA[0] + rB * gB[0], rA * gA[1] + rB * gB[1]
    assert np.max(np.abs(m["Fx"] - Fx)) <= 1e-16 and np.max(np.abs(m["Fy"] - Fy)) <= 1e-16
    assert np.max(np.abs(m["ux"] - Fx / (2 * rho))) <= 1e-16
    assert np.max(np.abs(m["uy"] - Fy / (2 * rho))) <= 1e-16
    d = orc.diagnostics(p, f, trim=2)
    u2 = (Fx * Fx + Fy * Fy) / (2 * rho) ** 2
    assert d["Ek"] == pytest.approx(0.5 * rho * u2, rel=1e-12)
    assert d["buoyancy"] == pytest.approx(-(Fx * Fx + Fy * Fy) / (2 * rho), rel=1e-12)
    assert d["umax"] == pytest.approx(np.sqrt(u2), rel=1e-14)


@pytest.mark.parametrize("n,N", [(1, 32), (3, 48)])
def test_enstrophy_and_kinetic_energy_taylor_green(orc, n, N):
    """Eq. 22 reduction on a Taylor-Green field u = U (sin kx cos ky,
    -cos kx sin ky), k = 2 pi n / N, loaded as the equilibrium of rho = 1 with
    G = g = 0 (so u_phys = u).  The centred difference of sin(kx) is
    sin(k) cos(kx), so the discrete vorticity is exactly
    2 U sin(k) sin(kx) sin(ky), giving <omega^2>_D = 4 U^2 sin(k)^2 / 2 *
    <sin^2 ky>_rows(D), and E_k = U^2 / 4 exactly."""
    U, trim = 0.02, 3
    k = 2 * np.pi * n / N
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    ux = U * np.sin(k * x) * np.cos(k * y)
    uy = -U * np.cos(k * x) * np.sin(k * y)
    p = orc.Params(nx=N, ny=N, tau=(1.0, 1.0), periodic_y=True)
    f = orc.fill_equilibrium(p, np.full((N, N), 0.5), np.full((N, N), 0.5), ux, uy)
    d = orc.diagnostics(p, f, trim=trim)
    rows = np.arange(trim, N - trim)
    s2y = np.mean(np.sin(k * rows) ** 2)
    assert d["omega2"] == pytest.approx(4 * U * U * np.sin(k) ** 2 * 0.5 * s2y, rel=1e-12)
    assert d["Ek"] == pytest.approx(U * U / 4, rel=1e-12)
    assert d["umax"] <= U * (1 + 1e-12)
    assert d["finite"]


@pytest.mark.parametrize("U,V", [(0.03, -0.07), (-0.05, 0.02)])
def test_max_speed_of_a_uniform_flow(orc, U, V):
    """A uniform flow u = (U, V) of a uniform mixture (G = 0, g = 0, so
    u_phys = u): max |u| over the lattice is the speed hypot(U, V), larger
    than either component, and E_k = rho |u|^2 / 2."""
    nx, ny = 12, 30
    p = orc.Params(nx=nx, ny=ny, tau=(0.9, 0.9), periodic_y=True)
    f = orc.fill_equilibrium(p, np.full((ny, nx), 0.6), np.full((ny, nx), 0.45),
                             np.full((ny, nx), U), np.full((ny, nx), V))
    d = orc.diagnostics(p, f, trim=5)
    speed = float(np.hypot(U, V))
    assert d["umax"] == pytest.approx(speed, rel=1e-14)
    assert d["umax"] > max(abs(U), abs(V)) * 1.05
    assert d["Ek"] == pytest.approx(0.5 * 1.05 * speed * speed, rel=1e-13)


def test_max_speed_finds_the_fastest_site(orc):
    """One site moving at (U, V) in a fluid at rest, placed in a trimmed row:
    max |u| runs over the whole lattice, not only the trimmed domain."""
    nx, ny = 10, 26
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    ux[1, 7], uy[1, 7] = -0.02, 0.09
    ux[13, 3] = 0.05
    p = orc.Params(nx=nx, ny=ny, tau=(1.0, 1.0), periodic_y=True)
    f = orc.fill_equilibrium(p, np.full((ny, nx), 0.5), np.full((ny, nx), 0.5), ux, uy)
    d = orc.diagnostics(p, f, trim=5)
    assert d["umax"] == pytest.approx(float(np.hypot(0.02, 0.09)), rel=1e-14)


def test_diagnostics_flag_non_finite(orc):
    p = orc.Params(nx=8, ny=30, tau=(1.0, 1.0))
    f = orc.fill_equilibrium(p, np.ones((30, 8)), np.ones((30, 8)))
    f[1, 3, 15, 2] = np.nan
    assert not orc.diagnostics(p, f, trim=10)["finite"]


def test_streaming_direction_by_advection(orc):
    """A composition wave phi ~ cos(k x) carried by a uniform flow U e_x
    (G = 0, uniform total density) moves with the flow: after t steps its
    Fourier phase has advanced by -k U t (convention phi ~ cos(k(x - U t))).
    Pushing populations the wrong way would reverse the shift."""
    nx, ny, U, t = 64, 4, 0.05, 200
    k = 2 * np.pi / nx
    x = np.arange(nx, dtype=np.float64)[None, :].repeat(ny, 0)
    rA = 0.5 + 1e-3 * np.cos(k * x)
    rB = 0.5 - 1e-3 * np.cos(k * x)
    p = orc.Params(nx=nx, ny=ny, tau=(0.8, 0.8), periodic_y=True)
    f = orc.fill_equilibrium(p, rA, rB, np.full((ny, nx), U), np.zeros((ny, nx)))
    f = orc.run(p, f, t)
    m = orc.macro(p, f)
    phi = (m["rhoA"] - m["rhoB"])[0]
    phase = np.angle(np.sum(phi * np.exp(-1j * k * np.arange(nx))))
    assert phase == pytest.approx(-k * U * t, abs=0.01 * k * U * t)
