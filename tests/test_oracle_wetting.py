"""Pins of the oracle's wall terms: the fluid-boundary force of Eq. 6 and
the two readings of psi on boundary nodes in Eq. 5.

* Brute force: on tiny random states, the total force F_A + F_B that the
  oracle reports equals Eq. 5 + Eq. 6 + Eq. 7 evaluated on a lattice padded
  with explicit boundary rows (S = 1 there, psi mirrored or zero), with the
  D2Q9 set typed here from Sec. 2.
* Cancellation: with psi = 0 on boundary nodes, a uniform mixture at rest
  feels -G rho_sbar / 6 towards each wall from Eq. 5; G_sb = G rho_sbar in
  Eq. 6 cancels it exactly, so the state stays at rest, while G_sb = 0 or
  the opposite sign drives a flow.
* Wetting: a drop of A on the bottom wall spreads wider when the wall
  attracts A (G_Ab < G_Bb) than when it repels it.
"""
import numpy as np
import pytest

import oracle

# D2Q9 of Sec. 2: rest, four axis links (weight 1/9), four diagonals (1/36)
C = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
WT = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4


def _brute_total_force(rhoA, rhoB, G, Gw, g, wall_psi, periodic):
    ny, nx = rhoA.shape
    rho = [rhoA, rhoB]
    # padded lattice: row 0 and row ny + 1 are the boundary nodes
    S = np.zeros((ny + 2, nx))
    psi = []
    for r in rho:
        pp = np.zeros((ny + 2, nx))
        pp[1:-1] = r
        if periodic:
            pp[0], pp[-1] = r[-1], r[0]
        else:
            S[0] = S[-1] = 1.0
            if wall_psi == oracle.PSI_MIRROR:
                pp[0], pp[-1] = r[0], r[-1]
        psi.append(pp)
    Fx = np.zeros((ny, nx))
    Fy = np.zeros((ny, nx))
    for s in range(2):
        for y in range(ny):
            for x in range(nx):
                fx = fy = 0.0
                for (cx, cy), w in zip(C, WT):
                    yy, xx = y + 1 + cy, (x + cx) % nx
                    fx += -G * rho[s][y, x] * w * psi[1 - s][yy, xx] * cx
                    fy += -G * rho[s][y, x] * w * psi[1 - s][yy, xx] * cy
                    fx += -Gw[s] * rho[s][y, x] * w * S[yy, xx] * cx
                    fy += -Gw[s] * rho[s][y, x] * w * S[yy, xx] * cy
                Fx[y, x] += fx + rho[s][y, x] * g[s][0]
                Fy[y, x] += fy + rho[s][y, x] * g[s][1]
    return Fx, Fy


@pytest.mark.parametrize("wall_psi", [oracle.PSI_MIRROR, oracle.PSI_ZERO])
@pytest.mark.parametrize("periodic", [False, True])
def test_total_force_equals_brute_force(wall_psi, periodic):
    rng = np.random.default_rng(11 + wall_psi + 2 * periodic)
    nx, ny = 7, 6
    G, Gw = 0.9, (0.35, -0.2)
    g = ((0.0, -1e-3), (2e-4, 1e-3))
    f = rng.uniform(0.02, 0.2, size=(2, 9, ny, nx))
    p = oracle.Params(nx=nx, ny=ny, G=G, g=g, G_wall=Gw, wall_psi=wall_psi, periodic_y=periodic)
    m = oracle.macro(p, f)
    rA, rB = f[0].sum(axis=0), f[1].sum(axis=0)
    Fx, Fy = _brute_total_force(rA, rB, G, Gw, g, wall_psi, periodic)
    scale = np.abs(Fy).max()
    assert np.max(np.abs(m["Fx"] - Fx)) <= 1e-14 * scale
    assert np.max(np.abs(m["Fy"] - Fy)) <= 1e-14 * scale
    if not periodic:
        # the wall term is not zero on the wall rows (the check above sees it)
        Fx0, Fy0 = _brute_total_force(rA, rB, G, (0.0, 0.0), g, wall_psi, periodic)
        assert np.max(np.abs(Fy0[0] - Fy[0])) > 1e-3 * scale


def _uniform_run(Gw, steps=40):
    nx, ny, G = 8, 10, 1.2
    rA, rB = np.full((ny, nx), 0.7), np.full((ny, nx), 0.3)
    p = oracle.Params(nx=nx, ny=ny, G=G, G_wall=Gw, wall_psi=oracle.PSI_ZERO)
    f = oracle.run(p, oracle.fill_equilibrium(p, rA, rB), steps)
    m = oracle.macro(p, f)
    return max(np.abs(m["ux"]).max(), np.abs(m["uy"]).max()), m


def test_zero_psi_wall_pull_cancelled_by_eq6():
    G = 1.2
    umax, m = _uniform_run((G * 0.3, G * 0.7))
    assert umax < 1e-14, umax
    assert np.max(np.abs(m["rhoA"] - 0.7)) < 1e-14
    for Gw in ((0.0, 0.0), (-G * 0.3, -G * 0.7)):
        umax, _ = _uniform_run(Gw)
        assert umax > 1e-4, (Gw, umax)


def _drop_base(Gw):
    """Width of the A drop's contact line on the bottom wall."""
    nx, ny, R = 64, 32, 10.0
    x = np.arange(nx)[None, :] - nx / 2 + 0.5
    y = np.arange(ny)[:, None] + 0.0
    d = np.hypot(x, y) - R
    s = 0.5 * (1 - np.tanh(d / 1.5))
    rA, rB = 0.05 + 1.0 * s, 0.05 + 1.0 * (1 - s)
    p = oracle.Params(nx=nx, ny=ny, G=1.6, G_wall=Gw)
    m = oracle.macro(p, oracle.run(p, oracle.fill_equilibrium(p, rA, rB), 3000))
    return int(np.count_nonzero(m["rhoA"][0] > m["rhoB"][0])), m


def test_wetting_walls_order_contact_line():
    base_wet, _ = _drop_base((-0.15, 0.15))
    base_neutral, _ = _drop_base((0.0, 0.0))
    base_dry, _ = _drop_base((0.15, -0.15))
    assert base_wet > base_neutral > base_dry, (base_wet, base_neutral, base_dry)
