"""Pins of the 3D (D3Q19) oracle, oracle/orc3.c.

* Lattice: 19 distinct velocities with |c|^2 <= 2 closed under reversal;
  the weights satisfy the isotropy conditions of Eq. 4 with c_s^2 = 1/3
  exactly (rational arithmetic), up to fourth order.
* Projections: summing D3Q19 over the velocity component along an axis
  gives D2Q9 with its weights, so a 3D state that does not vary along that
  axis evolves exactly like the 2D model.  For each of the three axes the
  3D oracle reproduces the (separately pinned) 2D oracle's densities and
  velocities to rounding, with walls or periodic y, gravity, G != 0 and
  tau_A != tau_B; the velocity along the invariant axis stays zero.
* Conservation on a fully 3D state: component masses to rounding between
  walls, and the total momentum gains exactly sum_s M_s g_s per step in a
  periodic box (the Shan-Chen forces cancel pairwise).
"""
from fractions import Fraction
from itertools import product

import numpy as np
import pytest

import oracle
from oracle import lb3


def test_velocity_set_and_isotropy():
    cx, cy, cz, opp, w = lb3.constants()
    c = np.stack([cx, cy, cz], axis=1)
    assert len({tuple(v) for v in c}) == 19
    assert all(int(v @ v) <= 2 for v in c)
    assert all((c[opp[i]] == -c[i]).all() for i in range(19))
    # the weights as exact rationals of the three shells
    frac = {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)}
    wf = [frac[int(v @ v)] for v in c]
    assert np.array_equal(w, np.array([float(x) for x in wf]))
    cs2 = Fraction(1, 3)
    assert sum(wf) == 1
    for a, b in product(range(3), repeat=2):
        assert sum(wi * int(v[a]) for wi, v in zip(wf, c)) == 0
        assert sum(wi * int(v[a] * v[b]) for wi, v in zip(wf, c)) == (cs2 if a == b else 0)
        for d in range(3):
            assert sum(wi * int(v[a] * v[b] * v[d]) for wi, v in zip(wf, c)) == 0
    for a, b, d, e in product(range(3), repeat=4):
        got = sum(wi * int(v[a] * v[b] * v[d] * v[e]) for wi, v in zip(wf, c))
        want = cs2 * cs2 * ((a == b) * (d == e) + (a == d) * (b == e) + (a == e) * (b == d))
        assert got == want, (a, b, d, e)


def _fields2d(n1, n2, seed):
    """Smooth two-phase pattern on an n1 x n2 plane (axis 0 length n1)."""
    rng = np.random.default_rng(seed)
    i = np.arange(n1)[:, None]
    j = np.arange(n2)[None, :]
    h = n1 / 2 + 2.0 * np.cos(2 * np.pi * j / n2 + rng.uniform(0, 6)) + 1.0 * np.sin(4 * np.pi * j / n2)
    s = 0.5 * (1 + np.tanh((i - h) / 1.5))
    return 0.06 + 1.0 * s, 0.06 + 0.9 * (1 - s)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


STEPS = 150


def test_z_invariant_state_is_the_2d_model_with_walls():
    nx, ny, nz = 24, 20, 3
    rA2, rB2 = _fields2d(ny, nx, 1)                      # [y][x]
    tau, G, g = (1.0, 0.8), 1.2, 2e-4
    p2 = oracle.Params(nx=nx, ny=ny, tau=tau, G=G, g=((1e-5, -g), (0.0, g)))
    m2 = oracle.macro(p2, oracle.run(p2, oracle.fill_equilibrium(p2, rA2, rB2), STEPS))
    p3 = lb3.Params3(nx=nx, ny=ny, nz=nz, tau=tau, G=G, g=((1e-5, -g, 0.0), (0.0, g, 0.0)))
    rA3 = np.broadcast_to(rA2, (nz, ny, nx)).copy()
    rB3 = np.broadcast_to(rB2, (nz, ny, nx)).copy()
    m3 = lb3.macro(p3, lb3.run(p3, lb3.fill_equilibrium(p3, rA3, rB3), STEPS))
    for z in range(nz):
        for k in ("rhoA", "rhoB", "ux", "uy"):
            assert _rel(m3[k][z], m2[k]) < 1e-12, (k, z, _rel(m3[k][z], m2[k]))
    assert np.max(np.abs(m3["uz"])) < 1e-15
    assert np.max(np.abs(m2["uy"])) > 1e-5          # the run is not trivial


def test_x_invariant_state_is_the_2d_model_in_the_zy_plane():
    nx, ny, nz = 3, 22, 18
    rA2, rB2 = _fields2d(ny, nz, 2)                      # [y][z]
    tau, G, g = (0.9, 0.9), 1.1, 2e-4
    # 2D oracle with x2 := z, y2 := y, periodic y2
    p2 = oracle.Params(nx=nz, ny=ny, tau=tau, G=G, g=((3e-5, -g), (0.0, g)), periodic_y=True)
    m2 = oracle.macro(p2, oracle.run(p2, oracle.fill_equilibrium(p2, rA2, rB2), STEPS))
    p3 = lb3.Params3(nx=nx, ny=ny, nz=nz, tau=tau, G=G, g=((0.0, -g, 3e-5), (0.0, g, 0.0)), periodic_y=True)
    rA3 = np.broadcast_to(rA2.T[:, :, None], (nz, ny, nx)).copy()
    rB3 = np.broadcast_to(rB2.T[:, :, None], (nz, ny, nx)).copy()
    m3 = lb3.macro(p3, lb3.run(p3, lb3.fill_equilibrium(p3, rA3, rB3), STEPS))
    for x in range(nx):
        assert _rel(m3["rhoA"][:, :, x].T, m2["rhoA"]) < 1e-12
        assert _rel(m3["rhoB"][:, :, x].T, m2["rhoB"]) < 1e-12
        assert _rel(m3["uy"][:, :, x].T, m2["uy"]) < 1e-12
        assert _rel(m3["uz"][:, :, x].T, m2["ux"]) < 1e-12
    assert np.max(np.abs(m3["ux"])) < 1e-15


def test_y_invariant_state_is_the_2d_model_in_the_xz_plane():
    nx, ny, nz = 20, 3, 16
    rA2, rB2 = _fields2d(nz, nx, 3)                      # [z][x]
    tau, G = (1.0, 0.7), 1.3
    # 2D oracle with (x2, y2) := (x, z); accelerations in the plane
    p2 = oracle.Params(nx=nx, ny=nz, tau=tau, G=G, g=((2e-4, 1e-4), (-2e-4, 0.0)), periodic_y=True)
    m2 = oracle.macro(p2, oracle.run(p2, oracle.fill_equilibrium(p2, rA2, rB2), STEPS))
    p3 = lb3.Params3(nx=nx, ny=ny, nz=nz, tau=tau, G=G, g=((2e-4, 0.0, 1e-4), (-2e-4, 0.0, 0.0)), periodic_y=True)
    rA3 = np.broadcast_to(rA2[:, None, :], (nz, ny, nx)).copy()
    rB3 = np.broadcast_to(rB2[:, None, :], (nz, ny, nx)).copy()
    m3 = lb3.macro(p3, lb3.run(p3, lb3.fill_equilibrium(p3, rA3, rB3), STEPS))
    for y in range(ny):
        assert _rel(m3["rhoA"][:, y, :], m2["rhoA"]) < 1e-12
        assert _rel(m3["ux"][:, y, :], m2["ux"]) < 1e-12
        assert _rel(m3["uz"][:, y, :], m2["uy"]) < 1e-12
    assert np.max(np.abs(m3["uy"])) < 1e-15


def _blob(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = np.sqrt((x - nx / 2 + 0.3) ** 2 + (y - ny / 2 + 0.7) ** 2 + (z - nz / 2 - 0.4) ** 2) - 4.0
    s = 0.5 * (1 - np.tanh(d / 1.5))
    return 0.06 + s, 0.06 + (1 - s)


def test_mass_conserved_between_walls():
    nx, ny, nz = 14, 12, 10
    rA, rB = _blob(nx, ny, nz)
    p = lb3.Params3(nx=nx, ny=ny, nz=nz, tau=(1.0, 0.8), G=1.4, g=((0.0, -1e-3, 2e-4), (1e-4, 1e-3, 0.0)))
    f0 = lb3.fill_equilibrium(p, rA, rB)
    f = lb3.run(p, f0, 300)
    m = lb3.macro(p, f)
    for key, r0 in (("rhoA", rA), ("rhoB", rB)):
        assert abs(m[key].sum() / r0.sum() - 1) < 1e-13
    assert np.max(np.abs(m["uy"])) > 1e-5


def test_momentum_gain_equals_total_body_force():
    nx, ny, nz = 12, 10, 8
    rA, rB = _blob(nx, ny, nz)
    g = ((2e-4, -1e-3, 5e-4), (-1e-4, 1e-3, 3e-4))
    p = lb3.Params3(nx=nx, ny=ny, nz=nz, tau=(1.0, 0.7), G=1.5, g=g, periodic_y=True)
    f = lb3.run(p, lb3.fill_equilibrium(p, rA, rB), 20)
    cx, cy, cz, _o, _w = lb3.constants()

    def momentum(f):
        tot = f.sum(axis=0)                              # [i][z][y][x]
        return np.array([np.tensordot(c, tot.reshape(19, -1).sum(axis=1), axes=1) for c in (cx, cy, cz)])

    M = [f[s].sum() for s in range(2)]
    want = np.array([M[0] * g[0][d] + M[1] * g[1][d] for d in range(3)])
    for _ in range(5):
        f1 = lb3.run(p, f, 1)
        got = momentum(f1) - momentum(f)
        assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want)) * 10 + 1e-15, (got, want)
        f = f1


def test_trivial_lattice_rejects_nothing_and_stays_at_rest():
    p = lb3.Params3(nx=3, ny=3, nz=3, tau=(1.0, 1.0), G=0.5)
    r = np.full((3, 3, 3), 0.5)
    m = lb3.macro(p, lb3.run(p, lb3.fill_equilibrium(p, r, r), 10))
    assert np.max(np.abs(m["ux"])) == 0.0 and np.max(np.abs(m["rhoA"] - 0.5)) < 1e-15
