"""GPU (gfx950) parity of wetting walls against the FP64 CPU oracle: the
fluid-boundary force of Eq. 6 (G_Ab, G_Bb != 0 on the wall rows) and psi on
the boundary nodes in Eq. 5 (the wall row's, or zero).

Drops of A sit on both walls (so both wall rows carry the force and the
contact lines move), on a lattice that is ragged for every tile width.  Both
passes (one and two steps per kernel pass), both forcing schemes and both
psi readings must match the oracle to 1e-12 relative in FP64, and so must
the field pass (whose velocity includes half the wall force).  A member with
neutral walls in an ensemble whose other member has wetting walls runs the
wetting kernels and must still equal its solo run with the neutral kernels
bit for bit.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def lb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2101_04847_amd import lb as mod
    return mod


def _say(*a):
    print("[case]", *a, flush=True)


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


def _drops(nx, ny):
    """A drops of radius 9 centred on the bottom wall (x = nx/3) and on the
    top wall (x = 2 nx/3), in B; trace 0.06."""
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    d = np.minimum(np.hypot(x - nx / 3, y + 0.5), np.hypot(x - 2 * nx / 3, y - (ny - 0.5))) - 9.0
    s = 0.5 * (1.0 - np.tanh(d / 1.5))
    return 0.06 + s, 0.06 + (1.0 - s)


def _member(lb, nx, ny, *, tau, G_wall, wall_psi, g=1e-5):
    rA, rB = _drops(nx, ny)
    return lb.Member(nx, ny, rA, rB, tau=tau, G=1.6, g=((0.0, -g), (0.0, g)), G_wall=G_wall, wall_psi=wall_psi)


def _params(m, forcing):
    return oracle.Params(nx=m.nx, ny=m.ny, tau=m.tau, G=m.G, g=m.g, forcing=forcing, G_wall=m.G_wall,
                         wall_psi=m.wall_psi)


CASES = [
    # forcing, steps per pass, wall_psi, G_wall, tau
    (0, 1, 0, (0.12, -0.08), (1.0, 0.8)),
    (0, 2, 0, (0.12, -0.08), (1.0, 0.8)),
    (1, 1, 0, (-0.1, 0.05), (0.9, 0.9)),
    (1, 2, 0, (-0.1, 0.05), (0.9, 0.9)),
    (0, 1, 1, (0.0, 0.0), (1.0, 1.0)),
    (0, 2, 1, (0.0, 0.0), (1.0, 1.0)),
    (0, 1, 1, (0.3, 0.05), (0.7, 0.7)),
    (0, 2, 1, (0.3, 0.05), (0.7, 0.7)),
    (1, 2, 1, (0.15, -0.15), (1.0, 1.0)),
]


@pytest.mark.parametrize("forcing,spp,wall_psi,G_wall,tau", CASES)
def test_wetting_walls_match_oracle(lb, forcing, spp, wall_psi, G_wall, tau):
    nx, ny = 131, 37
    _say("wetting", "forcing", forcing, "spp", spp, "wall_psi", wall_psi, "G_wall", G_wall, "tau", tau)
    m = _member(lb, nx, ny, tau=tau, G_wall=G_wall, wall_psi=wall_psi)
    lat = lb.Lattice([m], forcing=forcing, storage=lb.F64, tile_x=64, tile_h=7 if spp == 2 else 5,
                     graph_chunk=10, poison=True, steps_per_pass=spp, diag_trim=2)
    p = _params(m, forcing)
    f = oracle.fill_equilibrium(p, m.rhoA0, m.rhoB0)
    t = 0
    for target in (1, 30, 101):
        f = oracle.run(p, f, target - t)
        lat.step(target - t)
        t = target
        err = _rel(lat.get_populations(0).cpu().numpy(), f)
        assert err <= TOL, (target, err)
    mg = {k: v.cpu().numpy() for k, v in lat.fields(0).items()}
    mo = oracle.macro(p, f)
    for k in ("rhoA", "rhoB", "ux", "uy"):
        assert _rel(mg[k], mo[k]) <= TOL, k
    # the wall terms matter here: the state differs from that of neutral walls
    if G_wall != (0.0, 0.0) or wall_psi:
        pn = oracle.Params(nx=nx, ny=ny, tau=tau, G=m.G, g=m.g, forcing=forcing)
        fn = oracle.run(pn, oracle.fill_equilibrium(pn, m.rhoA0, m.rhoB0), 101)
        assert _rel(fn, f) > 1e-6
    lat.close()


@pytest.mark.parametrize("spp", [1, 2])
def test_neutral_member_unchanged_by_wetting_kernels(lb, spp):
    nx, ny = 96, 40
    _say("neutral member beside a wetting member, spp", spp)
    wet = _member(lb, 70, 33, tau=(1.0, 1.0), G_wall=(0.1, -0.1), wall_psi=1)
    neutral = _member(lb, nx, ny, tau=(1.0, 1.0), G_wall=(0.0, 0.0), wall_psi=0)
    kw = dict(storage=lb.F64, tile_x=64, tile_h=8, graph_chunk=20, poison=True, steps_per_pass=spp, diag_trim=2)
    both = lb.Lattice([wet, neutral], **kw)
    solo = lb.Lattice([neutral], **kw)
    both.step(61)
    solo.step(61)
    a = both.get_populations(1).cpu().numpy()
    b = solo.get_populations(0).cpu().numpy()
    assert np.array_equal(a, b)
    p = _params(wet, 0)
    f = oracle.run(p, oracle.fill_equilibrium(p, wet.rhoA0, wet.rhoB0), 61)
    assert _rel(both.get_populations(0).cpu().numpy(), f) <= TOL
    both.close()
    solo.close()


def test_wetting_f32_close_to_oracle(lb):
    """FP32 storage with wetting walls follows the FP64 oracle within the
    bound of the neutral case (5e-7 after one step, 2e-5 after 100)."""
    nx, ny = 131, 37
    _say("wetting f32")
    m = _member(lb, nx, ny, tau=(1.0, 1.0), G_wall=(0.12, -0.08), wall_psi=1)
    lat = lb.Lattice([m], storage=lb.F32, tile_x=64, tile_h=5, graph_chunk=10, steps_per_pass=1, diag_trim=2)
    p = _params(m, 0)
    f = oracle.fill_equilibrium(p, m.rhoA0, m.rhoB0)
    t = 0
    for target, tol in ((1, 5e-7), (100, 2e-5)):
        f = oracle.run(p, f, target - t)
        lat.step(target - t)
        t = target
        mg = {k: v.cpu().numpy() for k, v in lat.fields(0).items()}
        mo = oracle.macro(p, f)
        for k in ("rhoA", "rhoB"):
            assert _rel(mg[k], mo[k]) <= tol, (target, k, _rel(mg[k], mo[k]))
    lat.close()
