"""GPU (gfx950) parity of the three-step pass (three time steps fused per
kernel pass, steps_per_pass = 3) against the single-step pass and the FP64
CPU oracle.

The fused pass evaluates every site with the same arithmetic as the single
step and keeps the results of its first two steps in the stored form, so in
every storage mode it must reproduce single steps bit for bit: both forcing
schemes, both wall modes and wetting walls, ragged bands and tiles, lattices
narrower than a wave, remainders of one and two steps (a two-step pass) and
graph chunks, and an ensemble of uneven members.  In FP64 it must match the
oracle to 1e-12 relative on the 128 x 64 parity workload over 1000 steps.
"""
import numpy as np
import pytest

import oracle
from paper_2101_04847_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2101_04847_amd import lb as mod
    return mod


def _say(*a):
    print("[case]", *a, flush=True)


ST = {"f64": 0, "f32": 1, "f16s": 2, "bf16s": 3}


def _member(lb, nx, ny, *, G=1.5, g=1e-4, tau=(1.0, 1.0), seed=3, **kw):
    rA, rB = inputs.multi_mode(nx, ny, seed)
    return lb.Member(nx, ny, rA, rB, tau=tau, G=G, g=((0.0, -g), (0.0, g)), **kw)


def _pair(lb, members, storage, *, band, chunk3=-1, forcing=0, bc=0):
    """The same members with single steps and with the three-step pass."""
    ny = min(m.ny for m in members)
    kw = dict(forcing=forcing, storage=storage, bc_y=bc, poison=True, diag_trim=max(1, min(10, (ny - 1) // 2 - 1)))
    one = lb.Lattice(members, tile_x=64, tile_h=16, graph_chunk=-1, steps_per_pass=1, **kw)
    three = lb.Lattice(members, tile_x=64, tile_h=band, graph_chunk=chunk3, steps_per_pass=3, **kw)
    assert three.steps_per_pass == 3 and three.tile_shape() == (54, min(band, ny))
    return one, three


def _same(one, three, k=0):
    return np.array_equal(one.get_populations(k).cpu().numpy(), three.get_populations(k).cpu().numpy())


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s"])
@pytest.mark.parametrize("forcing", [0, 1], ids=["shift", "guo"])
@pytest.mark.parametrize("bc", [0, 1], ids=["walls", "periodic_y"])
def test_three_step_equals_single_step(lb, storage, forcing, bc):
    _say("three-step vs single-step", storage, "guo" if forcing else "shift", "periodic_y" if bc else "walls")
    m = _member(lb, 190, 70, seed=9)
    one, three = _pair(lb, [m], ST[storage], band=24, chunk3=8, forcing=forcing, bc=bc)
    # 3: one pass; 5: a pass and a two-step pass; 7: two passes and a single
    # step; 31: graph replays (8 steps: two passes and a two-step pass) and
    # eager remainders
    for n in (3, 5, 7, 31):
        one.step(n)
        three.step(n)
        assert _same(one, three), n
    one.close()
    three.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16s"])
@pytest.mark.parametrize("bc", [0, 1], ids=["walls", "periodic_y"])
def test_three_step_ragged_bands_and_narrow_lattices(lb, storage, bc):
    """Bands of 1 to 9 rows (march lengths of every parity, a ragged last
    band), a ragged last window, and lattices narrower than the 54-column
    window (the columns wrap inside one wave)."""
    for nx, ny in ((130, 23), (20, 17), (57, 9)):
        for band in (1, 2, 3, 5, 9):
            _say("three-step ragged", storage, "periodic_y" if bc else "walls", nx, ny, "band", band)
            m = _member(lb, nx, ny, seed=5, G=1.2)
            one, three = _pair(lb, [m], ST[storage], band=band, bc=bc)
            for n in (3, 4, 6):
                one.step(n)
                three.step(n)
                assert _same(one, three), (nx, ny, band, n)
            one.close()
            three.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16s"])
@pytest.mark.parametrize("band", [228, 455])
def test_three_step_tall_bands(lb, storage, band):
    """Bands as tall as the timing search picks at 10000 x 5000 (the heights
    that fill whole rounds of the wave slots), on a lattice of 1000 rows: a
    march of band + 10 rows per work item, and a ragged last band."""
    _say("three-step tall band", storage, band)
    m = _member(lb, 130, 1000, seed=7, G=1.3)
    one, three = _pair(lb, [m], ST[storage], band=band, chunk3=6)
    for n in (3, 7, 12):
        one.step(n)
        three.step(n)
        assert _same(one, three), (band, n)
    one.close()
    three.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("forcing", [0, 1], ids=["shift", "guo"])
@pytest.mark.parametrize("wall_psi,G_wall", [(0, (0.12, -0.08)), (1, (0.3, 0.05))], ids=["mirror", "zero"])
def test_three_step_wetting_walls(lb, storage, forcing, wall_psi, G_wall):
    """The wetting-wall kernels (Eq. 6 force on the wall rows, psi of the
    boundary nodes in Eq. 5) with unequal relaxation times under the shift
    scheme."""
    _say("three-step wetting", storage, "guo" if forcing else "shift", "wall_psi", wall_psi, "G_wall", G_wall)
    tau = (1.0, 1.0) if forcing else (1.0, 0.8)
    m = _member(lb, 131, 37, seed=6, G=1.6, tau=tau, G_wall=G_wall, wall_psi=wall_psi)
    one, three = _pair(lb, [m], ST[storage], band=7, chunk3=10, forcing=forcing)
    for n in (3, 20, 41):
        one.step(n)
        three.step(n)
        assert _same(one, three), n
    one.close()
    three.close()


def test_three_step_ensemble_equals_solo(lb):
    """One three-step launch over uneven members gives each member its solo
    result, and each solo result its single-step result."""
    _say("three-step ensemble vs solo")
    specs = [(96, 40, 0.5, 3), (160, 64, 1.5, 4), (64, 24, 1.5, 5)]
    members = [_member(lb, nx, ny, G=G, seed=seed) for nx, ny, G, seed in specs]
    kw = dict(storage=lb.F32, tile_x=64, tile_h=16, graph_chunk=6, poison=True, steps_per_pass=3, diag_trim=2)
    ens = lb.Lattice(members, **kw)
    ens.step(30)
    for k, m in enumerate(members):
        one, solo = _pair(lb, [m], lb.F32, band=16, chunk3=6)
        solo.step(30)
        one.step(30)
        assert np.array_equal(ens.get_populations(k).cpu().numpy(), solo.get_populations(0).cpu().numpy()), k
        assert _same(one, solo), k
        one.close()
        solo.close()
    ens.close()


def test_three_step_f32_close_to_oracle(lb):
    """FP32 storage through the three-step pass follows the FP64 oracle on
    the 128 x 64 Rayleigh-Taylor workload within the FP32 bound of the
    single-step pass (5e-7 relative density error after one pass, 2e-5
    after 99 steps)."""
    _say("three-step f32 vs oracle")
    rA, rB = inputs.single_mode(128, 64, 2.0)
    m = lb.Member(128, 64, rA, rB, tau=(1.0, 1.0), G=1.5, g=((0.0, -1e-5), (0.0, 1e-5)))
    lat = lb.Lattice([m], storage=lb.F32, tile_h=12, graph_chunk=-1, steps_per_pass=3, diag_trim=10)
    p = oracle.Params(nx=128, ny=64, tau=m.tau, G=m.G, g=m.g)
    f = oracle.fill_equilibrium(p, rA, rB)
    t = 0
    for target, tol in ((3, 5e-7), (99, 2e-5)):
        f = oracle.run(p, f, target - t)
        lat.step(target - t)
        t = target
        mg = {k: v.cpu().numpy() for k, v in lat.fields(0).items()}
        mo = oracle.macro(p, f)
        for k in ("rhoA", "rhoB"):
            err = float(np.max(np.abs(mg[k] - mo[k])) / np.max(np.abs(mo[k])))
            assert err <= tol, (target, k, err)
    lat.close()


@pytest.mark.parametrize("forcing", [1, 0], ids=["guo", "shift"])
def test_three_step_f64_rt_128x64_1000_steps(lb, forcing):
    """The 128 x 64 Rayleigh-Taylor parity workload through the FP64
    three-step pass at steps 1, 3, 10, 100 and 1000 (remainders take a
    two-step pass and single steps; 99-step graphs of 33 passes)."""
    _say("three-step f64 rt 128x64", "guo" if forcing else "shift")
    rA, rB = inputs.single_mode(128, 64, 2.0)
    m = lb.Member(128, 64, rA, rB, tau=(1.0, 1.0), G=1.5, g=((0.0, -1e-5), (0.0, 1e-5)))
    lat = lb.Lattice([m], forcing=forcing, storage=lb.F64, tile_h=16, graph_chunk=99 - 99 % 2,
                     steps_per_pass=3, poison=True, diag_trim=10)
    assert lat.steps_per_pass == 3
    p = oracle.Params(nx=128, ny=64, tau=m.tau, G=m.G, g=m.g, forcing=forcing)
    f = oracle.fill_equilibrium(p, rA, rB)
    t = 0
    for target in (1, 3, 10, 100, 1000):
        f = oracle.run(p, f, target - t)
        lat.step(target - t)
        t = target
        got = lat.get_populations(0).cpu().numpy()
        err = float(np.max(np.abs(got - f)) / np.max(np.abs(f)))
        assert err <= 1e-12, (target, err)
    lat.close()
