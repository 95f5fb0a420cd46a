"""GPU (gfx950) parity of the two-step pass (two time steps fused per kernel
pass, steps_per_pass = 2) against the FP64 CPU oracle and against the
single-step pass.

The fused pass evaluates every site with the same arithmetic as the single
step, so in FP64 it must match the oracle to 1e-12 relative (usually bit for
bit) and, in every storage mode, the single-step pass bit for bit.  Odd step
counts end with one single step; graph chunks may hold an odd number of
passes (the buffer parity then changes per replay).
"""
import numpy as np
import pytest

import oracle
from paper_2101_04847_amd import inputs

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


def _member(lb, nx, ny, *, G=1.5, g=1e-5, tau=(1.0, 1.0), seed=None, amp=2.0):
    if seed is None:
        rA, rB = inputs.single_mode(nx, ny, amp)
    else:
        rA, rB = inputs.multi_mode(nx, ny, seed)
    return lb.Member(nx, ny, rA, rB, tau=tau, G=G, g=((0.0, -g), (0.0, g)))


def _lattice(lb, members, *, spp=2, band=0, chunk=0, forcing=0, bc=0, storage=None, tile=(64, 16)):
    ny = min(m.ny for m in members)
    return lb.Lattice(members, forcing=forcing, storage=lb.F64 if storage is None else storage, bc_y=bc,
                      tile_x=tile[0], tile_h=band if spp == 2 else tile[1], graph_chunk=chunk, poison=True,
                      steps_per_pass=spp, diag_trim=max(1, min(10, (ny - 1) // 2 - 1)))


def _params(m, forcing=0, bc=0):
    return oracle.Params(nx=m.nx, ny=m.ny, tau=m.tau, G=m.G, g=m.g, forcing=forcing, periodic_y=bool(bc))


@pytest.mark.parametrize("forcing", [1, 0], ids=["guo", "shift"])
def test_two_step_rt_128x64_1000_steps(lb, forcing):
    """The 128 x 64 Rayleigh-Taylor parity workload at steps 1, 10, 100 and
    1000 (odd counts end with a single step; 100-step graphs of 50 passes)."""
    _say("two-step rt 128x64", "guo" if forcing else "shift")
    m = _member(lb, 128, 64)
    lat = _lattice(lb, [m], band=16, forcing=forcing)
    assert lat.steps_per_pass == 2 and lat.tile_shape() == (58, 16)
    p = _params(m, forcing)
    f = oracle.fill_equilibrium(p, m.rhoA0, m.rhoB0)
    t = 0
    exact = True
    for target in (1, 10, 100, 1000):
        f = oracle.run(p, f, target - t)
        lat.step(target - t)
        t = target
        err = _rel(lat.get_populations(0).cpu().numpy(), f)
        exact &= err == 0.0
        assert err <= TOL, (target, err)
        mg = {k: v.cpu().numpy() for k, v in lat.fields(0).items()}
        mo = oracle.macro(p, f)
        for k in ("rhoA", "rhoB", "ux", "uy"):
            assert _rel(mg[k], mo[k]) <= TOL, (target, k)
    print(f"bit-exact at every checkpoint: {exact}", flush=True)
    lat.close()


CASES = [
    # nx, ny, bc, forcing, band, tau
    (67, 13, 0, 0, 5, (1.0, 1.0)),
    (67, 13, 1, 1, 4, (0.8, 0.8)),
    (130, 23, 0, 1, 7, (0.7, 0.7)),
    (130, 23, 1, 0, 32, (1.0, 0.6)),
    (200, 37, 0, 0, 1, (0.53, 0.53)),
    (513, 21, 0, 0, 2, (1.0, 1.0)),
    (116, 40, 1, 0, 40, (1.0, 1.0)),     # two full 58-column tiles
    (117, 9, 0, 0, 3, (1.0, 1.0)),       # one column into a third tile
    (3, 3, 0, 0, 1, (1.0, 1.0)),
    (5, 7, 1, 1, 2, (0.9, 0.9)),
    (3, 4, 1, 0, 4, (1.0, 1.0)),         # the band wraps around the lattice in y
]


@pytest.mark.parametrize("nx,ny,bc,forcing,band,tau", CASES)
def test_two_step_ragged_grids_and_bands(lb, nx, ny, bc, forcing, band, tau):
    """Partial tiles and bands, x seams inside a wave (lattices narrower than
    the wave wrap several times), bands of one row, both wall modes and
    forcing schemes, unequal relaxation times; 1, 2 and 29 steps."""
    _say("two-step ragged", nx, ny, "bc", bc, "forcing", forcing, "band", band, "tau", tau)
    g = 1e-4 if ny > 5 else 0.0
    m = _member(lb, nx, ny, G=1.2, g=g, tau=tau, amp=min(2.0, ny / 6))
    lat = _lattice(lb, [m], band=band, chunk=-1, forcing=forcing, bc=bc)
    p = _params(m, forcing, bc)
    f = oracle.fill_equilibrium(p, m.rhoA0, m.rhoB0)
    for steps in (1, 2, 29):
        f = oracle.run(p, f, steps)
        lat.step(steps)
        assert _rel(lat.get_populations(0).cpu().numpy(), f) <= TOL, steps
    lat.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s"])
@pytest.mark.parametrize("forcing", [0, 1], ids=["shift", "guo"])
def test_two_step_equals_single_step(lb, storage, forcing):
    """In every storage mode the fused pass reproduces two single steps bit
    for bit (its step-1 results pass through the storage encoding)."""
    _say("two-step vs single-step", storage, "guo" if forcing else "shift")
    st = {"f64": lb.F64, "f32": lb.F32, "f16s": lb.F16S, "bf16s": lb.BF16S}[storage]
    m = _member(lb, 190, 70, seed=9, g=1e-4)
    one = _lattice(lb, [m], spp=1, chunk=-1, forcing=forcing, storage=st, tile=(128, 16))
    two = _lattice(lb, [m], spp=2, band=24, chunk=8, forcing=forcing, storage=st)
    for n in (2, 7, 31):
        one.step(n)
        two.step(n)
        assert np.array_equal(one.get_populations(0).cpu().numpy(), two.get_populations(0).cpu().numpy()), n
    one.close()
    two.close()


@pytest.mark.parametrize("storage", ["f32", "bf16s"])
@pytest.mark.parametrize("bc", [0, 1], ids=["walls", "periodic_y"])
def test_two_step_ragged_bands_reduced_precision(lb, storage, bc):
    """The 32-bit-arithmetic fused pass (three rotating register sets) equals
    single steps bit for bit for band heights whose march lengths leave every
    remainder modulo three, with a ragged last band and a ragged last tile."""
    st = {"f32": lb.F32, "bf16s": lb.BF16S}[storage]
    for band in (1, 2, 3, 5, 7):
        _say("two-step ragged bands", storage, "periodic_y" if bc else "walls", "band", band)
        m = _member(lb, 130, 23, seed=5, g=1e-4)
        one = _lattice(lb, [m], spp=1, chunk=-1, bc=bc, storage=st, tile=(64, 16))
        two = _lattice(lb, [m], spp=2, band=band, chunk=-1, bc=bc, storage=st)
        for n in (2, 5):
            one.step(n)
            two.step(n)
            assert np.array_equal(one.get_populations(0).cpu().numpy(), two.get_populations(0).cpu().numpy()), \
                (band, n)
        one.close()
        two.close()


@pytest.mark.parametrize("chunk", [2, 6, 8])
def test_two_step_graph_parity(lb, chunk):
    """Graphs of an odd number of passes flip the buffer parity on every
    replay; the result equals eager launches."""
    _say("two-step graph chunk", chunk)
    m = _member(lb, 160, 48, seed=2)
    a = _lattice(lb, [m], band=16, chunk=chunk)
    b = _lattice(lb, [m], band=16, chunk=-1)
    for n in (3, 20, 17, 40):
        a.step(n)
        b.step(n)
    assert a.t == b.t == 80
    assert np.array_equal(a.get_populations(0).cpu().numpy(), b.get_populations(0).cpu().numpy())
    a.close()
    b.close()


def test_two_step_ensemble_equals_solo(lb):
    """One fused launch over uneven members gives each member its solo result."""
    _say("two-step ensemble vs solo")
    specs = [(96, 40, 0.5, 3), (160, 64, 1.5, 4), (64, 24, 1.5, 5)]
    members = [_member(lb, nx, ny, G=G, g=1e-4, seed=seed) for nx, ny, G, seed in specs]
    ens = _lattice(lb, members, band=16, chunk=4)
    ens.step(30)
    for k, m in enumerate(members):
        solo = _lattice(lb, [m], band=16, chunk=4)
        solo.step(30)
        assert np.array_equal(ens.get_populations(k).cpu().numpy(), solo.get_populations(0).cpu().numpy()), k
        solo.close()
    ens.close()


def test_timed_choice_matches_oracle(lb):
    """steps_per_pass = 0 with timed tiles: whichever pass is chosen, the
    state after 21 steps equals the oracle's."""
    _say("timed pass choice")
    m = _member(lb, 300, 90, seed=4, g=1e-4)
    lat = lb.Lattice([m], graph_chunk=10, poison=True, steps_per_pass=0)
    print("[case] chosen", lat.steps_per_pass, lat.tile_shape(), flush=True)
    lat.step(21)
    p = _params(m)
    f = oracle.run(p, oracle.fill_equilibrium(p, m.rhoA0, m.rhoB0), 21)
    assert _rel(lat.get_populations(0).cpu().numpy(), f) <= TOL
    lat.close()
