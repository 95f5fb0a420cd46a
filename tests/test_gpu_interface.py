"""GPU (gfx950) parity of the interface pass (lb_interface_length, Sec. 3
Eq. 20-21) against the oracle (oracle/interface.py on the oracle's fields of
the same state): integer crossing counts bit-exact, the Cauchy-Crofton
length identical."""
import pytest

import oracle
from oracle import interface
from paper_2101_04847_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2101_04847_amd import lb as mod
    return mod


def _check(got, p, f, trim):
    m = oracle.macro(p, f)
    want = interface.interface_length(m["rhoA"], m["rhoB"], trim)
    print("[case]  ", {k: got[k] for k in ("n0", "n90", "n45", "n135", "length")}, flush=True)
    for k in ("n0", "n90", "n45", "n135", "length"):
        assert got[k] == want[k], (k, got[k], want[k])


@pytest.mark.parametrize("nx,ny,trim,G,steps", [(256, 120, 10, 1.5, 300), (67, 23, 2, 1.5, 40), (3, 9, 1, 1.2, 7)])
def test_interface_counts_match_oracle(lb, nx, ny, trim, G, steps):
    print("[case] interface", nx, ny, trim, flush=True)
    rA, rB = inputs.multi_mode(nx, ny, 11) if nx > 8 else inputs.single_mode(nx, ny, 1.0)
    g = ((0.0, -1e-4), (0.0, 1e-4))
    mem = lb.Member(nx, ny, rA, rB, tau=(1.0, 1.0), G=G, g=g)
    lat = lb.Lattice([mem], tile_x=64, tile_h=16, graph_chunk=-1, poison=True, diag_trim=trim)
    p = oracle.Params(nx=nx, ny=ny, tau=(1.0, 1.0), G=G, g=g)
    f = oracle.fill_equilibrium(p, rA, rB)
    _check(lat.interface_length(0), p, f, trim)
    lat.step(steps)
    oracle.run_inplace(p, f, steps)
    got = lat.interface_length(0)
    assert got["t"] == steps
    _check(got, p, f, trim)
    lat.close()


def test_sites_with_phi_zero_belong_to_b(lb):
    """Exact zeros of phi (rho_A = rho_B at rest) count as the B phase, as in
    the oracle: a checkerboard of phi = 0 and phi = 0.4 crosses on every row
    and column pair and on no diagonal pair."""
    import numpy as np
    print("[case] interface, phi = 0 checkerboard", flush=True)
    nx, ny, trim = 64, 20, 2
    y, x = np.mgrid[0:ny, 0:nx]
    rA = np.where((x + y) % 2 == 1, 0.95, 0.55)
    rB = np.full((ny, nx), 0.55)
    lat = lb.Lattice([lb.Member(nx, ny, rA, rB)], tile_x=64, tile_h=16, graph_chunk=-1, diag_trim=trim)
    p = oracle.Params(nx=nx, ny=ny)
    f = oracle.fill_equilibrium(p, rA, rB)
    got = lat.interface_length(0)
    m = ny - 2 * trim
    assert (got["n0"], got["n90"], got["n45"], got["n135"]) == (nx * m, nx * (m - 1), 0, 0)
    _check(got, p, f, trim)
    lat.close()


def test_interface_medium_timed_configuration(lb):
    wl = inputs.MEDIUM_2048x1024
    print("[case] interface", wl.name, flush=True)
    rA, rB = wl.densities()
    lat = lb.Lattice([lb.Member(wl.nx, wl.ny, rA, rB, tau=(wl.tau, wl.tau), G=wl.G, g=wl.gravity)], graph_chunk=100)
    lat.step(500)
    got = lat.interface_length(0)
    lat.close()
    p = oracle.Params(nx=wl.nx, ny=wl.ny, tau=(wl.tau, wl.tau), G=wl.G, g=wl.gravity)
    f = oracle.run(p, oracle.fill_equilibrium(p, rA, rB), 500)
    _check(got, p, f, 10)
