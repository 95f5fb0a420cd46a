"""GPU (gfx950) parity of the component count (lb_components) against the
oracle (oracle/topology.py on the oracle's fields of the same state): exact
integer counts for shapes with known topology, dense random masks (many
small components: the hardest case for the concurrent union-find) and
lattice Boltzmann states."""
import numpy as np
import pytest

import oracle
from oracle import topology
from paper_2101_04847_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2101_04847_amd import lb as mod
    return mod


def _lattice_from_phi(lb, phi, trim, G=0.0):
    ny, nx = phi.shape
    rA, rB = 0.55 + 0.5 * phi, 0.55 - 0.5 * phi
    lat = lb.Lattice([lb.Member(nx, ny, rA, rB, G=G)], tile_x=64, tile_h=16, graph_chunk=-1, diag_trim=trim)
    p = oracle.Params(nx=nx, ny=ny, G=G)
    return lat, p, oracle.fill_equilibrium(p, rA, rB)


def _check(got, p, f, trim):
    m = oracle.macro(p, f)
    want = topology.component_counts(m["rhoA"], m["rhoB"], trim)
    print("[case]   gpu", got["A"], got["B"], "oracle", want["A"], want["B"], flush=True)
    assert (got["A"], got["B"]) == (want["A"], want["B"])


def test_known_shapes(lb):
    print("[case] shapes", flush=True)
    nx, ny, trim = 200, 90, 5
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    disk = (np.hypot(x - 50, y - 45) < 15) | (np.hypot(((x + 100) % nx) - 100, y - 40) < 12) \
        | (np.hypot(x - 120, y - 30) < 6)
    phi = np.where(disk, 0.4, -0.4)
    lat, p, f = _lattice_from_phi(lb, phi, trim)
    got = lat.components(0)
    assert (got["A"], got["B"]) == (3, 1)
    _check(got, p, f, trim)
    lat.close()


def test_sites_with_phi_zero_belong_to_b(lb):
    """Exact zeros of phi (rho_A = rho_B at rest) count as the B phase, as in
    the oracle: on a checkerboard of phi = 0 and phi = 0.4 every site of D is
    its own 4-connected component."""
    print("[case] phi = 0 checkerboard", flush=True)
    nx, ny, trim = 64, 20, 2
    y, x = np.mgrid[0:ny, 0:nx]
    phi = np.where((x + y) % 2 == 1, 0.4, 0.0)
    lat, p, f = _lattice_from_phi(lb, phi, trim)
    got = lat.components(0)
    half = nx * (ny - 2 * trim) // 2
    assert (got["A"], got["B"]) == (half, half)
    _check(got, p, f, trim)
    lat.close()


@pytest.mark.parametrize("nx,ny,frac,seed", [(64, 40, 0.5, 1), (257, 130, 0.45, 2), (1000, 600, 0.55, 3),
                                             (2048, 1024, 0.5, 4)])
def test_random_masks(lb, nx, ny, frac, seed):
    print("[case] random mask", nx, ny, frac, flush=True)
    rng = np.random.default_rng(seed)
    phi = np.where(rng.random((ny, nx)) < frac, 0.3, -0.3)
    lat, p, f = _lattice_from_phi(lb, phi, 3)
    _check(lat.components(0), p, f, 3)
    lat.close()


def test_lattice_boltzmann_state(lb):
    print("[case] RT state", flush=True)
    nx, ny = 256, 120
    rA, rB = inputs.multi_mode(nx, ny, 13)
    g = ((0.0, -1e-4), (0.0, 1e-4))
    lat = lb.Lattice([lb.Member(nx, ny, rA, rB, tau=(1.0, 1.0), G=1.5, g=g)], tile_x=64, tile_h=16,
                     graph_chunk=-1, diag_trim=10)
    p = oracle.Params(nx=nx, ny=ny, tau=(1.0, 1.0), G=1.5, g=g)
    f = oracle.fill_equilibrium(p, rA, rB)
    for steps in (0, 600):
        lat.step(steps)
        oracle.run_inplace(p, f, steps)
        _check(lat.components(0), p, f, 10)
    lat.close()
