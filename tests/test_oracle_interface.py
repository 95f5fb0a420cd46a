"""Pins of the interface-length oracle (oracle/interface.py, Sec. 3 Eq. 21):
crossing counts against brute force on small lattices, the exact counts of
a flat interface, and the Cauchy-Crofton length of circles against 2 pi R."""
import numpy as np

from oracle import interface


def _brute_counts(phi, trim):
    ny, nx = phi.shape
    pos = phi > 0
    n = [0, 0, 0, 0]
    for y in range(trim, ny - trim):
        for x in range(nx):
            xp = (x + 1) % nx
            n[0] += pos[y, x] != pos[y, xp]
            if y + 1 < ny - trim:
                n[1] += pos[y, x] != pos[y + 1, x]
                n[2] += pos[y, x] != pos[y + 1, xp]
                n[3] += pos[y, xp] != pos[y + 1, x]
    return n


def test_counts_equal_brute_force():
    rng = np.random.default_rng(5)
    for nx, ny, trim in ((7, 9, 1), (12, 10, 2), (3, 6, 1)):
        phi = rng.standard_normal((ny, nx))
        c = interface.crossing_counts(phi, trim)
        assert [c["n0"], c["n90"], c["n45"], c["n135"]] == _brute_counts(phi, trim)


def test_flat_interface_counts_and_length():
    nx, ny, trim = 50, 40, 10
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    out = interface.interface_length(0.5 + 0.5 * np.tanh(y - 19.5), 0.5 - 0.5 * np.tanh(y - 19.5), trim)
    assert (out["n0"], out["n90"], out["n45"], out["n135"]) == (0, nx, nx, nx)
    assert out["length"] == np.pi / 8 * (nx + 2 * nx / np.sqrt(2))


def test_sites_with_phi_zero_belong_to_the_b_phase():
    """A site is in the A phase where phi > 0 strictly: on a checkerboard of
    phi = 0 and phi = 1 every row and column pair crosses and no diagonal
    pair does (counting phi = 0 as A would see no interface at all)."""
    nx, ny, trim = 8, 12, 2
    y, x = np.mgrid[0:ny, 0:nx]
    phi = ((x + y) % 2).astype(np.float64)
    c = interface.crossing_counts(phi, trim)
    m = ny - 2 * trim
    assert (c["n0"], c["n90"], c["n45"], c["n135"]) == (nx * m, nx * (m - 1), 0, 0)


def test_circle_length():
    """The four directions sample theta exactly for a circle (its crossing
    integral is 4R at every angle), so only the line spacing errs."""
    for R in (30.0, 60.0):
        n = int(2 * R + 40)
        x = np.arange(n, dtype=np.float64)[None, :] - n / 2 + 0.37
        y = np.arange(n, dtype=np.float64)[:, None] - n / 2 + 0.21
        phi = R - np.hypot(x, y)
        c = interface.crossing_counts(phi, trim=5)
        L = interface.crofton_length(c)
        assert abs(L / (2 * np.pi * R) - 1) < 0.01, (R, L)


def test_length_is_additive_over_disjoint_drops():
    n = 200
    x = np.arange(n, dtype=np.float64)[None, :]
    y = np.arange(n, dtype=np.float64)[:, None]
    a = 20 - np.hypot(x - 50.3, y - 60.1)
    b = 15 - np.hypot(x - 140.2, y - 120.7)
    ca, cb = interface.crossing_counts(a, 5), interface.crossing_counts(b, 5)
    cab = interface.crossing_counts(np.maximum(a, b), 5)
    assert all(cab[k] == ca[k] + cb[k] for k in cab)
    la, lb, lab = (interface.crofton_length(c) for c in (ca, cb, cab))
    assert abs(lab - (la + lb)) <= 1e-12 * lab
