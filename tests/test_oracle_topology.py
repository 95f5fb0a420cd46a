"""Pins of the component-count oracle (oracle/topology.py): brute-force
flood fill on small periodic-x lattices, and shapes with known counts."""
import numpy as np

from oracle import topology


def _flood_count(mask):
    ny, nx = mask.shape
    seen = np.zeros_like(mask, dtype=bool)
    count = 0
    for y in range(ny):
        for x in range(nx):
            if mask[y, x] and not seen[y, x]:
                count += 1
                stack = [(y, x)]
                seen[y, x] = True
                while stack:
                    cy, cx = stack.pop()
                    for ny_, nx_ in ((cy, (cx + 1) % nx), (cy, (cx - 1) % nx), (cy + 1, cx), (cy - 1, cx)):
                        if 0 <= ny_ < ny and mask[ny_, nx_] and not seen[ny_, nx_]:
                            seen[ny_, nx_] = True
                            stack.append((ny_, nx_))
    return count


def _fields(mask, trim):
    """Densities whose phi is +1 on mask and -1 elsewhere, padded by trim rows."""
    phi = np.where(mask, 1.0, -1.0)
    pad = np.full((trim, mask.shape[1]), -1.0)
    phi = np.vstack([pad, phi, pad])
    return 0.5 * (1 + phi), 0.5 * (1 - phi)


def test_counts_equal_flood_fill():
    rng = np.random.default_rng(3)
    for shape, p in (((9, 11), 0.5), ((16, 5), 0.45), ((4, 3), 0.6), ((20, 20), 0.3)):
        for _ in range(5):
            m = rng.random(shape) < p
            a, b = _fields(m, 2)
            c = topology.component_counts(a, b, trim=2)
            assert c["A"] == _flood_count(m) and c["B"] == _flood_count(~m)


def test_known_shapes():
    n = 60
    x = np.arange(n)[None, :]
    y = np.arange(40)[:, None]
    # two disks, one of them cut by the periodic seam
    m = (np.hypot(x - 20, y - 20) < 8) | (np.hypot(((x + 30) % n) - 30, y - 20) < 6)
    a, b = _fields(m, 3)
    assert topology.component_counts(a, b, 3) == {"A": 2, "B": 1}
    # a band that wraps around in x is one component and splits B in two
    m = (y > 10) & (y < 20) & (x >= 0)
    a, b = _fields(m, 3)
    assert topology.component_counts(a, b, 3) == {"A": 1, "B": 2}
    # checkerboard: every site is its own 4-connected component
    m = ((x[:, :8] + y[:8]) % 2) == 0
    a, b = _fields(m, 1)
    assert topology.component_counts(a, b, 1) == {"A": 32, "B": 32}
    # sites with phi = 0 exactly (rho_A = rho_B) belong to the B phase
    a0, b0 = np.where(a > 0.5, 1.0, 0.5), np.full_like(a, 0.5)
    assert topology.component_counts(a0, b0, 1) == {"A": 32, "B": 32}
