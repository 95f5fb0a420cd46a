"""The seeded input generators (paper_2101_04847_amd/inputs.py): determinism,
shapes and the geometry of the recipes (CPU only)."""
import numpy as np

from paper_2101_04847_amd import inputs


def test_multi_mode_is_seeded_and_bounded():
    a1, b1 = inputs.multi_mode(300, 120, 7)
    a2, b2 = inputs.multi_mode(300, 120, 7)
    a3, _ = inputs.multi_mode(300, 120, 8)
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2) and not np.array_equal(a1, a3)
    assert a1.shape == (120, 300) and a1.flags.c_contiguous
    assert a1.min() >= inputs.TRACE and a1.max() <= inputs.HEAVY_A
    # A on top: the top row is A-rich, the bottom row B-rich
    assert a1[-1].min() > 1.0 and b1[0].min() > 0.9


def test_white_noise_height_recipe():
    h = inputs.white_noise_height(10000, 5000, 3, 4.0)
    assert np.array_equal(h, inputs.white_noise_height(10000, 5000, 3, 4.0))
    assert np.all(np.abs(h - 0.5 * 4999) <= 4.0)
    # uniform on [-4, 4]: mean 0, variance 16/3
    assert abs(np.mean(h - 0.5 * 4999)) < 0.1 and abs(np.var(h - 0.5 * 4999) - 16 / 3) < 0.25


def test_profile_densities_follow_the_profile():
    yp = np.arange(-5.0, 6.0)
    pa = 0.1 + 0.9 * (yp > 0)
    pb = 1.1 - pa
    h = np.array([10.0, 12.0, 11.5])
    a, b = inputs.profile_densities(3, 25, h, yp, pa, pb)
    assert a.shape == (25, 3)
    # rows exactly at integer offsets reproduce the profile values
    assert np.allclose(a[10 + np.arange(-5, 6), 0], pa)
    assert np.allclose(a[12 + np.arange(-5, 6), 1], pa)
    # beyond the profile the end values hold
    assert a[0, 0] == pa[0] and a[-1, 2] == pa[-1]
    assert np.allclose(a + b, 1.1)


def test_rt3d_densities_recipe():
    a, b = inputs.rt3d_densities(40, 30, 20, 4)
    a2, _ = inputs.rt3d_densities(40, 30, 20, 4)
    assert a.shape == (20, 30, 40) and a.flags.c_contiguous and np.array_equal(a, a2)
    assert a.min() >= inputs.TRACE and a.max() <= inputs.HEAVY_A
    # heavy A on top in every column, light B below
    assert a[:, -1, :].min() > 1.0 and b[:, 0, :].min() > 0.9
    # the interface is perturbed along both x and z
    mid = a[:, 15, :]
    assert np.ptp(mid, axis=1).max() > 1e-3 and np.ptp(mid, axis=0).max() > 1e-3
