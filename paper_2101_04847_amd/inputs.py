"""Seeded synthetic inputs: initial component densities of Rayleigh-Taylor
set-ups in the shapes of the paper's runs (Sec. 2: heavy phase on top of a
light one, periodic in x, solid top and bottom, perturbed interface).

This module holds no lattice-Boltzmann arithmetic: it only draws interface
shapes and smooth density profiles.  Both the GPU library (through its Python
binding) and the CPU oracle take the arrays it returns as their inputs; each
side turns them into populations on its own.

Recipe (the paper initialises an equilibrium two-phase configuration with a
white-noise deformation of the interface; the workloads used here replace the
noise by the cosine-mode recipes below):
  interface height  y_int(x) = (ny - 1)/2 + sum_m a_m cos(2 pi m x / nx + theta_m)
  smooth step       s(x, y)  = (1 + tanh((y - y_int(x)) / w)) / 2,  w = 1.5
  densities         rho_A = trace + (heavy_A - trace) s
                    rho_B = trace + (heavy_B - trace) (1 - s)
A (the heavy component, pushed down by the buoyancy of Eq. 7) fills the top.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

WIDTH = 1.5
HEAVY_A = 1.05
HEAVY_B = 0.95
TRACE = 0.05


def interface_height(nx: int, ny: int, amps, phases, center: float | None = None) -> np.ndarray:
    """y_int(x) for mode numbers m = 1..len(amps)."""
    x = np.arange(nx, dtype=np.float64)
    yc = 0.5 * (ny - 1) if center is None else float(center)
    h = np.full(nx, yc)
    for m, (a, th) in enumerate(zip(amps, phases), start=1):
        h += float(a) * np.cos(2.0 * np.pi * m * x / nx + float(th))
    return h


def random_modes(seed: int, n_modes: int = 32, amp_max: float = 0.5):
    """Amplitudes a_m ~ U[0, amp_max] and phases theta_m ~ U[0, 2 pi), seeded."""
    rng = np.random.default_rng(seed)
    amps = rng.uniform(0.0, amp_max, n_modes)
    phases = rng.uniform(0.0, 2.0 * np.pi, n_modes)
    return amps, phases


def two_phase_densities(nx: int, ny: int, height: np.ndarray, heavy_a: float = HEAVY_A,
                        heavy_b: float = HEAVY_B, trace: float = TRACE, width: float = WIDTH):
    """Smooth A-over-B densities [ny][nx] around the interface height(x)."""
    y = np.arange(ny, dtype=np.float64)[:, None]
    s = 0.5 * (1.0 + np.tanh((y - height[None, :]) / width))
    rho_a = trace + (heavy_a - trace) * s
    rho_b = trace + (heavy_b - trace) * (1.0 - s)
    return np.ascontiguousarray(rho_a), np.ascontiguousarray(rho_b)


def single_mode(nx: int, ny: int, amplitude: float = 2.0, **kw):
    """One cosine mode of wavelength nx (the 128 x 64 parity workload)."""
    return two_phase_densities(nx, ny, interface_height(nx, ny, [amplitude], [0.0]), **kw)


def multi_mode(nx: int, ny: int, seed: int, n_modes: int = 32, amp_max: float = 0.5, **kw):
    """Sum of n_modes seeded random modes (the large workloads)."""
    amps, phases = random_modes(seed, n_modes, amp_max)
    return two_phase_densities(nx, ny, interface_height(nx, ny, amps, phases), **kw)


def white_noise_height(nx: int, ny: int, seed: int, amplitude: float = 4.0) -> np.ndarray:
    """Interface height (ny - 1)/2 + amplitude * xi(x) with xi ~ U[-1, 1]
    independent per column (the paper's white-noise deformation of
    amplitude 4 grid points), seeded."""
    rng = np.random.default_rng(seed)
    return 0.5 * (ny - 1) + float(amplitude) * rng.uniform(-1.0, 1.0, nx)


def profile_densities(nx: int, ny: int, height: np.ndarray, y_prof: np.ndarray, rho_a_prof: np.ndarray,
                      rho_b_prof: np.ndarray):
    """Densities [ny][nx] that follow a given one-dimensional interface
    profile (values at offsets y_prof from the interface, increasing) shifted
    to height(x) in every column (linear interpolation, constant beyond the
    ends of the profile)."""
    y = np.arange(ny, dtype=np.float64)[:, None] - height[None, :]
    rho_a = np.interp(y.ravel(), y_prof, rho_a_prof).reshape(ny, nx)
    rho_b = np.interp(y.ravel(), y_prof, rho_b_prof).reshape(ny, nx)
    return np.ascontiguousarray(rho_a), np.ascontiguousarray(rho_b)


@dataclass
class Workload:
    """One realisation: grid, coupling, gravity and the seed of its interface."""
    nx: int
    ny: int
    G: float = 1.5
    g: float = 1e-5
    tau: float = 1.0
    seed: int | None = None          # None: single cosine mode of amplitude 2
    name: str = ""

    def densities(self):
        if self.seed is None:
            return single_mode(self.nx, self.ny, 2.0)
        return multi_mode(self.nx, self.ny, self.seed)

    @property
    def gravity(self):
        """Eq. 7: component A pushed down, B pushed up, equal magnitude."""
        return ((0.0, -self.g), (0.0, self.g))


# The five reference workloads (sizes, couplings, seeds).  Gravity 1e-5 and
# tau = 1 throughout; the ensemble alternates miscible (G = 0.5) and
# immiscible (G = 1.5) members inside each size class.
SMALL_128x64 = Workload(128, 64, seed=None, name="rt-128x64-cos")
MEDIUM_2048x1024 = Workload(2048, 1024, seed=1, name="rt-2048x1024-32modes")
LARGE_10000x5000 = Workload(10000, 5000, seed=2, name="rt-10000x5000-32modes")
PRECISION_4096x2048 = (Workload(4096, 2048, G=0.5, seed=3, name="rt-4096x2048-miscible"),
                       Workload(4096, 2048, G=1.5, seed=3, name="rt-4096x2048-immiscible"))


def ensemble_16():
    """16 realisations: 4 x 1024x512, 8 x 2048x1024, 4 x 4096x2048, seeds
    100..115, half miscible and half immiscible within each size class."""
    members = []
    seed = 100
    for count, (nx, ny) in ((4, (1024, 512)), (8, (2048, 1024)), (4, (4096, 2048))):
        for k in range(count):
            G = 0.5 if k % 2 == 0 else 1.5
            members.append(Workload(nx, ny, G=G, seed=seed, name=f"ens-{nx}x{ny}-s{seed}"))
            seed += 1
    return members


def rt3d_densities(nx: int, ny: int, nz: int, seed: int, n_modes: int = 8, amp_max: float = 0.5):
    """3D Rayleigh-Taylor set-up for the D3Q19 extension: heavy A on top of
    light B with the interface y_int(x, z) = (ny - 1)/2 + sum over random
    modes (m, l) of a cos(2 pi (m x / nx + l z / nz) + theta), m, l in
    1..n_modes, a ~ U[0, amp_max), theta ~ U[0, 2 pi); densities as in 2D.
    Arrays [nz][ny][nx]."""
    rng = np.random.default_rng(seed)
    m = rng.integers(1, n_modes + 1, size=n_modes)
    l = rng.integers(1, n_modes + 1, size=n_modes)
    a = rng.uniform(0.0, amp_max, size=n_modes)
    th = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    x = np.arange(nx, dtype=np.float64)[None, :]
    z = np.arange(nz, dtype=np.float64)[:, None]
    h = np.full((nz, nx), 0.5 * (ny - 1))
    for k in range(n_modes):
        h += a[k] * np.cos(2.0 * np.pi * (m[k] * x / nx + l[k] * z / nz) + th[k])
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    s = 0.5 * (1.0 + np.tanh((y - h[:, None, :]) / WIDTH))
    rho_a = TRACE + (HEAVY_A - TRACE) * s
    rho_b = TRACE + (HEAVY_B - TRACE) * (1.0 - s)
    return np.ascontiguousarray(rho_a), np.ascontiguousarray(rho_b)


# The 3D workload of the D3Q19 extension: 384^3 sites (about the site count
# of the 10000 x 5000 lattice), tau = 1, G = 1.5, g = 1e-5, walls in y.
D3_384 = dict(nx=384, ny=384, nz=384, seed=4, G=1.5, g=1e-5, tau=1.0, name="rt3d-384^3-8modes")
