"""Python access to the FP64 CPU oracle in ``orc.c``.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check in
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``.  The GPU
library never imports, links or calls anything in this directory, and this
module imports nothing from the GPU package.

The oracle implements one time step of the two-component D2Q9 Shan-Chen
lattice Boltzmann model of Sec. 2 of the paper (Eq. 1-7) in push form, the
energy-budget averages of Sec. 3 (Eq. 15-18, Eq. 22) and, in ``budget.py``,
the momentum-flux and viscous terms of the kinetic-energy balance
(Eq. 11-14, 17-19).  Arrays follow the
layout f[s][i][y][x] (s = A, B; i = 0..8), densities and velocities [y][x].
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

FORCE_SHIFT = 0
FORCE_GUO = 1
PSI_MIRROR = 0
PSI_ZERO = 1

NQ = 9


def build(force: bool = True) -> str:
    """Compile ``orc.c`` into ``liborc.so`` with gcc (FP64, no FMA contraction,
    no fast-math, OpenMP over rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("forcing", ctypes.c_int32), ("periodic_y", ctypes.c_int32),
                ("tau", ctypes.c_double * 2), ("G", ctypes.c_double),
                ("g", ctypes.c_double * 4), ("Gw", ctypes.c_double * 2),
                ("psi_wall", ctypes.c_int32), ("pad_", ctypes.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        lib.orc_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_constants.argtypes = [ctypes.POINTER(ctypes.c_int32)] * 3 + [dp]
        lib.orc_equilibrium.argtypes = [ctypes.c_double] * 3 + [dp]
        lib.orc_fill_equilibrium.argtypes = [pp, dp, dp, dp, dp, dp]
        lib.orc_scratch_doubles.argtypes = [pp]
        lib.orc_scratch_doubles.restype = ctypes.c_size_t
        lib.orc_step.argtypes = [pp, dp, dp, dp]
        lib.orc_run.argtypes = [pp, dp, ctypes.c_int64]
        lib.orc_run.restype = ctypes.c_int
        lib.orc_macro.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp]
        lib.orc_macro.restype = ctypes.c_int
        lib.orc_diagnostics.argtypes = [pp, dp, ctypes.c_int32, dp, dp]
        lib.orc_diagnostics.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Params:
    """Model parameters of one lattice (Sec. 2).  ``g`` holds the body
    acceleration of each component; Eq. 7 is gA = (0, -g~), gB = (0, +g~).
    ``G_wall`` are the fluid-boundary couplings (G_Ab, G_Bb) of Eq. 6;
    ``wall_psi`` selects psi on the boundary nodes in Eq. 5 (PSI_MIRROR: the
    adjacent fluid row; PSI_ZERO: zero)."""
    nx: int
    ny: int
    tau: tuple = (1.0, 1.0)
    G: float = 0.0
    g: tuple = ((0.0, 0.0), (0.0, 0.0))
    forcing: int = FORCE_SHIFT
    periodic_y: bool = False
    G_wall: tuple = (0.0, 0.0)
    wall_psi: int = 0

    def c(self) -> _Params:
        p = _Params()
        p.nx, p.ny = int(self.nx), int(self.ny)
        p.forcing = int(self.forcing)
        p.periodic_y = 1 if self.periodic_y else 0
        p.tau[0], p.tau[1] = float(self.tau[0]), float(self.tau[1])
        p.G = float(self.G)
        flat = [float(self.g[0][0]), float(self.g[0][1]), float(self.g[1][0]), float(self.g[1][1])]
        for k in range(4):
            p.g[k] = flat[k]
        p.Gw[0], p.Gw[1] = float(self.G_wall[0]), float(self.G_wall[1])
        p.psi_wall = int(self.wall_psi)
        return p


def threads() -> int:
    return _load().orc_threads()


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def constants():
    """Velocity set, opposite table and weights used by the oracle."""
    lib = _load()
    cx = (ctypes.c_int32 * NQ)()
    cy = (ctypes.c_int32 * NQ)()
    opp = (ctypes.c_int32 * NQ)()
    w = (ctypes.c_double * NQ)()
    lib.orc_constants(cx, cy, opp, w)
    return (np.array(cx[:], dtype=np.int64), np.array(cy[:], dtype=np.int64),
            np.array(opp[:], dtype=np.int64), np.array(w[:], dtype=np.float64))


def equilibrium(rho: float, vx: float, vy: float) -> np.ndarray:
    """Eq. 3 equilibrium populations for one site."""
    out = np.zeros(NQ)
    _load().orc_equilibrium(float(rho), float(vx), float(vy), _ptr(out))
    return out


def fill_equilibrium(p: Params, rhoA, rhoB, ux=None, uy=None) -> np.ndarray:
    """Populations f[2][9][ny][nx] at equilibrium with the given densities and
    common velocity (rest if ux, uy are None)."""
    rhoA = np.ascontiguousarray(rhoA, dtype=np.float64)
    rhoB = np.ascontiguousarray(rhoB, dtype=np.float64)
    assert rhoA.shape == (p.ny, p.nx) and rhoB.shape == (p.ny, p.nx)
    ux = None if ux is None else np.ascontiguousarray(np.broadcast_to(ux, (p.ny, p.nx)), dtype=np.float64)
    uy = None if uy is None else np.ascontiguousarray(np.broadcast_to(uy, (p.ny, p.nx)), dtype=np.float64)
    f = np.empty((2, NQ, p.ny, p.nx))
    pc = p.c()
    _load().orc_fill_equilibrium(ctypes.byref(pc), _ptr(rhoA), _ptr(rhoB), _ptr(ux), _ptr(uy), _ptr(f))
    return f


def step(p: Params, f: np.ndarray) -> np.ndarray:
    """One time step; returns a new array f(t+1)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    assert f.shape == (2, NQ, p.ny, p.nx)
    pc = p.c()
    lib = _load()
    out = np.empty_like(f)
    scratch = np.empty(lib.orc_scratch_doubles(ctypes.byref(pc)))
    lib.orc_step(ctypes.byref(pc), _ptr(f), _ptr(out), _ptr(scratch))
    return out


def run(p: Params, f: np.ndarray, nsteps: int) -> np.ndarray:
    """Advance a copy of f by nsteps time steps."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    assert f.shape == (2, NQ, p.ny, p.nx)
    pc = p.c()
    if _load().orc_run(ctypes.byref(pc), _ptr(f), int(nsteps)) != 0:
        raise MemoryError("oracle run: allocation failed")
    return f


def run_inplace(p: Params, f: np.ndarray, nsteps: int) -> None:
    """Advance f (C-contiguous float64) in place by nsteps time steps."""
    assert f.dtype == np.float64 and f.flags.c_contiguous and f.shape == (2, NQ, p.ny, p.nx)
    pc = p.c()
    if _load().orc_run(ctypes.byref(pc), _ptr(f), int(nsteps)) != 0:
        raise MemoryError("oracle run: allocation failed")


def macro(p: Params, f: np.ndarray) -> dict:
    """rhoA, rhoB, hydrodynamic velocity ux, uy and total force Fx, Fy at time t."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = {k: np.empty((p.ny, p.nx)) for k in ("rhoA", "rhoB", "ux", "uy", "Fx", "Fy")}
    pc = p.c()
    rc = _load().orc_macro(ctypes.byref(pc), _ptr(f), _ptr(out["rhoA"]), _ptr(out["rhoB"]),
                           _ptr(out["ux"]), _ptr(out["uy"]), _ptr(out["Fx"]), _ptr(out["Fy"]))
    if rc != 0:
        raise MemoryError("oracle macro: allocation failed")
    return out


DIAG_KEYS = ("mass_A", "mass_B", "Ek", "Ep", "buoyancy", "omega2", "umax", "finite")


def diagnostics(p: Params, f: np.ndarray, trim: int = 10, profile: bool = False) -> dict:
    """Energy-budget averages of Sec. 3 over the trimmed subdomain."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(8)
    prof = np.zeros(p.ny) if profile else None
    pc = p.c()
    rc = _load().orc_diagnostics(ctypes.byref(pc), _ptr(f), int(trim), _ptr(out), _ptr(prof))
    if rc == -2:
        raise ValueError("trimmed subdomain is empty")
    if rc != 0:
        raise MemoryError("oracle diagnostics: allocation failed")
    d = dict(zip(DIAG_KEYS, out.tolist()))
    d["finite"] = bool(d["finite"])
    if profile:
        d["phi_profile"] = prof
    return d


def energy_budget(p: Params, f: np.ndarray, trim: int = 10) -> dict:
    """Kinetic-energy budget terms (Eq. 17-19) of the state f: the fields of
    ``macro`` passed to ``budget.budget_from_fields`` with tau the mean of
    tau_A and tau_B."""
    from .budget import budget_from_fields
    m = macro(p, f)
    tau = 0.5 * (float(p.tau[0]) + float(p.tau[1]))
    return budget_from_fields(m["rhoA"], m["rhoB"], m["ux"], m["uy"], float(p.G), tau, trim)
