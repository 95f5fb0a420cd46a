"""Python access to the FP64 CPU oracle of the 3D (D3Q19) step in ``orc3.c``.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``.  The GPU library never
imports, links or calls anything in this directory.

Arrays: f[s][i][z][y][x] (s = A, B; i = 0..18), fields [z][y][x].
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc3.c")
_LIB = os.path.join(_HERE, "liborc3.so")

NQ = 19


def build(force: bool = True) -> str:
    """Compile ``orc3.c`` into ``liborc3.so`` (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("periodic_y", ctypes.c_int32), ("tau", ctypes.c_double * 2), ("G", ctypes.c_double),
                ("g", ctypes.c_double * 6)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        pp = ctypes.POINTER(_Params)
        lib.orc3_constants.argtypes = [ip, ip, ip, ip, dp]
        lib.orc3_fill_equilibrium.argtypes = [pp, dp, dp, dp]
        lib.orc3_run.argtypes = [pp, dp, ctypes.c_int64]
        lib.orc3_run.restype = ctypes.c_int
        lib.orc3_macro.argtypes = [pp, dp] + [dp] * 8
        lib.orc3_macro.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Params3:
    """One 3D lattice: x and z periodic, y walls (or periodic); ``g`` holds
    the body acceleration (x, y, z) of each component."""
    nx: int
    ny: int
    nz: int
    tau: tuple = (1.0, 1.0)
    G: float = 0.0
    g: tuple = ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    periodic_y: bool = False

    def c(self) -> _Params:
        p = _Params()
        p.nx, p.ny, p.nz = int(self.nx), int(self.ny), int(self.nz)
        p.periodic_y = 1 if self.periodic_y else 0
        p.tau[0], p.tau[1] = float(self.tau[0]), float(self.tau[1])
        p.G = float(self.G)
        for s in range(2):
            for d in range(3):
                p.g[3 * s + d] = float(self.g[s][d])
        return p


def constants():
    """Velocity set (cx, cy, cz), opposite table and weights of the oracle."""
    lib = _load()
    arrs = [(ctypes.c_int32 * NQ)() for _ in range(4)]
    w = (ctypes.c_double * NQ)()
    lib.orc3_constants(*arrs, w)
    return tuple(np.array(a[:], dtype=np.int64) for a in arrs) + (np.array(w[:]),)


def fill_equilibrium(p: Params3, rhoA, rhoB) -> np.ndarray:
    rA = np.ascontiguousarray(rhoA, dtype=np.float64)
    rB = np.ascontiguousarray(rhoB, dtype=np.float64)
    assert rA.shape == (p.nz, p.ny, p.nx) and rB.shape == rA.shape
    f = np.empty((2, NQ, p.nz, p.ny, p.nx))
    pc = p.c()
    _load().orc3_fill_equilibrium(ctypes.byref(pc), _ptr(rA), _ptr(rB), _ptr(f))
    return f


def run(p: Params3, f: np.ndarray, steps: int) -> np.ndarray:
    """f after ``steps`` steps (a new array)."""
    out = np.array(f, dtype=np.float64, order="C", copy=True)
    pc = p.c()
    if _load().orc3_run(ctypes.byref(pc), _ptr(out), int(steps)) != 0:
        raise MemoryError("oracle 3D run: allocation failed")
    return out


def run_inplace(p: Params3, f: np.ndarray, steps: int) -> None:
    """Advance f (C-contiguous float64) by ``steps`` steps in place."""
    assert f.dtype == np.float64 and f.flags.c_contiguous
    pc = p.c()
    if _load().orc3_run(ctypes.byref(pc), _ptr(f), int(steps)) != 0:
        raise MemoryError("oracle 3D run: allocation failed")


def macro(p: Params3, f: np.ndarray) -> dict:
    """rhoA, rhoB, hydrodynamic velocity (ux, uy, uz) and total force (Fx, Fy, Fz)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    keys = ("rhoA", "rhoB", "ux", "uy", "uz", "Fx", "Fy", "Fz")
    out = {k: np.empty((p.nz, p.ny, p.nx)) for k in keys}
    pc = p.c()
    if _load().orc3_macro(ctypes.byref(pc), _ptr(f), *[_ptr(out[k]) for k in keys]) != 0:
        raise MemoryError("oracle 3D macro: allocation failed")
    return out
