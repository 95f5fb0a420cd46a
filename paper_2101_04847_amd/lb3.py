"""ctypes binding of the 3D (D3Q19) entry points of liblb.so (include/lb3.h).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies the device workspace and the stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .lb import F32, F64, LB_EINVAL, LB_ENONFINITE, LBError, PERIODIC_Y, WALLS, _check, _lib

_dp = ctypes.POINTER(ctypes.c_double)
_h = ctypes.c_void_p
NQ3 = 19


class Lb3Config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("bc_y", ctypes.c_int32), ("storage", ctypes.c_int32), ("diag_trim", ctypes.c_int32),
                ("two_pass", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tau", ctypes.c_double * 2), ("G_AB", ctypes.c_double), ("g", (ctypes.c_double * 3) * 2),
                ("rhoA0", _dp), ("rhoB0", _dp)]


class Lb3Diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("mass", ctypes.c_double * 2), ("Ek", ctypes.c_double),
                ("umax", ctypes.c_double), ("finite", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib.lb3_workspace_bytes.argtypes = [ctypes.POINTER(Lb3Config)]
_lib.lb3_workspace_bytes.restype = ctypes.c_size_t
_lib.lb3_init.argtypes = [ctypes.POINTER(Lb3Config), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                          ctypes.POINTER(ctypes.c_void_p)]
_lib.lb3_init.restype = ctypes.c_int32
_lib.lb3_step.argtypes = [_h, ctypes.c_int64]
_lib.lb3_step.restype = ctypes.c_int32
_lib.lb3_fields.argtypes = [_h] + [ctypes.c_void_p] * 5
_lib.lb3_fields.restype = ctypes.c_int32
_lib.lb3_diagnostics.argtypes = [_h, ctypes.POINTER(Lb3Diag)]
_lib.lb3_diagnostics.restype = ctypes.c_int32
_lib.lb3_get_populations.argtypes = [_h, ctypes.c_void_p]
_lib.lb3_get_populations.restype = ctypes.c_int32
_lib.lb3_set_populations.argtypes = [_h, ctypes.c_void_p]
_lib.lb3_set_populations.restype = ctypes.c_int32
_lib.lb3_time.argtypes = [_h]
_lib.lb3_time.restype = ctypes.c_int64
_lib.lb3_destroy.argtypes = [_h]
_lib.lb3_destroy.restype = ctypes.c_int32

EXPORTS3 = ("lb3_workspace_bytes", "lb3_init", "lb3_step", "lb3_fields", "lb3_diagnostics",
            "lb3_get_populations", "lb3_set_populations", "lb3_time", "lb3_destroy")


def make_config3(nx, ny, nz, rhoA0, rhoB0, *, tau=(1.0, 1.0), G=0.0, g=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),
                 bc_y=WALLS, storage=F64, diag_trim=0, two_pass=False):
    """Build an Lb3Config; returns (config, keepalive list)."""
    a = np.ascontiguousarray(rhoA0, dtype=np.float64)
    b = np.ascontiguousarray(rhoB0, dtype=np.float64)
    if a.shape != (nz, ny, nx) or b.shape != (nz, ny, nx):
        raise ValueError(f"initial densities must be [{nz}][{ny}][{nx}]")
    c = Lb3Config()
    c.nx, c.ny, c.nz = int(nx), int(ny), int(nz)
    c.bc_y, c.storage, c.diag_trim = int(bc_y), int(storage), int(diag_trim)
    c.two_pass, c.reserved = (1 if two_pass else 0), 0
    c.tau[0], c.tau[1] = float(tau[0]), float(tau[1])
    c.G_AB = float(G)
    for s in range(2):
        for d in range(3):
            c.g[s][d] = float(g[s][d])
    c.rhoA0 = a.ctypes.data_as(_dp)
    c.rhoB0 = b.ctypes.data_as(_dp)
    return c, [a, b]


class Lattice3:
    """A 3D lattice on the GPU: x and z periodic, y walls or periodic."""

    def __init__(self, nx, ny, nz, rhoA0, rhoB0, *, tau=(1.0, 1.0), G=0.0, g=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),
                 bc_y=WALLS, storage=F64, diag_trim=0, two_pass=False, device="cuda", stream=None, poison=False):
        import torch
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.device = torch.device(device)
        cfg, keep = make_config3(nx, ny, nz, rhoA0, rhoB0, tau=tau, G=G, g=g, bc_y=bc_y, storage=storage,
                                 diag_trim=diag_trim, two_pass=two_pass)
        nbytes = _lib.lb3_workspace_bytes(ctypes.byref(cfg))
        if nbytes == 0:
            raise LBError(LB_EINVAL, "lb3_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if poison:
            self.workspace.fill_(0xFF)   # every unwritten double reads as NaN
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace tensor is not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(_lib.lb3_init(ctypes.byref(cfg), ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "lb3_init")
        self._h = h
        del keep

    @property
    def t(self) -> int:
        return int(_lib.lb3_time(self._h))

    def step(self, n: int = 1) -> None:
        _check(_lib.lb3_step(self._h, int(n)), "lb3_step")

    def fields(self) -> dict:
        import torch
        keys = ("rhoA", "rhoB", "ux", "uy", "uz")
        out = {k: torch.empty((self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device) for k in keys}
        _check(_lib.lb3_fields(self._h, *[ctypes.c_void_p(out[k].data_ptr()) for k in keys]), "lb3_fields")
        return out

    def diagnostics(self, check_finite: bool = True) -> dict:
        """Masses, E_k and max|u| (lb3_diag).  A non-finite state raises
        unless check_finite is False (then "finite" is False)."""
        d = Lb3Diag()
        rc = _lib.lb3_diagnostics(self._h, ctypes.byref(d))
        if rc != 0 and not (rc == LB_ENONFINITE and not check_finite):
            raise LBError(rc, "lb3_diagnostics")
        return {"t": d.t, "mass_A": d.mass[0], "mass_B": d.mass[1], "Ek": d.Ek, "umax": d.umax,
                "finite": bool(d.finite)}

    def get_populations(self):
        import torch
        f = torch.empty((2, NQ3, self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
        _check(_lib.lb3_get_populations(self._h, ctypes.c_void_p(f.data_ptr())), "lb3_get_populations")
        return f

    def set_populations(self, f) -> None:
        if tuple(f.shape) != (2, NQ3, self.nz, self.ny, self.nx) or not f.is_contiguous():
            raise ValueError("populations must be a contiguous (2, 19, nz, ny, nx) float64 device tensor")
        if str(f.dtype) != "torch.float64":
            raise ValueError("populations must be float64")
        _check(_lib.lb3_set_populations(self._h, ctypes.c_void_p(f.data_ptr())), "lb3_set_populations")
        self._keep_f = f

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _check(_lib.lb3_destroy(self._h), "lb3_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["Lattice3", "make_config3", "Lb3Config", "Lb3Diag", "EXPORTS3", "F64", "F32", "WALLS", "PERIODIC_Y"]
