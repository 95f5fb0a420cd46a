"""ctypes binding of liblb.so (C ABI in include/lb.h).

Argument marshalling only: every step of the lattice Boltzmann path runs in
the library's HIP kernels.  PyTorch provides the device workspace and the
stream.  Importing this module fails loudly if the library is not built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblb.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2101_04847_amd.build` "
                      "(or __graft_entry__.build()) first")

_lib = ctypes.CDLL(LIB_PATH)

# constants of lb.h
LB_OK, LB_EINVAL, LB_ENOMEM, LB_EHIP, LB_ESTATE, LB_ENONFINITE, LB_EINTERNAL = 0, -1, -2, -3, -4, -5, -6
FORCE_SHIFT, FORCE_GUO = 0, 1
F64, F32, F16S, BF16S = 0, 1, 2, 3
WALLS, PERIODIC_Y = 0, 1
PSI_MIRROR, PSI_ZERO = 0, 1
MAX_MEMBERS = 64
NOALLOC_MAX_NY = 16384
STORAGE_NAMES = {F64: "f64", F32: "f32", F16S: "f16s", BF16S: "bf16s"}
ELEM_BYTES = {F64: 8, F32: 4, F16S: 2, BF16S: 2}

_dp = ctypes.POINTER(ctypes.c_double)


class LbMember(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("tau", ctypes.c_double * 2), ("G_AB", ctypes.c_double),
                ("g", (ctypes.c_double * 2) * 2),
                ("rhoA0", _dp), ("rhoB0", _dp),
                ("reserved2", ctypes.c_double * 2),
                ("G_wall", ctypes.c_double * 2), ("wall_psi", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class LbConfig(ctypes.Structure):
    _fields_ = [("n_members", ctypes.c_int32), ("members", ctypes.POINTER(LbMember)),
                ("forcing", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("bc_y", ctypes.c_int32), ("diag_trim", ctypes.c_int32),
                ("tile_x", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("graph_chunk", ctypes.c_int32), ("steps_per_pass", ctypes.c_int32)]


class LbDiag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("mass", ctypes.c_double * 2),
                ("Ek", ctypes.c_double), ("Ep", ctypes.c_double),
                ("buoyancy", ctypes.c_double), ("omega2", ctypes.c_double),
                ("umax", ctypes.c_double), ("finite", ctypes.c_int32)]


class LbBudget(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("pb", ctypes.c_double), ("korteweg", ctypes.c_double),
                ("ktau", ctypes.c_double), ("viscous", ctypes.c_double), ("eta", ctypes.c_double),
                ("buoyancy", ctypes.c_double)]


class LbInterface(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("crossings", ctypes.c_int64 * 4), ("length", ctypes.c_double)]


class LbMixing(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("width", ctypes.c_double), ("bulk_ref", ctypes.c_double * 2)]


class LbTopology(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("components", ctypes.c_int64 * 2)]


_h = ctypes.c_void_p
_lib.lb_workspace_bytes.argtypes = [ctypes.POINTER(LbConfig)]
_lib.lb_workspace_bytes.restype = ctypes.c_size_t
_lib.lb_init.argtypes = [ctypes.POINTER(LbConfig), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                         ctypes.POINTER(ctypes.c_void_p)]
_lib.lb_init.restype = ctypes.c_int32
_lib.lb_step.argtypes = [_h, ctypes.c_int64]
_lib.lb_step.restype = ctypes.c_int32
_lib.lb_fields.argtypes = [_h, ctypes.c_int32] + [ctypes.c_void_p] * 4
_lib.lb_fields.restype = ctypes.c_int32
_lib.lb_diagnostics.argtypes = [_h, ctypes.c_int32, ctypes.POINTER(LbDiag), _dp]
_lib.lb_diagnostics.restype = ctypes.c_int32
_lib.lb_mixing_width.argtypes = [_h, ctypes.c_int32, _dp, ctypes.POINTER(LbMixing)]
_lib.lb_mixing_width.restype = ctypes.c_int32
_lib.lb_diagnostics_noalloc.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int32] * 3 + [_dp, ctypes.c_void_p,
                                                                                    ctypes.POINTER(LbDiag), _dp]
_lib.lb_diagnostics_noalloc.restype = ctypes.c_int32
_lib.lb_energy_budget.argtypes = [_h, ctypes.c_int32, ctypes.POINTER(LbBudget)]
_lib.lb_energy_budget.restype = ctypes.c_int32
_lib.lb_interface_length.argtypes = [_h, ctypes.c_int32, ctypes.POINTER(LbInterface)]
_lib.lb_interface_length.restype = ctypes.c_int32
_lib.lb_components.argtypes = [_h, ctypes.c_int32, ctypes.POINTER(LbTopology)]
_lib.lb_components.restype = ctypes.c_int32
_lib.lb_get_populations.argtypes = [_h, ctypes.c_int32, ctypes.c_void_p]
_lib.lb_get_populations.restype = ctypes.c_int32
_lib.lb_set_populations.argtypes = [_h, ctypes.c_int32, ctypes.c_void_p]
_lib.lb_set_populations.restype = ctypes.c_int32
_lib.lb_time.argtypes = [_h]
_lib.lb_time.restype = ctypes.c_int64
_lib.lb_tile_shape.argtypes = [_h, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
_lib.lb_tile_shape.restype = ctypes.c_int32
_lib.lb_steps_per_pass.argtypes = [_h]
_lib.lb_steps_per_pass.restype = ctypes.c_int32
_lib.lb_tiles_cached.argtypes = [_h]
_lib.lb_tiles_cached.restype = ctypes.c_int32
_lib.lb_storage_scale.argtypes = [_h, ctypes.c_int32, _dp, _dp]
_lib.lb_storage_scale.restype = ctypes.c_int32
_lib.lb_destroy.argtypes = [_h]
_lib.lb_destroy.restype = ctypes.c_int32
_lib.lb_last_error.argtypes = []
_lib.lb_last_error.restype = ctypes.c_char_p

EXPORTS = ("lb_workspace_bytes", "lb_init", "lb_step", "lb_fields", "lb_diagnostics", "lb_diagnostics_noalloc",
           "lb_mixing_width",
           "lb_energy_budget",
           "lb_interface_length", "lb_components",
           "lb_get_populations", "lb_set_populations", "lb_time", "lb_tile_shape",
           "lb_steps_per_pass", "lb_tiles_cached", "lb_storage_scale", "lb_destroy", "lb_last_error")


class LBError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.lb_last_error().decode(errors="replace")
        super().__init__(f"{where}: status {code}: {msg}")


def _check(rc: int, where: str) -> None:
    if rc != LB_OK:
        raise LBError(rc, where)


def last_error() -> str:
    return _lib.lb_last_error().decode(errors="replace")


@dataclass
class Member:
    """One realisation: lattice size, relaxation times, coupling, per-component
    body accelerations and initial densities ([ny][nx] float64).  ``G_wall``
    are the fluid-boundary couplings (G_Ab, G_Bb) of Eq. 6 and ``wall_psi``
    the psi of boundary nodes in Eq. 5 (PSI_MIRROR or PSI_ZERO)."""
    nx: int
    ny: int
    rhoA0: np.ndarray
    rhoB0: np.ndarray
    tau: tuple = (1.0, 1.0)
    G: float = 0.0
    g: tuple = ((0.0, 0.0), (0.0, 0.0))
    G_wall: tuple = (0.0, 0.0)
    wall_psi: int = 0


def _member_struct(m: Member, keep: list) -> LbMember:
    a = np.ascontiguousarray(m.rhoA0, dtype=np.float64)
    b = np.ascontiguousarray(m.rhoB0, dtype=np.float64)
    if a.shape != (m.ny, m.nx) or b.shape != (m.ny, m.nx):
        raise ValueError(f"initial densities must be [{m.ny}][{m.nx}]")
    keep += [a, b]
    s = LbMember()
    s.nx, s.ny = int(m.nx), int(m.ny)
    tau = (m.tau, m.tau) if np.isscalar(m.tau) else m.tau
    s.tau[0], s.tau[1] = float(tau[0]), float(tau[1])
    s.G_AB = float(m.G)
    for c in range(2):
        for d in range(2):
            s.g[c][d] = float(m.g[c][d])
    s.rhoA0 = a.ctypes.data_as(_dp)
    s.rhoB0 = b.ctypes.data_as(_dp)
    s.reserved2[0] = s.reserved2[1] = 0.0
    s.G_wall[0], s.G_wall[1] = float(m.G_wall[0]), float(m.G_wall[1])
    s.wall_psi = int(m.wall_psi)
    s.reserved = 0
    return s


def make_config(members, forcing=FORCE_SHIFT, storage=F64, bc_y=WALLS, diag_trim=10, tile_x=0,
                tile_h=0, graph_chunk=0, steps_per_pass=0):
    """Build an LbConfig; returns (config, keepalive list)."""
    keep: list = []
    arr = (LbMember * len(members))(*[_member_struct(m, keep) for m in members])
    keep.append(arr)
    c = LbConfig()
    c.n_members = len(members)
    c.members = ctypes.cast(arr, ctypes.POINTER(LbMember))
    c.forcing, c.storage, c.bc_y = int(forcing), int(storage), int(bc_y)
    c.diag_trim, c.tile_x, c.tile_h, c.graph_chunk = int(diag_trim), int(tile_x), int(tile_h), int(graph_chunk)
    c.steps_per_pass = int(steps_per_pass)
    return c, keep


def workspace_bytes(members, **kw) -> int:
    c, _keep = make_config(members, **kw)
    n = _lib.lb_workspace_bytes(ctypes.byref(c))
    if n == 0:
        raise LBError(LB_EINVAL, "lb_workspace_bytes")
    return int(n)


class Lattice:
    """An ensemble of lattices advanced together on one GPU.

    The workspace is a torch uint8 tensor on ``device``; work runs on
    ``stream`` (default: torch's current stream of that device)."""

    def __init__(self, members, forcing=FORCE_SHIFT, storage=F64, bc_y=WALLS, diag_trim=10,
                 tile_x=0, tile_h=0, graph_chunk=0, device="cuda", stream=None, poison=False,
                 steps_per_pass=0):
        import torch
        self.members = list(members)
        self.storage, self.forcing, self.bc_y, self.diag_trim = storage, forcing, bc_y, diag_trim
        self.device = torch.device(device)
        cfg, keep = make_config(self.members, forcing, storage, bc_y, diag_trim, tile_x, tile_h, graph_chunk,
                                steps_per_pass)
        nbytes = _lib.lb_workspace_bytes(ctypes.byref(cfg))
        if nbytes == 0:
            raise LBError(LB_EINVAL, "lb_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if poison:
            self.workspace.fill_(0xFF)   # every unwritten double reads as NaN
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace tensor is not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(_lib.lb_init(ctypes.byref(cfg), ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "lb_init")
        self._h = h
        del keep

    # -- state -------------------------------------------------------------
    @property
    def handle(self):
        return self._h

    @property
    def t(self) -> int:
        return int(_lib.lb_time(self._h))

    def tile_shape(self, m: int = 0):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.lb_tile_shape(self._h, m, ctypes.byref(a), ctypes.byref(b)), "lb_tile_shape")
        return a.value, b.value

    @property
    def steps_per_pass(self) -> int:
        n = int(_lib.lb_steps_per_pass(self._h))
        if n < 0:
            raise LBError(n, "lb_steps_per_pass")
        return n

    @property
    def tiles_cached(self) -> bool:
        """True if lb_init took the tile shapes from the persisted cache."""
        n = int(_lib.lb_tiles_cached(self._h))
        if n < 0:
            raise LBError(n, "lb_tiles_cached")
        return bool(n)

    def storage_scale(self, m: int = 0):
        """(scale, weight), each [2][9]: the code scales of the 16-bit modes and
        the factors w_i of the per-site shift (1 and 0 in the other modes)."""
        sc, w = (ctypes.c_double * 18)(), (ctypes.c_double * 18)()
        _check(_lib.lb_storage_scale(self._h, m, sc, w), "lb_storage_scale")
        return np.array(sc[:]).reshape(2, 9), np.array(w[:]).reshape(2, 9)

    def step(self, n: int = 1) -> None:
        _check(_lib.lb_step(self._h, int(n)), "lb_step")

    def fields(self, m: int = 0) -> dict:
        import torch
        mm = self.members[m]
        out = {k: torch.empty((mm.ny, mm.nx), dtype=torch.float64, device=self.device)
               for k in ("rhoA", "rhoB", "ux", "uy")}
        _check(_lib.lb_fields(self._h, m, *[ctypes.c_void_p(out[k].data_ptr()) for k in ("rhoA", "rhoB", "ux", "uy")]),
               "lb_fields")
        return out

    def diagnostics(self, m: int = 0, profile: bool = False, check_finite: bool = True) -> dict:
        d = LbDiag()
        prof = np.zeros(self.members[m].ny) if profile else None
        rc = _lib.lb_diagnostics(self._h, m, ctypes.byref(d), prof.ctypes.data_as(_dp) if profile else None)
        if rc != LB_OK and not (rc == LB_ENONFINITE and not check_finite):
            raise LBError(rc, "lb_diagnostics")
        out = {"t": d.t, "mass_A": d.mass[0], "mass_B": d.mass[1], "Ek": d.Ek, "Ep": d.Ep,
               "buoyancy": d.buoyancy, "omega2": d.omega2, "umax": d.umax, "finite": bool(d.finite)}
        if profile:
            out["phi_profile"] = prof
        return out

    def mixing_width(self, m: int = 0, ref=None) -> dict:
        """Integral width of the mixing layer (lb_mixing): ``width`` and the
        bulk references ``lo``, ``hi`` used (by default those of t = 0)."""
        r = LbMixing()
        rr = None if ref is None else (ctypes.c_double * 2)(float(ref[0]), float(ref[1]))
        _check(_lib.lb_mixing_width(self._h, m, rr, ctypes.byref(r)), "lb_mixing_width")
        return {"t": r.t, "width": r.width, "lo": r.bulk_ref[0], "hi": r.bulk_ref[1]}

    def energy_budget(self, m: int = 0) -> dict:
        """Terms of the kinetic-energy balance (lb_budget): pb, korteweg,
        ktau, viscous, eta, buoyancy and t."""
        b = LbBudget()
        _check(_lib.lb_energy_budget(self._h, m, ctypes.byref(b)), "lb_energy_budget")
        return {k: getattr(b, k) for k, _ in LbBudget._fields_}

    def interface_length(self, m: int = 0) -> dict:
        """Interface crossings n0, n90, n45, n135 and Cauchy-Crofton length
        of phi = 0 inside the trimmed domain (lb_interface)."""
        r = LbInterface()
        _check(_lib.lb_interface_length(self._h, m, ctypes.byref(r)), "lb_interface_length")
        c = list(r.crossings)
        return {"t": r.t, "n0": c[0], "n90": c[1], "n45": c[2], "n135": c[3], "length": r.length}

    def components(self, m: int = 0) -> dict:
        """Connected components of phi > 0 ("A") and phi <= 0 ("B") inside
        the trimmed domain (lb_topology)."""
        r = LbTopology()
        _check(_lib.lb_components(self._h, m, ctypes.byref(r)), "lb_components")
        return {"t": r.t, "A": r.components[0], "B": r.components[1]}

    def get_populations(self, m: int = 0):
        import torch
        mm = self.members[m]
        f = torch.empty((2, 9, mm.ny, mm.nx), dtype=torch.float64, device=self.device)
        _check(_lib.lb_get_populations(self._h, m, ctypes.c_void_p(f.data_ptr())), "lb_get_populations")
        return f

    def set_populations(self, f, m: int = 0) -> None:
        mm = self.members[m]
        if tuple(f.shape) != (2, 9, mm.ny, mm.nx) or not f.is_contiguous():
            raise ValueError("populations must be a contiguous (2, 9, ny, nx) float64 device tensor")
        if str(f.dtype) != "torch.float64":
            raise ValueError("populations must be float64")
        _check(_lib.lb_set_populations(self._h, m, ctypes.c_void_p(f.data_ptr())), "lb_set_populations")
        self._keep_f = f   # keep alive until the stream has consumed it

    def synchronize(self) -> None:
        self.stream.synchronize()

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _check(_lib.lb_destroy(self._h), "lb_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

