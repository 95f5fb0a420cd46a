"""lb_diagnostics_noalloc (the entry point for callers that cannot allocate)
against lb_diagnostics on the same states, through the C ABI: two calls in
a row, the second on a smaller lattice, and the size limit."""
import ctypes

import numpy as np
import pytest

from paper_2101_04847_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2101_04847_amd import lb as mod
    return mod


def _noalloc(lb, lat, m, trim):
    mm = lat.members[m]
    f = lat.fields(m)
    g = (ctypes.c_double * 4)(mm.g[0][0], mm.g[0][1], mm.g[1][0], mm.g[1][1])
    d = lb.LbDiag()
    prof = np.full(mm.ny, np.nan)
    rc = lb._lib.lb_diagnostics_noalloc(*[ctypes.c_void_p(f[k].data_ptr()) for k in ("rhoA", "rhoB", "ux", "uy")],
                                        mm.nx, mm.ny, trim, g, ctypes.c_void_p(lat.stream.cuda_stream),
                                        ctypes.byref(d), prof.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return rc, d, prof


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_noalloc_equals_diagnostics(lb, storage):
    st = {"f64": lb.F64, "f32": lb.F32}[storage]
    runs = [(384, 200, 3, 1.5, 150), (130, 57, 4, 0.5, 77)]   # the second call is smaller
    for nx, ny, seed, G, steps in runs:
        print("[case] noalloc", storage, nx, ny, flush=True)
        rA, rB = inputs.multi_mode(nx, ny, seed)
        g = ((0.0, -1e-4), (2e-6, 1e-4))
        lat = lb.Lattice([lb.Member(nx, ny, rA, rB, tau=(1.0, 1.0), G=G, g=g)], storage=st, diag_trim=10)
        lat.step(steps)
        ref = lat.diagnostics(0, profile=True)
        rc, d, prof = _noalloc(lb, lat, 0, 10)
        assert rc == lb.LB_OK, lb.last_error()
        got = {"mass_A": d.mass[0], "mass_B": d.mass[1], "Ek": d.Ek, "Ep": d.Ep, "buoyancy": d.buoyancy,
               "omega2": d.omega2, "umax": d.umax}
        for k, v in got.items():
            assert v == ref[k], (k, v, ref[k])
        assert d.finite == 1
        assert np.array_equal(prof, ref["phi_profile"])
        lat.close()


def test_noalloc_rejects_sizes_beyond_its_scratch(lb):
    import torch
    ny = lb.NOALLOC_MAX_NY + 1
    buf = torch.zeros(4, dtype=torch.float64, device="cuda")
    g = (ctypes.c_double * 4)()
    d = lb.LbDiag()
    p = ctypes.c_void_p(buf.data_ptr())
    rc = lb._lib.lb_diagnostics_noalloc(p, p, p, p, 1, ny, 10, g, None, ctypes.byref(d), None)
    assert rc == lb.LB_EINVAL and "LB_NOALLOC_MAX_NY" in lb.last_error()
    rc = lb._lib.lb_diagnostics_noalloc(p, p, p, p, 1, 20, 10, g, None, ctypes.byref(d), None)
    assert rc == lb.LB_EINVAL
