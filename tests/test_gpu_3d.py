"""GPU (gfx950) parity of the 3D (D3Q19) step against the FP64 3D oracle.

FP64 populations, densities and velocities must match oracle/orc3.c to
1e-12 relative (the kernels evaluate its expressions in the same order, so
the match is usually exact) on lattices that are ragged for the 64 x 4
thread blocks, with walls and with periodic y, tau_A != tau_B, gravity and a
3D drop; the diagnostics agree with sums of the oracle's fields; populations
round-trip through set/get; FP32 storage stays within its rounding bound.
"""
import numpy as np
import pytest

from oracle import lb3 as orc3

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def lb3():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2101_04847_amd import lb3 as mod
    return mod


def _say(*a):
    print("[case]", *a, flush=True)


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


def _drop(nx, ny, nz, R=5.0):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = np.sqrt((x - nx / 2 + 0.3) ** 2 + (y - ny / 3 + 0.2) ** 2 + (z - nz / 2 - 0.4) ** 2) - R
    s = 0.5 * (1 - np.tanh(d / 1.5))
    return 0.06 + s, 0.06 + 0.95 * (1 - s)


CASES = [
    # nx, ny, nz, periodic y, tau, G, g
    (70, 13, 9, False, (1.0, 0.8), 1.4, 1e-4),
    (70, 13, 9, True, (0.9, 0.9), 1.2, 1e-4),
    (3, 5, 3, False, (1.0, 1.0), 1.0, 0.0),
    (64, 4, 7, True, (0.7, 1.1), 0.9, 2e-4),
    (130, 21, 5, False, (0.53, 0.53), 0.1381, 1e-5),      # the paper's immiscible tau and G
]


@pytest.mark.parametrize("two_pass", [False, True], ids=["fused", "two-pass"])
@pytest.mark.parametrize("nx,ny,nz,per,tau,G,g", CASES)
def test_3d_matches_oracle(lb3, nx, ny, nz, per, tau, G, g, two_pass):
    _say("3d", nx, ny, nz, "periodic_y" if per else "walls", "tau", tau, "G", G, "g", g,
         "two-pass" if two_pass else "fused")
    R = min(5.0, 0.35 * min(nx, ny, nz))
    rA, rB = _drop(nx, ny, nz, R)
    gg = ((2e-5, -g, 1e-5), (0.0, g, 0.0))
    lat = lb3.Lattice3(nx, ny, nz, rA, rB, tau=tau, G=G, g=gg, bc_y=lb3.PERIODIC_Y if per else lb3.WALLS,
                       poison=True, two_pass=two_pass)
    p = orc3.Params3(nx=nx, ny=ny, nz=nz, tau=tau, G=G, g=gg, periodic_y=per)
    f = orc3.fill_equilibrium(p, rA, rB)
    assert _rel(lat.get_populations().cpu().numpy(), f) <= TOL
    t = 0
    for target in (1, 20, 61):
        f = orc3.run(p, f, target - t)
        assert np.isfinite(f).all(), "the oracle run itself is not finite: an unstable case"
        lat.step(target - t)
        t = target
        assert lat.t == t
        err = _rel(lat.get_populations().cpu().numpy(), f)
        assert err <= TOL, (target, err)
    mg = {k: v.cpu().numpy() for k, v in lat.fields().items()}
    mo = orc3.macro(p, f)
    for k in ("rhoA", "rhoB", "ux", "uy", "uz"):
        assert _rel(mg[k], mo[k]) <= TOL, k
    lat.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("per", [False, True], ids=["walls", "periodic_y"])
def test_3d_fused_equals_two_pass(lb3, per, storage):
    """The fused pass and the two-pass step agree bit for bit (both storage
    modes), over nine z bands (the last one ragged), tiles ragged in x and
    y."""
    nx, ny, nz = 130, 45, 70
    _say("3d fused vs two-pass", nx, ny, nz, "periodic_y" if per else "walls", storage)
    rA, rB = _drop(nx, ny, nz, R=9.0)
    gg = ((0.0, -1e-4, 0.0), (0.0, 1e-4, 0.0))
    kw = dict(tau=(1.0, 0.9), G=1.3, g=gg, bc_y=lb3.PERIODIC_Y if per else lb3.WALLS,
              storage=lb3.F64 if storage == "f64" else lb3.F32)
    a = lb3.Lattice3(nx, ny, nz, rA, rB, two_pass=False, **kw)
    b = lb3.Lattice3(nx, ny, nz, rA, rB, two_pass=True, **kw)
    a.step(50)
    b.step(50)
    assert np.array_equal(a.get_populations().cpu().numpy(), b.get_populations().cpu().numpy())
    a.close()
    b.close()


def test_3d_diagnostics_and_round_trip(lb3):
    import torch
    nx, ny, nz, trim = 48, 20, 12, 3
    _say("3d diagnostics", nx, ny, nz)
    rA, rB = _drop(nx, ny, nz)
    gg = ((0.0, -1e-4, 0.0), (0.0, 1e-4, 0.0))
    lat = lb3.Lattice3(nx, ny, nz, rA, rB, tau=(1.0, 0.9), G=1.3, g=gg, diag_trim=trim)
    p = orc3.Params3(nx=nx, ny=ny, nz=nz, tau=(1.0, 0.9), G=1.3, g=gg)
    lat.step(40)
    f = orc3.run(p, orc3.fill_equilibrium(p, rA, rB), 40)
    d = lat.diagnostics()
    m = orc3.macro(p, f)
    u2 = m["ux"] ** 2 + m["uy"] ** 2 + m["uz"] ** 2
    ek = 0.5 * (m["rhoA"] + m["rhoB"]) * u2
    assert d["t"] == 40 and d["finite"]
    assert abs(d["mass_A"] - m["rhoA"].sum()) <= 1e-12 * m["rhoA"].sum()
    assert abs(d["mass_B"] - m["rhoB"].sum()) <= 1e-12 * m["rhoB"].sum()
    assert abs(d["Ek"] - ek[:, trim:ny - trim, :].mean()) <= 1e-12 * ek[:, trim:ny - trim, :].mean()
    assert abs(d["umax"] - np.sqrt(u2.max())) <= 1e-12 * np.sqrt(u2.max())
    # set / get round trip, and stepping from a set state equals the oracle
    fg = torch.from_numpy(f).to("cuda")
    lat.set_populations(fg)
    assert np.array_equal(lat.get_populations().cpu().numpy(), f)
    lat.step(5)
    assert _rel(lat.get_populations().cpu().numpy(), orc3.run(p, f, 5)) <= TOL
    lat.close()


def test_3d_f32_close_to_oracle(lb3):
    nx, ny, nz = 70, 13, 9
    _say("3d f32")
    rA, rB = _drop(nx, ny, nz)
    gg = ((0.0, -1e-4, 0.0), (0.0, 1e-4, 0.0))
    lat = lb3.Lattice3(nx, ny, nz, rA, rB, tau=(1.0, 1.0), G=1.4, g=gg, storage=lb3.F32)
    p = orc3.Params3(nx=nx, ny=ny, nz=nz, tau=(1.0, 1.0), G=1.4, g=gg)
    f = orc3.fill_equilibrium(p, rA, rB)
    t = 0
    for target, tol in ((1, 5e-7), (100, 2e-5)):
        f = orc3.run(p, f, target - t)
        lat.step(target - t)
        t = target
        mg = {k: v.cpu().numpy() for k, v in lat.fields().items()}
        mo = orc3.macro(p, f)
        for k in ("rhoA", "rhoB"):
            assert _rel(mg[k], mo[k]) <= tol, (target, k, _rel(mg[k], mo[k]))
    lat.close()


def test_3d_medium_lattice(lb3):
    """128 x 64 x 48 with walls, 100 steps: the grid spans many blocks in
    every direction."""
    nx, ny, nz = 128, 64, 48
    _say("3d medium", nx, ny, nz)
    rA, rB = _drop(nx, ny, nz, R=12.0)
    gg = ((0.0, -1e-5, 0.0), (0.0, 1e-5, 0.0))
    lat = lb3.Lattice3(nx, ny, nz, rA, rB, tau=(1.0, 1.0), G=1.5, g=gg)
    p = orc3.Params3(nx=nx, ny=ny, nz=nz, tau=(1.0, 1.0), G=1.5, g=gg)
    lat.step(100)
    f = orc3.run(p, orc3.fill_equilibrium(p, rA, rB), 100)
    mg = {k: v.cpu().numpy() for k, v in lat.fields().items()}
    mo = orc3.macro(p, f)
    for k in ("rhoA", "rhoB", "ux", "uy", "uz"):
        assert _rel(mg[k], mo[k]) <= TOL, k
    lat.close()


@pytest.mark.timeout(900)
def test_3d_bench_size_two_steps(lb3):
    """The benchmark's 3D lattice (384^3, 8 random interface modes, walls,
    tau = 1, G = 1.5, g = 1e-5): two steps of the fused and of the two-pass
    step (equal bit for bit), every density and velocity against the oracle;
    the FP32 lattice's densities within 1e-6."""
    import torch
    from paper_2101_04847_amd import inputs
    w = inputs.D3_384
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    _say("3d bench size", nx, ny, nz)
    rA, rB = inputs.rt3d_densities(nx, ny, nz, w["seed"])
    gg = ((0.0, -w["g"], 0.0), (0.0, w["g"], 0.0))
    lat = lb3.Lattice3(nx, ny, nz, rA, rB, tau=(w["tau"], w["tau"]), G=w["G"], g=gg)
    lat.step(2)
    mg = {k: v.cpu().numpy() for k, v in lat.fields().items()}
    lat.close()
    del lat
    torch.cuda.empty_cache()
    # the two-pass step of the benchmark's two-pass line on the same lattice
    _say("3d bench size, two passes")
    l2 = lb3.Lattice3(nx, ny, nz, rA, rB, tau=(w["tau"], w["tau"]), G=w["G"], g=gg, two_pass=True)
    l2.step(2)
    m2 = {k: v.cpu().numpy() for k, v in l2.fields().items()}
    l2.close()
    del l2
    torch.cuda.empty_cache()
    for k in ("rhoA", "rhoB", "ux", "uy", "uz"):
        assert np.array_equal(m2[k], mg[k]), k
    # the FP32 lattice of the benchmark's FP32 line: densities within the format's bound
    l32 = lb3.Lattice3(nx, ny, nz, rA, rB, tau=(w["tau"], w["tau"]), G=w["G"], g=gg, storage=lb3.F32)
    l32.step(2)
    m32 = {k: v.cpu().numpy() for k, v in l32.fields().items() if k in ("rhoA", "rhoB")}
    l32.close()
    del l32
    torch.cuda.empty_cache()
    p = orc3.Params3(nx=nx, ny=ny, nz=nz, tau=(w["tau"], w["tau"]), G=w["G"], g=gg)
    f = orc3.fill_equilibrium(p, rA, rB)
    orc3.run_inplace(p, f, 2)
    mo = orc3.macro(p, f)
    del f
    for k in ("rhoA", "rhoB", "ux", "uy", "uz"):
        err = _rel(mg[k], mo[k])
        print(f"[case] {k} max rel err {err:.3e}", flush=True)
        assert err <= TOL, k
    for k in ("rhoA", "rhoB"):
        err = _rel(m32[k], mo[k])
        print(f"[case] FP32 {k} max rel err {err:.3e}", flush=True)
        assert err <= 1e-6, k


def test_3d_non_finite_state_is_reported(lb3):
    """A NaN planted in the populations (through set_populations) makes
    lb3_diagnostics report LB_ENONFINITE: the binding raises, or returns
    finite = False when asked not to check."""
    import torch
    from paper_2101_04847_amd.lb import LBError, LB_ENONFINITE
    nx, ny, nz = 20, 10, 6
    _say("3d non-finite detection")
    rA, rB = _drop(nx, ny, nz, R=2.5)
    lat = lb3.Lattice3(nx, ny, nz, rA, rB, tau=(1.0, 1.0), G=1.2)
    assert lat.diagnostics()["finite"]
    f = lat.get_populations()
    f[0, 3, 2, 4, 7] = float("nan")
    lat.set_populations(f)
    with pytest.raises(LBError) as e:
        lat.diagnostics()
    assert e.value.code == LB_ENONFINITE
    assert lat.diagnostics(check_finite=False)["finite"] is False
    torch.cuda.synchronize()
    lat.close()
