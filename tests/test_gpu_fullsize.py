"""Parity at the production size, in the launch configuration the benchmark
times (pass and tile shape chosen by timing; graphs of a few steps so that a
graph replay is exercised, then one more step so that both the fused
two-step pass and the single step run): 10000 x 5000, FP64, velocity shift
forcing, 32 random interface modes.  Every density and velocity of the
lattice is compared with the oracle's, and the densities of the FP32, FP16S
and BF16S lattices (each in the configuration the benchmark times) with the
bound their storage rounding implies."""
import numpy as np
import pytest

import oracle
from paper_2101_04847_amd import inputs

pytestmark = pytest.mark.gpu


UNIT_ROUNDOFF = {"f32": 2.0 ** -24, "f16s": 2.0 ** -11, "bf16s": 2.0 ** -8}
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def _residual_band(f, rows):
    """max over the sites of rows [a, b) (away from the walls) of
    sum_j |f*_j - w_j rho*| and of sum_j |f*_j| for the stored values
    f*_j(z) = f_j(z + c_j) of the canonical state f."""
    a, b = rows
    blk = f[:, :, a - 1:b + 1]
    v = np.empty((2, 9, b - a, f.shape[3]))
    for j in range(9):
        v[:, j] = np.roll(blk[:, j], -CX[j], axis=2)[:, 1 + CY[j]:1 + CY[j] + (b - a)]
    rho = v.sum(axis=1, keepdims=True)
    return float(np.max(np.abs(v - W[None, :, None, None] * rho).sum(axis=1))), float(np.max(np.abs(v).sum(axis=1)))


def _bound(states, rows, storage, scale):
    """Rounding bound of the stored values over the given oracle states (one
    store per state): 2 u max sum_j |d_j| per 16-bit store, u max sum_j |f*_j|
    per FP32 store, plus 8 FP32 roundings per collision; relative to scale.
    The residuals vanish in the bulk at rest, so their maximum lies in the
    band of rows around the interface that `rows` covers."""
    u = UNIT_ROUNDOFF[storage]
    acc = 0.0
    for k, f in enumerate(states):
        d, a = _residual_band(f, rows)
        acc += (u * a if storage == "f32" else 2.0 * u * d) + (8 * 2.0 ** -24 * a if k else 0.0)
    return acc / scale


@pytest.mark.timeout(900)
def test_production_size():
    """FP64 in the benchmark's launch configuration (the pass and band of the
    timing search) with a graph of 10 steps (three three-step passes and a
    single step) replayed once and one more single step: every density and
    velocity after 11 steps against the oracle.  Then FP32 (fused pass),
    FP16S and BF16S (single step, 256-column tiles) in their timed
    configurations after three steps, each within its rounding bound."""
    import torch
    from paper_2101_04847_amd import lb
    assert torch.cuda.is_available()
    wl = inputs.LARGE_10000x5000
    print("[case] full size", wl.nx, wl.ny, flush=True)
    rA, rB = wl.densities()
    m = lb.Member(wl.nx, wl.ny, rA, rB, tau=(wl.tau, wl.tau), G=wl.G, g=wl.gravity)
    lat = lb.Lattice([m], storage=lb.F64, graph_chunk=10)
    print("[case] steps per pass", lat.steps_per_pass, "tile shape", lat.tile_shape(), flush=True)
    lat.step(11)
    fg = lat.fields(0)
    fg = {k: v.cpu().numpy() for k, v in fg.items()}
    dg = lat.diagnostics(0)
    ig = lat.interface_length(0)
    hg = lat.mixing_width(0)
    lat.close()
    del lat
    torch.cuda.empty_cache()
    reduced = {}
    for name, st in (("f32", lb.F32), ("f16s", lb.F16S), ("bf16s", lb.BF16S)):
        lr = lb.Lattice([m], storage=st, graph_chunk=2)
        print("[case] full size", name, "steps per pass", lr.steps_per_pass, "tile shape", lr.tile_shape(), flush=True)
        lr.step(3)
        reduced[name] = {k: v.cpu().numpy() for k, v in lr.fields(0).items() if k in ("rhoA", "rhoB")}
        lr.close()
        del lr
        torch.cuda.empty_cache()

    p = oracle.Params(nx=wl.nx, ny=wl.ny, tau=(wl.tau, wl.tau), G=wl.G, g=wl.gravity)
    f = oracle.fill_equilibrium(p, rA, rB)
    # rows around the interface (the only non-bulk rows over a few steps)
    mixed = np.where(np.any((rA > 0.06) & (rA < 1.04), axis=1))[0]
    rows = (int(mixed.min()) - 10, int(mixed.max()) + 11)
    states = [f.copy()]
    for _ in range(3):
        oracle.run_inplace(p, f, 1)
        states.append(f.copy())
    m3 = oracle.macro(p, f)
    scale = max(np.max(np.abs(m3["rhoA"])), np.max(np.abs(m3["rhoB"])))
    # errors measured on the MI355X (deterministic for a build); the bar is
    # four times these, inside the rounding bound (ratios 8 to 12)
    measured = {"f32": 1.39e-7, "f16s": 4.22e-5, "bf16s": 3.75e-4}
    for name in ("f32", "f16s", "bf16s"):
        b = _bound(states, rows, name, scale)
        err = max(np.max(np.abs(reduced[name][k] - m3[k])) for k in ("rhoA", "rhoB")) / scale
        print(f"[case] {name} density max rel err {err:.3e}, rounding bound {b:.3e} (ratio {b / err:.1f})", flush=True)
        assert err <= b, (name, err, b)
        assert err <= 4.0 * measured[name], (name, err)
    del states
    oracle.run_inplace(p, f, 8)
    mo = oracle.macro(p, f)
    do = oracle.diagnostics(p, f, trim=10, profile=True)
    del f
    for k in ("rhoA", "rhoB", "ux", "uy"):
        err = np.max(np.abs(fg[k] - mo[k])) / np.max(np.abs(mo[k]))
        print(f"[case] {k} max rel err {err:.3e}", flush=True)
        assert err <= 1e-12, k
    from oracle import interface, mixing
    io = interface.interface_length(mo["rhoA"], mo["rhoB"], 10)
    for k in ("n0", "n90", "n45", "n135", "length"):
        assert ig[k] == io[k], k
    assert dg["mass_A"] == pytest.approx(do["mass_A"], rel=1e-12)
    assert dg["Ek"] == pytest.approx(do["Ek"], rel=1e-12)
    assert abs(dg["umax"] - do["umax"]) <= 1e-12 * do["umax"]
    lo, hi = hg["lo"], hg["hi"]
    assert hg["width"] == pytest.approx(mixing.mixing_width(do["phi_profile"], lo, hi, 10), rel=1e-10)


@pytest.mark.timeout(600)
def test_production_size_wetting_walls_three_steps():
    """The same lattice with wetting walls (G_Ab = 0.05, G_Bb = -0.05, psi = 0
    on boundary nodes: the wetting kernel variant), three steps, every
    density and velocity against the oracle."""
    import torch
    from paper_2101_04847_amd import lb
    wl = inputs.LARGE_10000x5000
    print("[case] full size wetting", wl.nx, wl.ny, flush=True)
    rA, rB = wl.densities()
    gw = (0.05, -0.05)
    m = lb.Member(wl.nx, wl.ny, rA, rB, tau=(wl.tau, wl.tau), G=wl.G, g=wl.gravity, G_wall=gw,
                  wall_psi=lb.PSI_ZERO)
    lat = lb.Lattice([m], storage=lb.F64, graph_chunk=2)
    lat.step(3)
    fg = {k: v.cpu().numpy() for k, v in lat.fields(0).items()}
    lat.close()
    del lat
    torch.cuda.empty_cache()
    p = oracle.Params(nx=wl.nx, ny=wl.ny, tau=(wl.tau, wl.tau), G=wl.G, g=wl.gravity, G_wall=gw,
                      wall_psi=oracle.PSI_ZERO)
    f = oracle.fill_equilibrium(p, rA, rB)
    oracle.run_inplace(p, f, 3)
    mo = oracle.macro(p, f)
    del f
    for k in ("rhoA", "rhoB", "ux", "uy"):
        err = np.max(np.abs(fg[k] - mo[k])) / np.max(np.abs(mo[k]))
        print(f"[case] {k} max rel err {err:.3e}", flush=True)
        assert err <= 1e-12, k


@pytest.mark.timeout(600)
def test_paper_parameters_full_size_three_steps():
    """The configuration of the paper-parameter runs (10000 x 5000, tau = 0.53,
    G = 0.1381, g = 9e-6, a white-noise interface of amplitude 4 on a tanh
    profile of the paper's bulk densities 1.0 / 0.1), pass and band chosen by
    timing: three steps, every density and velocity against the oracle."""
    import torch
    from paper_2101_04847_amd import lb
    nx, ny, tau, G, g = 10000, 5000, 0.53, 0.1381, 9e-6
    print("[case] full size, paper parameters", nx, ny, tau, G, g, flush=True)
    yp = np.linspace(-30.0, 30.0, 241)
    s = 0.5 * (1.0 + np.tanh(yp / 2.0))
    rA, rB = inputs.profile_densities(nx, ny, inputs.white_noise_height(nx, ny, 9, 4.0), yp,
                                      0.1 + 0.9 * s, 0.1 + 0.9 * (1.0 - s))
    gg = ((0.0, -g), (0.0, g))
    m = lb.Member(nx, ny, rA, rB, tau=(tau, tau), G=G, g=gg)
    lat = lb.Lattice([m], storage=lb.F64, graph_chunk=2)
    print("[case] steps per pass", lat.steps_per_pass, "tile shape", lat.tile_shape(), flush=True)
    lat.step(3)
    fg = {k: v.cpu().numpy() for k, v in lat.fields(0).items()}
    lat.close()
    del lat
    torch.cuda.empty_cache()
    p = oracle.Params(nx=nx, ny=ny, tau=(tau, tau), G=G, g=gg)
    f = oracle.fill_equilibrium(p, rA, rB)
    oracle.run_inplace(p, f, 3)
    mo = oracle.macro(p, f)
    del f
    for k in ("rhoA", "rhoB", "ux", "uy"):
        err = np.max(np.abs(fg[k] - mo[k])) / np.max(np.abs(mo[k]))
        print(f"[case] {k} max rel err {err:.3e}", flush=True)
        assert err <= 1e-12, k
