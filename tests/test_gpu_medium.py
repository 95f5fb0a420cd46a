"""Parity on the 2048 x 1024 Rayleigh-Taylor workload (32 seeded interface
modes, tau = 1, G = 1.5, g = 1e-5) to 1000 steps, in the configuration the
library chooses by timing (pass and tiles) with 100-step graphs, for both
forcing schemes: the energy-budget series every 100 steps and the final
populations against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_2101_04847_amd import inputs

pytestmark = pytest.mark.gpu

KEYS = ("mass_A", "mass_B", "Ek", "Ep", "buoyancy", "omega2", "umax")


@pytest.mark.parametrize("forcing", [0, 1], ids=["shift", "guo"])
def test_medium_1000_steps_series(forcing):
    import torch
    from paper_2101_04847_amd import lb
    assert torch.cuda.is_available()
    wl = inputs.MEDIUM_2048x1024
    print("[case] medium", wl.nx, wl.ny, "guo" if forcing else "shift", flush=True)
    rA, rB = wl.densities()
    m = lb.Member(wl.nx, wl.ny, rA, rB, tau=(wl.tau, wl.tau), G=wl.G, g=wl.gravity)
    lat = lb.Lattice([m], forcing=forcing, storage=lb.F64, graph_chunk=100, poison=True)
    print("[case] steps per pass", lat.steps_per_pass, "tile", lat.tile_shape(), flush=True)
    p = oracle.Params(nx=wl.nx, ny=wl.ny, tau=(wl.tau, wl.tau), G=wl.G, g=wl.gravity, forcing=forcing)
    f = oracle.fill_equilibrium(p, rA, rB)
    worst = 0.0
    for t in range(100, 1001, 100):
        lat.step(100)
        oracle.run_inplace(p, f, 100)
        dg = lat.diagnostics(0)
        do = oracle.diagnostics(p, f, trim=10)
        # |difference| <= 1e-12 * (mean of |terms|): the averages with signed
        # terms (E_p, buoyancy flux) cancel, so their own size is no scale
        mo = oracle.macro(p, f)
        D = slice(10, wl.ny - 10)
        rho = mo["rhoA"] + mo["rhoB"]
        yj = (np.arange(wl.ny) - 0.5 * (wl.ny - 1))[:, None]
        fy = mo["rhoA"] * p.g[0][1] + mo["rhoB"] * p.g[1][1]
        scale = {"mass_A": np.sum(mo["rhoA"]), "mass_B": np.sum(mo["rhoB"]),
                 "Ek": np.mean((0.5 * rho * (mo["ux"] ** 2 + mo["uy"] ** 2))[D]),
                 "Ep": np.mean(np.abs(yj * fy)[D]), "buoyancy": np.mean(np.abs(mo["uy"] * fy)[D]),
                 "omega2": do["omega2"], "umax": do["umax"]}
        for k in KEYS:
            err = abs(dg[k] - do[k]) / scale[k]
            worst = max(worst, err)
            assert err <= 1e-12, (t, k, dg[k], do[k])
        assert dg["t"] == t and dg["finite"]
    fg = lat.get_populations(0).cpu().numpy()
    err = float(np.max(np.abs(fg - f)) / np.max(np.abs(f)))
    print(f"[case] worst series rel err {worst:.3e}; populations at t = 1000 max rel err {err:.3e}", flush=True)
    assert err <= 1e-12
    lat.close()
