"""The 2048 x 1024 workload (32 seeded modes, tau = 1, G = 1.5, g = 1e-5) run
for 20000 steps on the GPU under both forcing schemes, its energy-budget
averages, max |u| and mixing width every 100 steps against the series the
FP64 CPU oracle wrote (tests/golden/energy_series_2048x1024.json, made by
tests/golden/make_energy_series.py, which calls only the oracle).

The FP64 step matches the oracle bit for bit, so the series differ only by
the summation order of the averages (the oracle's compensated serial sums,
the GPU's fixed reduction tree): each sample must agree to 1e-12 of the
largest magnitude the quantity takes over the run (measured: 3e-15 or less,
max |u| exactly)."""
import json
import os

import numpy as np
import pytest

from paper_2101_04847_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "energy_series_2048x1024.json")
KEYS = ("mass_A", "mass_B", "Ek", "Ep", "buoyancy", "omega2", "umax", "width")


@pytest.fixture(scope="module")
def lb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2101_04847_amd import lb as mod
    return mod


@pytest.mark.timeout(600)
@pytest.mark.parametrize("forcing", ["shift", "guo"])
def test_series_2048x1024_20000_steps(lb, forcing):
    with open(GOLDEN) as fh:
        gold = json.load(fh)
    ref = gold["series"][forcing]
    wl = inputs.MEDIUM_2048x1024
    assert (gold["nx"], gold["ny"], gold["seed"], gold["G"], gold["g"], gold["tau"]) == \
        (wl.nx, wl.ny, wl.seed, wl.G, wl.g, wl.tau)
    print("[case] series", wl.name, forcing, flush=True)
    rA, rB = wl.densities()
    m = lb.Member(wl.nx, wl.ny, rA, rB, tau=(wl.tau, wl.tau), G=wl.G, g=wl.gravity)
    lat = lb.Lattice([m], forcing=lb.FORCE_SHIFT if forcing == "shift" else lb.FORCE_GUO, storage=lb.F64,
                     graph_chunk=100, diag_trim=gold["trim"])
    every = gold["every"]
    got = {k: [] for k in KEYS}
    for t in ref["t"]:
        lat.step(t - lat.t)
        d = lat.diagnostics(0)
        for k in KEYS[:-1]:
            got[k].append(d[k])
        got["width"].append(lat.mixing_width(0)["width"])
        if t % (50 * every) == 0:
            print(f"[case] t = {t}", flush=True)
    lat.close()
    worst = {}
    for k in KEYS:
        a, b = np.array(got[k]), np.array(ref[k])
        scale = np.max(np.abs(b))
        worst[k] = float(np.max(np.abs(a - b)) / scale)
    print("[case] largest difference / largest magnitude:", worst, flush=True)
    for k, v in worst.items():
        assert v <= 1e-12, (k, v)
