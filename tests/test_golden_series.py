"""Consistency of the stored oracle energy series of the 2048 x 1024 workload
(tests/golden/energy_series_2048x1024.json, written by make_energy_series.py
from the FP64 CPU oracle only) against what the method fixes whatever the
flow does: each component's mass is conserved by the step (Eq. 1 with
streaming and bounce-back walls; FP64 rounding accumulates to about 1e-12
over 20000 steps), and both forcing schemes start from the same state, whose
averages do not depend on the scheme (the diagnostic velocity of f = w_i rho
is half the force over the density, the same under both), so their t = 0
samples are identical."""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "energy_series_2048x1024.json")


def _load():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_series_layout():
    g = _load()
    assert (g["nx"], g["ny"], g["steps"], g["every"]) == (2048, 1024, 20000, 100)
    for name in ("shift", "guo"):
        s = g["series"][name]
        assert s["t"] == list(range(0, 20001, 100))
        for k in ("mass_A", "mass_B", "Ek", "Ep", "buoyancy", "omega2", "umax", "width"):
            assert len(s[k]) == 201 and np.all(np.isfinite(s[k])), (name, k)


def test_series_conserves_each_mass():
    g = _load()
    for name in ("shift", "guo"):
        s = g["series"][name]
        for k in ("mass_A", "mass_B"):
            m = np.array(s[k])
            assert np.max(np.abs(m - m[0])) / m[0] < 5e-12, (name, k)


def test_series_share_the_initial_state():
    g = _load()
    a, b = g["series"]["shift"], g["series"]["guo"]
    for k in ("mass_A", "mass_B", "Ek", "Ep", "buoyancy", "omega2", "umax", "width"):
        assert a[k][0] == b[k][0], k
    assert a["bulk_ref"] == b["bulk_ref"]
    # the initial velocity is the half-force term only: small, not zero
    assert 0.0 < a["umax"][0] < 0.05
    # the flow develops: the mixing layer grows under both schemes
    assert a["width"][-1] > a["width"][0] and b["width"][-1] > b["width"][0]
