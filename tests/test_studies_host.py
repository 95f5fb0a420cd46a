"""Host logic of the study summaries (no GPU): the paper-run tables with and
without the members that fail before the end of the run."""
import math

from paper_2101_04847_amd import studies


def _series(t, base, fail_at=None):
    d = {"t": t}
    for k in studies.SUMMARY_KEYS:
        d[k] = [base + 0.5 * j for j in range(len(t))]
        if fail_at is not None:
            for j in range(fail_at, len(t)):
                d[k][j] = math.nan
    return d


def test_summary_separates_failed_members():
    t = list(range(0, 90001, 1000))
    runs = [{"case": "immiscible", "G": 0.1381, "storage": "f64", "seed0": 4,
             "members": [_series(t, 1.0), _series(t, 3.0)]},
            {"case": "immiscible", "G": 0.1381, "storage": "f64", "seed0": 9,
             "members": [_series(t, 8.0, fail_at=t.index(85000))]}]
    out = studies.summarise_paper_runs(runs)["immiscible"]
    assert out["members"] == 3 and out["finite_to_end"] == 2
    assert out["last_finite_t"] == {"4": 90000, "5": 90000, "9": 84000}
    j = t.index(80000)
    row = out["tables"]["80000"]["h"]
    # survivors: members 4 and 5 only
    assert row["survivors"]["n"] == 2 and math.isclose(row["survivors"]["mean"], 2.0 + 0.5 * j)
    # finite at t = 80000: the failed member still counts
    assert row["finite_at_t"]["n"] == 3 and math.isclose(row["finite_at_t"]["mean"], 4.0 + 0.5 * j)
    # after its failure only the survivors remain
    assert out["tables"]["90000"]["h"]["finite_at_t"]["n"] == 2


def test_markdown_tables_show_both_member_sets():
    t = list(range(0, 90001, 1000))
    runs = [{"case": "miscible", "G": 0.0805, "storage": "f64", "seed0": 0,
             "members": [_series(t, 100.0), _series(t, 300.0, fail_at=t.index(85000))]}]
    md = studies.paper_tables_markdown(studies.summarise_paper_runs(runs))
    lines = md.splitlines()
    assert lines[0].startswith("miscible (G = 0.0805, f64; 1 of 2 members finite to the end)")
    j = t.index(80000)
    h_end = next(ln for ln in lines if ln.startswith("| mixing width h | finite to end |")).split(" | ")
    h_all = next(ln for ln in lines if ln.startswith("| mixing width h | finite at t |")).split(" | ")
    # column 80 000 is the 8th sample column; cells carry the member count where not all members count
    assert h_end[2 + 7] == f"{100 + 0.5 * j:.0f} ± 0 [1]"
    assert h_all[2 + 7] == f"{200 + 0.5 * j:.0f} ± 100"
    assert "last finite sample of the failed members (seed: t): 1: 84000" in lines


def _closed_form_run(gamma=0.0068, nx=10000, ny=5000):
    """A member whose series satisfy Eq. 17 and Eq. 22 exactly and whose
    Korteweg flux is gamma times the rate of change of the interface length
    per unit area, with a known growth-rate peak and dip and a first
    topology change at t = 23000."""
    import numpy as np
    t = np.arange(0, 90001, 1000, dtype=np.float64)
    slope = np.where(t < 30000, 5.0, np.where(t < 35000, 9.0, np.where(t < 45000, 3.0, 6.0)))
    length = 100.0 + np.concatenate([[0.0], np.cumsum(slope[:-1] * 1000.0)])
    area = nx * (ny - 2 * studies.TRIM)
    kort = gamma * np.gradient(length, t) / area
    n = len(t)
    pb, ktau, buoy = -1e-9 * np.ones(n), 2e-11 * np.ones(n), -3e-8 * (1 + t / 9e4)
    eta, visc = 0.01 * np.ones(n), -2e-9 * (1 + 0.5 * np.sin(t / 7e3))
    rhs = -pb - kort - ktau + visc - buoy
    ek = 1e-6 + np.concatenate([[0.0], np.cumsum(0.5 * (rhs[1:] + rhs[:-1]) * np.diff(t))])
    d = {"t": t.tolist(), "Ek": ek.tolist(), "pb": pb.tolist(), "korteweg": kort.tolist(), "ktau": ktau.tolist(),
         "viscous": visc.tolist(), "buoyancy": buoy.tolist(), "eta": eta.tolist(), "omega2": (-visc / eta).tolist(),
         "length": length.tolist(), "comp_A": [1 if x < 23000 else 4 for x in t], "comp_B": [1] * n,
         "h": (10 + t / 100).tolist(), "Ep": [0.01] * n, "umax": [0.1] * n}
    return {"case": "immiscible", "G": 0.1381, "storage": "f64", "seed0": 0, "params": {"nx": nx, "ny": ny},
            "members": [d]}


def test_paper_analysis_closed_forms():
    out = studies.summarise_paper_runs([_closed_form_run()])["immiscible"]
    a = out["analysis"]
    assert a["members"] == 1
    assert a["eq17_residual_rel"]["max"] < 1e-12
    assert a["eq22"]["max_rel_diff"] < 1e-14 and abs(a["eq22"]["integral_ratio_min"] - 1) < 1e-14
    assert a["length_rate"] == {"peak_t": 31000, "peak": 9.0, "dip_t": 44000, "dip": 3.0}
    assert math.isclose(a["eq21_gamma_fit"]["mean"], 0.0068, rel_tol=1e-12)
    assert a["eq21_gamma_fit"]["correlation_mean"] > 1 - 1e-12
    assert out["first_split_t"] == {"0": 23000}
    # the integrated terms: buoyancy grows linearly, so its integral over
    # [10000, 90000] is -3e-8 (80000 + (90000^2 - 10000^2) / 1.8e5)
    assert math.isclose(a["eq17_integrals"]["-buoyancy"], 3e-8 * (80000 + (90000 ** 2 - 10000 ** 2) / 1.8e5),
                        rel_tol=1e-12)


def test_paper_analysis_sees_a_dropped_term():
    run = _closed_form_run()
    m = run["members"][0]
    m["pb"] = [-v for v in m["pb"]]              # a sign error in one flux
    a = studies.summarise_paper_runs([run])["immiscible"]["analysis"]
    assert a["eq17_residual_rel"]["max"] > 1e-2
