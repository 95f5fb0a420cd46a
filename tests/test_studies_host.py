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
