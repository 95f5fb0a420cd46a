import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU physics check (still part of the CPU suite)")


def paper_value(key):
    """A number the paper prints (tests/golden/paper_values.json, with its
    citation there)."""
    import json
    with open(os.path.join(ROOT, "tests", "golden", "paper_values.json")) as fh:
        return json.load(fh)[key]["value"]


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle
