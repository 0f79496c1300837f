import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run through the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def golden_path(name: str) -> str:
    return os.path.join(GOLDEN, name)


@pytest.fixture
def fig2_text():
    with open(golden_path("fig2_circuit.txt")) as f:
        return f.read()
