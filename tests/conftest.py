import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def oracle_problem(inst):
    """Wrap a generator instance as an oracle Problem."""
    from oracle.grid import Problem
    return Problem(inst["n"], inst["box"], inst["w"], inst["counts"], inst["pk"], inst["amp"],
                   inst["mu"], inst["nbar"], inst.get("beta", 1.0), inst.get("inv_p0", 0.0))


@pytest.fixture
def rng():
    return np.random.default_rng(1234)
