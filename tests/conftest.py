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


def assert_elementwise(got, ref, tol, floor=1e-2, what=""):
    """Every element within tol of the reference, in units of
    max(|ref_i|, floor * max|ref|) (complex arrays by modulus): a wrong value
    confined to small entries (masked cells, a Nyquist plane, the ragged
    edge of a tile) cannot hide under a norm.  Returns the worst error in
    units of the bound (<= 1)."""
    a = np.asarray(got)
    b = np.asarray(ref)
    assert a.shape == b.shape, (a.shape, b.shape)
    mag = np.abs(b)
    scale = np.maximum(mag, floor * float(mag.max()))
    worst = float(np.max(np.abs(a.astype(np.complex128) - b) / (tol * scale))) if mag.max() > 0 else \
        float(np.abs(a).max())
    print(f"elementwise {what}: worst error {worst:.3f} of the bound (tol {tol:g}, floor {floor:g})", flush=True)
    assert worst <= 1.0, (what, worst)
    return worst
