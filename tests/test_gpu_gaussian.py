"""MAP of the Gaussian-prior model (section 2.2, unit bias, eq. MAPG) on the
GPU against the oracle, through the C ABI."""
import numpy as np
import pytest

from conftest import oracle_problem
from oracle import gaussian
from oracle import newton as o_newton
from oracle.grid import Problem
from paper_0911_1407_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _inst(n, cell, seed=0, inv_p0=0.5, nbar=1.3):
    box = tuple(cell * v for v in n)
    inst = synth.make_instance(n, box, 1.0, nbar, 1.0, radius=0.45 * box[0], mask_frac=0.2, seed=seed, block=4)
    inst["inv_p0"] = inv_p0
    return inst


def _plan(inst, precision="fp64"):
    from paper_0911_1407_amd.binding import Plan
    p = Plan(inst["n"], inst["box"], precision=precision)
    p.set_instance(inst)
    return p


@pytest.mark.parametrize("n,cell", [((8, 8, 8), 8.0), ((32, 32, 32), 4.0), ((16, 24, 32), 2.0)])
def test_gaussian_map_matches_oracle(n, cell):
    inst = _inst(n, cell)
    P = oracle_problem(inst)
    ref, _ = gaussian.newton_dense(P) if np.prod(n) <= 512 else gaussian.newton_spectral(P, rtol=1e-13)
    plan = _plan(inst, "mixed")
    d, info = plan.solve_gaussian(rtol=1e-11, max_newton=200, max_cg=5000, precision=0)
    assert info["status"] == 0, info
    assert _rel(d.cpu().numpy(), ref) <= 1e-7
    dm, infom = plan.solve_gaussian(rtol=1e-8, max_newton=200, max_cg=5000, precision=1)
    assert infom["status"] == 0, infom
    assert _rel(dm.cpu().numpy(), ref) <= 1e-4


def test_gaussian_white_prior_closed_form_and_eq_mapg():
    n, box, sigma2 = (64, 64, 64), (128.0,) * 3, 0.6
    inst = synth.make_instance(n, box, 1.0, 1.2, 1.0, radius=50.0, mask_frac=0.2, seed=3, block=8)
    inst["pk"] = np.full(inst["pk"].shape, sigma2 * np.prod(box) / np.prod(n))
    inst["amp"] = 1.0
    inst["inv_p0"] = 1.0 / sigma2
    plan = _plan(inst)
    d, info = plan.solve_gaussian(rtol=1e-12)
    assert info["status"] == 0, info
    ref = gaussian.white_prior_map(sigma2, inst["nbar"], inst["w"], inst["counts"])
    assert _rel(d.cpu().numpy(), ref) <= 1e-10
    # the paper's equation, through S, on a correlated prior
    inst2 = _inst((32, 32, 32), 4.0, seed=6, inv_p0=0.8)
    plan2 = _plan(inst2)
    d2, info2 = plan2.solve_gaussian(rtol=1e-12, max_newton=200, max_cg=5000)
    assert info2["status"] == 0, info2
    P2 = oracle_problem(inst2)
    dn = d2.cpu().numpy()
    assert np.linalg.norm(gaussian.mapg_residual(P2, dn)) <= 1e-8 * np.linalg.norm(dn)


def test_gaussian_domain_and_model_reset():
    from paper_0911_1407_amd.binding import PLError
    inst = _inst((16, 16, 16), 8.0, seed=2)
    plan = _plan(inst)
    start = np.zeros(inst["n"])
    start[inst["counts"] > 0] = -2.0
    with pytest.raises(PLError):
        plan.solve_gaussian(delta0=start)
    # a lognormal solve on the same plan after a Gaussian one is unaffected
    s_before, _ = plan.solve(rtol=1e-11)
    plan.solve_gaussian(rtol=1e-10)
    s_after, info = plan.solve(rtol=1e-11)
    assert info["status"] == 0, info
    assert np.array_equal(s_before.cpu().numpy(), s_after.cpu().numpy())
    P = oracle_problem(inst)
    ref, _ = o_newton.newton_krylov(P, rtol=1e-12)
    assert _rel(s_after.cpu().numpy(), ref) <= 1e-6
