"""The paper-literal Krylov step (section 3.1, eq. New5) with nonlinear-CG
search vectors: it reaches the unique MAP of the oracle, through the C ABI."""
import numpy as np
import pytest

from conftest import oracle_problem
from oracle import closed_form
from oracle import newton as o_newton
from paper_0911_1407_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _plan(inst):
    from paper_0911_1407_amd.binding import Plan
    p = Plan(inst["n"], inst["box"])
    p.set_instance(inst)
    return p


@pytest.mark.parametrize("n,cell,beta", [((16, 16, 16), 8.0, 1.3), ((32, 32, 32), 2.0, 1.0),
                                         ((24, 32, 16), 4.0, 1.5)])
def test_nlcg_reaches_the_oracle_map(n, cell, beta):
    box = tuple(cell * v for v in n)
    inst = synth.make_instance(n, box, 1.2, 1.1, beta, radius=0.4 * box[0], mask_frac=0.2, seed=2, block=4)
    P = oracle_problem(inst)
    ref, _ = o_newton.newton_krylov(P, rtol=1e-12, max_newton=200, max_cg=5000)
    plan = _plan(inst)
    s, info = plan.solve_nlcg(rtol=1e-11, max_cg=50000)
    assert info["status"] == 0, info
    assert info["rel_grad"] <= 1e-11
    assert info["hvps"] == info["cg_its"]
    assert _rel(s.cpu().numpy(), ref) <= 1e-6


def test_nlcg_white_prior_closed_form():
    n, box, sigma2 = (64, 64, 64), (128.0,) * 3, 0.7
    inst = synth.make_instance(n, box, 1.0, 0.8, 1.4, radius=50.0, mask_frac=0.2, seed=3, block=8)
    pk = np.full(inst["pk"].shape, sigma2 * np.prod(box) / np.prod(n))
    plan = _plan(inst)
    plan.set_problem(inst["w"], inst["counts"], pk, 1.0, -0.3, 0.8, 1.4, 1.0 / sigma2)
    s, info = plan.solve_nlcg(rtol=1e-12, max_cg=5000)
    assert info["status"] == 0, info
    ref = closed_form.white_prior_map(mu=-0.3, sigma2=sigma2, beta=1.4, nbar=0.8, w=inst["w"], counts=inst["counts"])
    assert _rel(s.cpu().numpy(), ref) <= 1e-10


def test_nlcg_matches_newton_krylov_on_selection_workload():
    inst = synth.config_instance("sel256", n=64)
    plan = _plan(inst)
    s_n, info_n = plan.solve(rtol=1e-10, max_newton=200, max_cg=5000)
    s_c, info_c = plan.solve_nlcg(rtol=1e-10, max_cg=50000)
    assert info_n["status"] == 0 and info_c["status"] == 0, (info_n, info_c)
    assert _rel(s_c.cpu().numpy(), s_n.cpu().numpy()) <= 1e-7


def test_nlcg_rejects_mixed_and_unset_problem():
    from paper_0911_1407_amd.binding import Plan, PLError
    inst = synth.config_instance("plain32")
    plan = Plan(inst["n"], inst["box"])
    with pytest.raises(PLError):
        plan.solve_nlcg()
    plan.set_instance(inst)
    with pytest.raises(PLError):
        plan.solve_nlcg(precision=1)
    s, info = plan.solve_nlcg(rtol=1e-8)
    assert info["status"] == 0, info
