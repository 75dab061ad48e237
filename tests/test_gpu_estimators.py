"""Parity of the comparison estimators (section 4.1.1: inverse weighting,
LSQ-Wiener filter) and quality measures (section 4.1.2) with the oracle,
through the C ABI."""
import numpy as np
import pytest

from conftest import oracle_problem
from oracle import wiener
from oracle.grid import Problem
from oracle.newton import SpectralOps
from paper_0911_1407_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _plan(inst, precision="fp64"):
    from paper_0911_1407_amd.binding import Plan
    p = Plan(inst["n"], inst["box"], precision=precision)
    p.set_instance(inst)
    return p


def _inst(n, cell=8.0, seed=0, mask=0.2, nbar=1.1):
    box = tuple(cell * v for v in n)
    blk = 4 if min(n) % 4 == 0 and min(n) >= 8 else 2
    return synth.make_instance(n, box, 1.2, nbar, 1.0, radius=0.4 * box[0], mask_frac=mask, seed=seed, block=blk)


@pytest.mark.parametrize("n", [(8, 8, 8), (16, 16, 16), (16, 24, 32), (48, 48, 48), (96, 96, 96)])
def test_lsq_matches_oracle(n):
    inst = _inst(n)
    P = oracle_problem(inst)
    ref = wiener.lsq_dense(P) if n[0] * n[1] * n[2] <= 4096 else wiener.lsq_pcg(P, rtol=1e-13)[0]
    plan = _plan(inst, "mixed")
    d, info = plan.lsq(rtol=1e-12, max_cg=20000, precision=0)
    assert info["status"] == 0, info
    assert _rel(d.cpu().numpy(), ref) <= 1e-9
    dm, infom = plan.lsq(rtol=1e-8, max_cg=20000, precision=1)
    assert infom["status"] == 0, infom
    assert _rel(dm.cpu().numpy(), ref) <= 1e-6


def test_lsq_ill_conditioned_cells():
    # 2 Mpc/h cells: 1/lambda spans many decades
    n = (32, 32, 32)
    inst = _inst(n, cell=2.0, seed=3)
    P = oracle_problem(inst)
    ref, _ = wiener.lsq_pcg(P, rtol=1e-13)
    plan = _plan(inst)
    d, info = plan.lsq(rtol=1e-12, max_cg=20000)
    assert info["status"] == 0, info
    assert _rel(d.cpu().numpy(), ref) <= 1e-8


def test_lsq_white_prior_closed_form_128():
    n = (128, 128, 128)
    box = (256.0,) * 3
    inst = synth.make_instance(n, box, 1.0, 0.9, 1.0, radius=100.0, mask_frac=0.2, seed=5)
    sigma2 = 0.6
    inst["pk"] = np.full(inst["pk"].shape, sigma2 * box[0] ** 3 / (n[0] * n[1] * n[2]))
    inst["amp"] = 1.0
    inst["inv_p0"] = 1.0 / sigma2
    ref = (inst["counts"] - inst["nbar"] * inst["w"]) / (1.0 / sigma2 + inst["nbar"] * inst["w"])
    plan = _plan(inst)
    d, info = plan.lsq(rtol=1e-13, max_cg=200)
    assert info["status"] == 0, info
    assert np.abs(d.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()


def test_inverse_weight_and_measures():
    n = (32, 48, 16)
    inst = _inst(n, mask=0.3)
    P = oracle_problem(inst)
    plan = _plan(inst)
    iw = plan.inverse_weight().cpu().numpy()
    ref = wiener.inverse_weight(P)
    assert np.all(iw[P.w == 0] == 0.0)
    assert np.abs(iw - ref).max() <= 1e-14 * np.abs(ref).max()
    truth = np.expm1(inst["s_true"])
    r, dist = plan.compare(torch.from_numpy(iw), torch.from_numpy(truth))
    assert abs(r - wiener.corr_coeff(iw, truth)) <= 1e-12
    assert abs(dist - wiener.euclidean_distance(iw, truth)) <= 1e-12 * wiener.euclidean_distance(iw, truth)
    r0, d0 = plan.compare(torch.from_numpy(truth), torch.from_numpy(truth))
    assert abs(r0 - 1.0) <= 1e-14 and d0 == 0.0


def test_lsq_rejects_mixed_on_fp64_plan_and_empty_problem():
    from paper_0911_1407_amd.binding import Plan, PLError
    n = (16, 16, 16)
    inst = _inst(n)
    plan = Plan(n, inst["box"])
    with pytest.raises(PLError):
        plan.lsq()
    plan.set_instance(inst)
    with pytest.raises(PLError):
        plan.lsq(precision=1)
