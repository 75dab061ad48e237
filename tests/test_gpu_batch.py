"""Batched MAP solves (many uneven grids, one launch per pass) against the
oracle and against single-plan solves."""
import numpy as np
import pytest

from conftest import oracle_problem
from oracle import newton as o_newton
from paper_0911_1407_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _mixed_batch():
    insts = synth.batch_instances(count=6, master_seed=5)
    # one instance with selection, mask and bias; one whose gradient vanishes
    insts.append(synth.make_instance((48, 32, 64), (150.0, 100.0, 200.0), 1.3, 1.5, 1.4, radius=60.0,
                                     mask_frac=0.2, seed=9, block=8))
    empty = synth.make_instance((32, 32, 32), (100.0,) * 3, 1.0, 1.0, 1.0, seed=10)
    empty["w"] = np.zeros((32, 32, 32))
    empty["counts"] = np.zeros((32, 32, 32))
    insts.append(empty)
    return insts


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_matches_oracle_and_single(prec):
    from paper_0911_1407_amd.binding import Batch, Plan
    insts = _mixed_batch()
    b = Batch(insts, precision=prec)
    # mixed solves take FP32 Krylov directions; steps that stall at tight
    # tolerances are refined with FP64 inner solves
    s_list, infos = b.solve(rtol=1e-10, max_newton=100, max_cg=2000)
    tol = 1e-6 if prec == "fp64" else 1e-4
    for i, (inst, s, info) in enumerate(zip(insts, s_list, infos)):
        assert info["status"] == 0, (i, info)
        got = s.cpu().numpy()
        if i == len(insts) - 1:
            # all w = 0 from s0 = mu: gradient vanishes, no iteration, s = mu
            assert info["newton_its"] == 0 and np.all(got == inst["mu"])
            continue
        assert info["rel_grad"] <= 1e-10
        ref, _ = o_newton.newton_krylov(oracle_problem(inst), rtol=1e-11)
        assert _rel(got, ref) <= tol, (i, inst["n"])
        if i in (0, 6):
            plan = Plan(inst["n"], inst["box"], precision=prec)
            plan.set_instance(inst)
            s1, info1 = plan.solve(rtol=1e-10, max_cg=2000)
            assert _rel(got, s1.cpu().numpy()) <= tol


def test_batch_workload_64_instances():
    # the batched workload: 64 instances, n in {32, 48, 64, 96}, mixed precision
    from paper_0911_1407_amd.binding import Batch
    from oracle.grid import Problem
    from oracle.model import gradient
    insts = synth.batch_instances(count=64)
    b = Batch(insts, precision="mixed")
    s_list, infos = b.solve(rtol=1e-6)
    for i, info in enumerate(infos):
        assert info["status"] == 0 and info["rel_grad"] <= 1e-6, (i, info)
    # spot-check a few against the oracle solution
    for i in (0, 17, 42, 63):
        ref, _ = o_newton.newton_krylov(oracle_problem(insts[i]), rtol=1e-10)
        assert _rel(s_list[i].cpu().numpy(), ref) <= 1e-4, i


def test_batch_rejects_unsupported_lengths():
    from paper_0911_1407_amd import binding
    with pytest.raises(binding.PLError) as e:
        binding.pl_batch_create([(32, 32, 32), (256, 256, 256)], [(1.0,) * 3] * 2)
    assert e.value.code == binding.PL_ERR_UNSUPPORTED_SIZE
