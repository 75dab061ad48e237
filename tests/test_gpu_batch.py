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


def _arch():
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_tile_variants_give_the_same_map(prec, tmp_path):
    # every combination of default / narrow tiles per length (forced through
    # the schedule cache) reaches the oracle's MAP; the narrow tiles change
    # only which lanes hold which columns, and the partial-sum rounding
    from paper_0911_1407_amd.binding import Batch
    insts = synth.batch_instances(count=5, master_seed=11)
    insts.append(synth.make_instance((48, 32, 64), (150.0, 100.0, 200.0), 1.3, 1.5, 1.4, radius=60.0,
                                     mask_frac=0.2, seed=9, block=8))
    refs = [o_newton.newton_krylov(oracle_problem(it), rtol=1e-11)[0] for it in insts]
    # the library orders lengths by total cells; a cache line must list them
    # in that order, so probe it with an autotune into an empty cache first
    probe = tmp_path / "probe.txt"
    b = Batch(insts, precision="mixed")
    b.autotune(str(probe))
    keys = [l.split() for l in probe.read_text().splitlines() if not l.startswith("#")]
    order = keys[0][3]
    nl = len(order.split(","))
    tol = 1e-6 if prec == "fp64" else 1e-4
    for vc, vr in (("0", "0"), ("2", "2"), ("2", "0"), ("0", "2")):
        cache = tmp_path / f"c{vc}{vr}.txt"
        cache.write_text("".join(f"{_arch()} batch {p} {order} {','.join([vc] * nl)} {','.join([vr] * nl)} 0.0\n"
                                 for p in ("fp64", "fp32")))
        b = Batch(insts, precision="mixed")
        b.autotune(str(cache))
        s_list, infos = b.solve(rtol=1e-10, precision=0 if prec == "fp64" else 1, max_newton=100, max_cg=2000)
        for i, (s, info, ref) in enumerate(zip(s_list, infos, refs)):
            assert info["status"] == 0 and info["rel_grad"] <= 1e-10, (vc, vr, i, info)
            assert _rel(s.cpu().numpy(), ref) <= tol, (vc, vr, i)
        b.close()
