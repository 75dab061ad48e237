"""Tile variants and the FFT schedule autotuner."""
import itertools
import os

import numpy as np
import pytest

from conftest import oracle_problem
from oracle import model as o_model
from oracle import newton as o_newton
from paper_0911_1407_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

COL_VARIANTS = (0, 1, 3, 4, 5, 6)  # column-pass tiles (2, narrow, is for batches)
TABLES = (0, 1, 2)  # 1/lambda per mode, radial shells, per mode through the kx mirror


@pytest.mark.parametrize("n", [(128, 128, 128), (256, 192, 512)])
def test_every_variant_matches_oracle(n):
    from paper_0911_1407_amd import binding
    box = tuple(8.0 * v for v in n)
    inst = synth.make_instance(n, box, 1.2, 1.1, 1.3, radius=0.4 * box[0], mask_frac=0.2, seed=2)
    P = oracle_problem(inst)
    plan = binding.Plan(n, box, precision="mixed")
    plan.set_instance(inst)
    rng = np.random.default_rng(4)
    s = inst["s_true"]
    v = rng.standard_normal(n)
    v_hat = np.fft.rfftn(v)
    ref_hat = o_newton.SpectralOps(P).hessvec(o_model.hess_diag(P, s), v_hat)
    ref = o_model.hessvec(P, s, v)
    vt = torch.from_numpy(v_hat).cuda()
    radial = binding.pl_plan_prior_is_radial(plan.h)
    assert radial == (len(set(n)) == 1)
    # the operator's passes: every x (operator) and y column tile (default,
    # wide, split, extra wide, wide split, extra-wide split) under both load
    # policies, then the z variants and the table
    combos = [(0, y, 0, xo, 0, 0, nt) for xo, y, nt in itertools.product(COL_VARIANTS, COL_VARIANTS, (0, 31))]
    combos += [(0, 0, z, 0, 0, tab, 0) for z, tab in itertools.product((0, 1), TABLES)]
    for combo in combos:
        binding.pl_plan_set_variants(plan.h, fp64=combo, fp32=combo)
        plan.grad(s)
        out = plan.hessvec_hat(vt).cpu().numpy()
        assert np.linalg.norm(out - ref_hat) <= 1e-11 * np.linalg.norm(ref_hat), combo
        out32 = plan.hessvec_hat(vt.to(torch.complex64)).cpu().numpy()
        assert np.linalg.norm(out32 - ref_hat) <= 2e-5 * np.linalg.norm(ref_hat), combo
        hv = plan.hessvec(v, s=s).cpu().numpy()
        assert np.linalg.norm(hv - ref) <= 1e-11 * np.linalg.norm(ref), combo
    if len(set(n)) == 1:
        # the Krylov-carrying passes: every x variant and table choice
        # reaches the same MAP (FP64 and mixed)
        ref_s = None
        for xk, tab, nt in itertools.product(COL_VARIANTS, TABLES, (0, 1, 2, 4, 8, 16, 31)):
            combo = (xk, 0, 0, 0, tab, 0, nt)
            binding.pl_plan_set_variants(plan.h, fp64=combo, fp32=combo)
            for prec in (binding.PL_FP64, binding.PL_MIXED):
                sm, info = plan.solve(rtol=1e-10, precision=prec)
                assert info["status"] == 0, (combo, prec, info)
                sm = sm.cpu().numpy()
                if ref_s is None:
                    ref_s = sm
                assert np.linalg.norm(sm - ref_s) <= 1e-7 * np.linalg.norm(ref_s), (combo, prec)


def test_autotune_picks_and_caches(tmp_path):
    from paper_0911_1407_amd import binding
    inst = synth.config_instance("sel256", n=128)
    plan = binding.Plan(inst["n"], inst["box"], precision="mixed")
    plan.set_instance(inst)
    cache = str(tmp_path / "tune.txt")
    v1 = plan.autotune(cache)
    assert os.path.exists(cache)
    lines = [l for l in open(cache) if not l.startswith("#")]
    assert len(lines) == 2  # fp64 and fp32
    # a second plan reads the cache instead of timing
    plan2 = binding.Plan(inst["n"], inst["box"], precision="mixed")
    plan2.set_instance(inst)
    assert plan2.autotune(cache) == v1
    # the tuned plan still solves to the same MAP
    s, info = plan.solve(rtol=1e-8)
    s2, info2 = plan2.solve(rtol=1e-8)
    assert info["status"] == 0 and np.array_equal(s.cpu().numpy(), s2.cpu().numpy())
