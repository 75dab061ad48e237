"""Full-size parity with the CPU oracle at the workloads the benchmark is
quoted on, through the C ABI.

The oracle's MAP and adjoint at 256^3 take many minutes of host CPU, so they
are stored (``tests/golden/*.json``, written by ``tests/golden/make_golden.py``,
which calls only the oracle and the seeded input generator): the MAP s* at
a seeded sample of cells plus structurally special ones (masked cells, the
largest counts, the extremes of s*), full-field sums, and the adjoint
derivatives.  Each test first recomputes the input fingerprint stored beside
them, so a generator that drew different inputs fails loudly instead of
comparing different problems.

Checks per workload:

* cell by cell, |gpu - oracle| <= tol * max(|oracle|, 1e-2 max|oracle|) on
  every stored cell, and the relative L2 error over the sample;
* full-field sum and sum of squares against the oracle's (a necessary
  condition of rel-L2 <= tol over the whole field);
* the oracle's own spectral gradient evaluated at the solver's spectral
  iterate (``pl_newton_krylov_solve_hat``): ||g|| <= rtol ||g0||, the
  roundoff-free statement that the returned field is the MAP to the
  requested tolerance (the real field carries an FFT-roundoff floor
  amplified by max 1/lambda ~ 1e12).

Tolerances: plain FP64 rel <= 1e-6, mixed (FP32 FFT/HVP, FP64 sums) <= 1e-4,
against the oracle solved to ||g|| / ||g0|| <= 1e-10.  Both the tight solves
(rtol 1e-10) and the benchmark's configuration solves (rtol 1e-6) are
checked; the relative L2 errors are printed per configuration.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from conftest import oracle_problem
from oracle.newton import SpectralOps
from paper_0911_1407_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TUNE_CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_0911_1407_amd",
                          "tune_cache_gfx950.txt")


def _golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


def _check_inputs(inst, ref):
    fp = ref["inputs"] if "inputs" in ref else ref
    sha = hashlib.sha256(np.ascontiguousarray(inst["counts"]).tobytes()).hexdigest()
    assert sha == fp["counts_sha256"], "the generator drew different counts than the stored oracle run"
    assert float(np.sum(inst["w"])) == pytest.approx(fp["w_sum"], rel=1e-12)
    assert float(np.sum(inst["s_true"])) == pytest.approx(fp["s_true_sum"], rel=1e-10, abs=1e-6)
    assert float(np.sum(inst["s_true"] ** 2)) == pytest.approx(fp["s_true_sumsq"], rel=1e-12)


def cell_compare(got, cells, ref_cells, tol, floor=1e-2):
    """Element-wise bound on the stored cells; returns (sample rel-L2, worst
    error in units of the bound)."""
    ref = np.asarray(ref_cells, dtype=np.float64)
    a = np.asarray(got, dtype=np.float64).ravel()[np.asarray(cells)]
    scale = np.maximum(np.abs(ref), floor * np.abs(ref).max())
    worst = float(np.max(np.abs(a - ref) / (tol * scale)))
    rel = float(np.linalg.norm(a - ref) / np.linalg.norm(ref))
    return rel, worst


def stats_compare(got, ref_stats, tol):
    x = np.asarray(got, dtype=np.float64)
    n2 = float(np.sum(x * x))
    # ||x|| within tol of ||ref|| and the sum within tol ||ref|| sqrt(N)
    assert abs(np.sqrt(n2) - np.sqrt(ref_stats["sumsq"])) <= tol * np.sqrt(ref_stats["sumsq"])
    assert abs(float(np.sum(x)) - ref_stats["sum"]) <= tol * np.sqrt(ref_stats["sumsq"] * x.size)


def oracle_rel_grad(inst, s_hat):
    """||g(s_hat)|| / ||g(F mu)|| with the oracle's spectral gradient."""
    P = oracle_problem(inst)
    ops = SpectralOps(P)
    g0 = ops.norm(ops.grad(ops.fwd(np.full(P.n, P.mu)))[2])
    g = ops.norm(ops.grad(np.asarray(s_hat))[2])
    return g / g0


def _plan(inst):
    from paper_0911_1407_amd.binding import Plan
    plan = Plan(inst["n"], inst["box"], precision="mixed")
    plan.set_instance(inst)
    plan.autotune(TUNE_CACHE)
    return plan


@pytest.fixture(scope="module")
def sel256():
    inst = synth.config_instance("sel256")
    ref = _golden("sel256_map")
    _check_inputs(inst, ref)
    print("sel256: inputs match the stored oracle run", flush=True)
    return inst, ref


@pytest.fixture(scope="module")
def bias256():
    if not os.path.exists(os.path.join(GOLDEN, "bias256_map.json")):
        pytest.skip("tests/golden/bias256_map.json not written (make_golden.py bias256 runs for hours)")
    inst = synth.config_instance("bias256")
    ref = _golden("bias256_map")
    _check_inputs(inst, ref)
    print("bias256: inputs match the stored oracle run", flush=True)
    return inst, ref


# (precision, stopping tolerance, bound on the field error vs the oracle).
# Tight solves carry the parity bar: 1e-6 (FP64) and 1e-4 (mixed).  At the
# benchmark's stopping tolerance 1e-6 the gradient residual, amplified by the
# smallest Hessian eigenvalues (~1/lambda in the masked blocks), leaves a
# field error of ~1.6e-6 (FP64) / ~1.2e-6 (mixed) in relative L2 and up to
# ~3e-4 in single cells; there the binding check is the oracle's gradient
# at the returned iterate (<= rtol ||g0||) and the field error is reported
# against a 1e-5 / 1e-3 bound.  rtol 2e-7 brings the FP64 field within 1e-6.
MAP_CASES = [("fp64", 1e-10, 1e-6, 1e-6), ("mixed", 1e-10, 1e-4, 1e-4), ("fp64", 2e-7, 1e-6, 1e-4),
             ("fp64", 1e-6, 1e-5, 1e-3), ("mixed", 1e-6, 1e-5, 1e-3)]


@pytest.mark.parametrize("prec,rtol,tol,tol_cell", MAP_CASES)
def test_map_256_selection_workload_matches_oracle(sel256, prec, rtol, tol, tol_cell):
    inst, ref = sel256
    plan = _plan(inst)
    s, s_hat, info = plan.solve(want_hat=True, rtol=rtol, precision=0 if prec == "fp64" else 1, max_newton=200,
                                max_cg=5000)
    assert info["status"] == 0 and info["rel_grad"] <= rtol, info
    got = s.cpu().numpy()
    rel, worst = cell_compare(got, ref["cells"], ref["s_star_cells"], tol_cell)
    print(f"sel256 {prec} rtol {rtol:g}: rel-L2 vs oracle (sample of {len(ref['cells'])}) {rel:.3e}, "
          f"worst cell {worst:.3f} of the {tol_cell:g} bound, fp64 steps {info['fp64_steps']}, "
          f"newton {info['newton_its']} cg {info['cg_its']}", flush=True)
    assert worst <= 1.0 and rel <= tol
    stats_compare(got, ref["s_star"], tol)
    rg = oracle_rel_grad(inst, s_hat.cpu().numpy())
    print(f"sel256 {prec} rtol {rtol:g}: oracle ||g||/||g0|| at the returned iterate {rg:.3e}", flush=True)
    assert rg <= 1.05 * rtol
    if prec == "mixed" and rtol == 1e-6:
        # the benchmark's mixed configuration runs every Newton step in FP32
        assert info["fp64_steps"] == 0, info


def test_map_and_adjoint_256_bias_workload_match_oracle(bias256):
    # beta = 1.5, nbar = 2: forward MAP, then the adjoint of
    # L = sum (s* - s_true)^2 with respect to A, beta, nbar and N (along the
    # stored direction u), FP64 and mixed, against the oracle's adjoint at
    # the oracle MAP
    inst, ref = bias256
    plan = _plan(inst)
    s, s_hat, info = plan.solve(want_hat=True, rtol=1e-10, precision=0, max_newton=200, max_cg=5000)
    assert info["status"] == 0, info
    got = s.cpu().numpy()
    rel, worst = cell_compare(got, ref["cells"], ref["s_star_cells"], 1e-6)
    print(f"bias256 fp64 MAP: rel-L2 vs oracle {rel:.3e}, worst cell {worst:.3f} of the bound", flush=True)
    assert worst <= 1.0 and rel <= 1e-6
    stats_compare(got, ref["s_star"], 1e-6)
    assert oracle_rel_grad(inst, s_hat.cpu().numpy()) <= 1.05e-10
    st = torch.from_numpy(inst["s_true"]).cuda()
    adj = ref["adjoint"]
    u = np.random.default_rng(adj["u_seed"]).choice([-1.0, 1.0], size=inst["n"])
    u = np.where(inst["counts"] > 0, u, 0.0)
    for prec, rtol, tol in (("fp64", 1e-10, 1e-6), ("mixed", 1e-10, 1e-4), ("mixed", 1e-6, 1e-4)):
        grads, ainfo = plan.adjoint(s, 2.0 * (s - st), want_fields=True, rtol=rtol,
                                    precision=0 if prec == "fp64" else 1, max_cg=50000)
        assert ainfo["status"] == 0, ainfo
        dN_u = float(np.sum(grads["N"].cpu().numpy() * u))
        errs = {
            "A": abs(grads["A"] - adj["dL_dA"]) / abs(adj["dL_dA"]),
            "beta": abs(grads["beta"] - adj["dL_dbeta"]) / abs(adj["dL_dbeta"]),
            "nbar": abs(grads["nbar"] - adj["dL_dnbar"]) / abs(adj["dL_dnbar"]),
            "N.u": abs(dN_u - adj["dL_dN_dot_u"]) / abs(adj["dL_dN_dot_u"]),
        }
        # lambda solves H(s*) lambda = 2 (s* - s_true) at each side's own MAP
        # (3e-9 apart): that difference, amplified by H's conditioning,
        # lands in the cells where lambda is small, so the cell floor is a
        # tenth of max|lambda| (a tile or index error gives O(1) errors)
        lrel, lworst = cell_compare(grads["lam"].cpu().numpy(), ref["cells"], adj["lambda_cells"], tol, floor=0.1)
        print(f"bias256 adjoint {prec} rtol {rtol:g}: rel errors vs oracle {errs}, lambda rel-L2 {lrel:.3e} "
              f"(worst cell {lworst:.3f} of the bound), cg {ainfo['cg_its']}", flush=True)
        for k, e in errs.items():
            assert e <= tol, (prec, rtol, k, e)
        assert lrel <= tol and lworst <= 1.0


def test_adjoint_256_bias_workload_matches_central_fd(bias256):
    # central differences of L(s*(theta)) at relative step 1e-5 on A and
    # beta, and along the stored direction u of the counts (step 1e-3),
    # through FP64 GPU solves, against the FP64 adjoint.  The counts enter
    # the gradient linearly, so s*(N) is smooth and the O(h^2) truncation
    # stays near 1e-6 at h = 1e-3; at h = 1e-5 the change of L (about 0.2)
    # sinks into the spread of two MAP solves stopped at rtol 1e-12
    inst, ref = bias256
    plan = _plan(inst)
    st = torch.from_numpy(inst["s_true"]).cuda()
    base = dict(w=inst["w"], counts=inst["counts"], pk=inst["pk"], amp=inst["amp"], mu=inst["mu"],
                nbar=inst["nbar"], beta=inst["beta"])
    adj = ref["adjoint"]
    u = np.random.default_rng(adj["u_seed"]).choice([-1.0, 1.0], size=inst["n"])
    u = np.where(inst["counts"] > 0, u, 0.0)

    def L_at(**over):
        prm = dict(base)
        prm.update(over)
        plan.set_problem(**prm)
        s, info = plan.solve(rtol=1e-12, precision=0, max_newton=200, max_cg=10000)
        assert info["status"] == 0, info
        return float(torch.sum((s - st) ** 2))

    plan.set_problem(**base)
    s, info = plan.solve(rtol=1e-12, precision=0, max_newton=200, max_cg=10000)
    grads, ainfo = plan.adjoint(s, 2.0 * (s - st), want_fields=True, rtol=1e-12, precision=0, max_cg=50000)
    assert ainfo["status"] == 0, ainfo
    dN_u = float(np.sum(grads["N"].cpu().numpy() * u))
    for key, name, h in (("amp", "A", 1e-5 * inst["amp"]), ("beta", "beta", 1e-5 * inst["beta"])):
        fd = (L_at(**{key: inst[key] + h}) - L_at(**{key: inst[key] - h})) / (2 * h)
        print(f"bias256 dL/d{name}: adjoint {grads[name]:.10e} central FD {fd:.10e} "
              f"rel {abs(grads[name] - fd) / abs(fd):.2e}", flush=True)
        assert abs(grads[name] - fd) <= 1e-4 * abs(fd), (name, grads[name], fd)
    h = 1e-3
    fd = (L_at(counts=inst["counts"] + h * u) - L_at(counts=inst["counts"] - h * u)) / (2 * h)
    print(f"bias256 dL/dN . u: adjoint {dN_u:.10e} central FD {fd:.10e} rel {abs(dN_u - fd) / abs(fd):.2e}",
          flush=True)
    assert abs(dN_u - fd) <= 1e-4 * abs(fd)


@pytest.mark.parametrize("prec,rtol,tol", [("fp64", 1e-10, 1e-6), ("mixed", 1e-6, 1e-4)])
def test_batch_workload_64_instances_match_oracle(prec, rtol, tol):
    # all 64 instances of the batched workload against the oracle, cell by
    # cell on each instance's stored sample
    from paper_0911_1407_amd.binding import Batch
    ref = _golden("batch64_map")
    insts = synth.batch_instances(count=64)
    for inst, r in zip(insts, ref["instances"]):
        assert list(inst["n"]) == r["n"]
        _check_inputs(inst, r)
    b = Batch(insts, precision="mixed")
    s_list, infos = b.solve(rtol=rtol, precision=0 if prec == "fp64" else 1, max_newton=200, max_cg=5000)
    rels, worsts = [], []
    for i, (s, info, r) in enumerate(zip(s_list, infos, ref["instances"])):
        assert info["status"] == 0 and info["rel_grad"] <= rtol, (i, info)
        rel, worst = cell_compare(s.cpu().numpy(), r["cells"], r["s_star_cells"], tol)
        stats_compare(s.cpu().numpy(), r["s_star"], tol)
        rels.append(rel)
        worsts.append(worst)
    print(f"batch64 {prec} rtol {rtol:g}: max rel-L2 vs oracle over 64 instances {max(rels):.3e}, "
          f"worst cell {max(worsts):.3f} of the bound, fp64 steps {sum(i['fp64_steps'] for i in infos)}",
          flush=True)
    assert max(rels) <= tol and max(worsts) <= 1.0
