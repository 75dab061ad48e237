"""Pins for the oracle MAP solvers (section 3.1 Newton-Raphson / Krylov step,
eq. New5), against dense Newton and closed forms."""
import numpy as np
import pytest

from conftest import oracle_problem
from oracle import closed_form, model, newton
from oracle.grid import Problem
from paper_0911_1407_amd import synth


def white_problem(n, box, sigma2, nbar, beta, seed, mask=0.3):
    """Problem whose prior eigenvalues all equal sigma2 (inv_p0 = 1/sigma2)."""
    inst = synth.make_instance(n, box, 1.0, nbar, beta, radius=box[0] * 0.5, mask_frac=mask,
                               seed=seed, block=2)
    ncell = n[0] * n[1] * n[2]
    vol = box[0] * box[1] * box[2]
    pk = np.full(inst["pk"].shape, sigma2 * vol / ncell)
    return Problem(n, box, inst["w"], inst["counts"], pk, 1.0, -0.4, nbar, beta, 1.0 / sigma2)


@pytest.mark.parametrize("beta", [1.0, 1.5])
def test_dense_newton_matches_lambert_w(beta):
    p = white_problem((8, 8, 8), (16.0,) * 3, 0.8, 1.3, beta, seed=2)
    s, info = newton.newton_dense(p)
    ref = closed_form.white_prior_map(mu=p.mu, sigma2=0.8, beta=beta, nbar=p.nbar, w=p.w, counts=p.counts)
    assert np.abs(s - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n,beta", [((8, 8, 8), 1.2), ((32, 32, 32), 1.0), ((24, 16, 32), 1.5)])
def test_krylov_matches_lambert_w(n, beta):
    p = white_problem(n, (2.0 * n[0], 2.0 * n[1], 2.0 * n[2]), 1.7, 0.6, beta, seed=4)
    s, info = newton.newton_krylov(p, rtol=1e-13, max_newton=60)
    ref = closed_form.white_prior_map(mu=p.mu, sigma2=1.7, beta=beta, nbar=p.nbar, w=p.w, counts=p.counts)
    assert info["status"] == "ok"
    assert np.linalg.norm(s - ref) <= 1e-12 * np.linalg.norm(ref)


def test_krylov_matches_dense_newton_8():
    inst = synth.make_instance((8, 8, 8), (25.0,) * 3, 1.0, 1.0, 1.3, radius=10.0, mask_frac=0.2,
                               seed=5, block=2)
    p = oracle_problem(inst)
    sd, i1 = newton.newton_dense(p)
    sk, i2 = newton.newton_krylov(p, rtol=1e-12)
    assert i2["status"] == "ok"
    assert np.linalg.norm(sd - sk) <= 1e-10 * np.linalg.norm(sd)


@pytest.mark.slow
def test_krylov_matches_dense_newton_16():
    inst = synth.make_instance((16,) * 3, (50.0,) * 3, 1.2, 0.7, 1.0, radius=20.0, mask_frac=0.2,
                               seed=1, block=4)
    p = oracle_problem(inst)
    sd, _ = newton.newton_dense(p)
    sk, i2 = newton.newton_krylov(p, rtol=1e-12)
    assert np.linalg.norm(sd - sk) <= 1e-10 * np.linalg.norm(sd)


@pytest.mark.parametrize("beta", [1.0, 1.6])
def test_uniform_data_closed_form(beta):
    n, box = (16, 16, 16), (40.0,) * 3
    inst = synth.make_instance(n, box, 1.0, 1.0, beta, seed=0)
    p = Problem(n, box, np.full(n, 0.3), np.full(n, 3.0), inst["pk"], inst["amp"], -0.5, 2.0, beta, 0.0)
    s, info = newton.newton_krylov(p, rtol=1e-13)
    expect = closed_form.uniform_data_map(3.0, 2.0, 0.3, beta)
    assert np.abs(s - expect).max() <= 1e-13 * max(1.0, abs(expect)) * 10


@pytest.mark.parametrize("inv_p0", [0.0, 2.5])
def test_zero_completeness_gives_prior_mean(inv_p0, rng):
    n, box = (16, 16, 16), (40.0,) * 3
    inst = synth.make_instance(n, box, 1.0, 1.0, 1.0, seed=0)
    p = Problem(n, box, np.zeros(n), np.zeros(n), inst["pk"], inst["amp"], -0.5, 2.0, 1.0, inv_p0)
    s0 = -0.5 + 0.3 * rng.standard_normal(n)
    s, info = newton.newton_krylov(p, s0=s0, rtol=1e-13)
    expect = closed_form.zero_completeness_map(s0, -0.5, inv_p0)
    assert np.abs(s - expect).max() <= 1e-10
    # from s0 = mu no iteration is needed (the gradient vanishes)
    s2, info2 = newton.newton_krylov(p, rtol=1e-13)
    assert info2["newton_its"] == 0 and np.all(s2 == -0.5)


def test_map_properties_on_selection_workload():
    inst = synth.config_instance("sel256", n=32)
    p = oracle_problem(inst)
    s, s_hat, info = newton.newton_krylov(p, rtol=1e-11, return_hat=True)
    assert info["status"] == "ok"
    ops = newton.SpectralOps(p)
    _, e, g_hat = ops.grad(s_hat)
    _, _, g0_hat = ops.grad(ops.fwd(np.full(p.n, p.mu)))
    # vanishing gradient at the MAP (spectral evaluation)
    assert ops.norm(g_hat) <= 1e-11 * ops.norm(g0_hat)
    # k = 0 component of the gradient: total expected counts equal total counts
    assert abs(e.sum() - p.counts.sum()) <= 1e-10 * p.counts.sum()
    # masked cells carry no data: the MAP there is the prior's conditional mean,
    # finite and below the data-dominated peaks
    assert np.all(np.isfinite(s))


def test_not_converged_and_info():
    inst = synth.config_instance("plain32")
    p = oracle_problem(inst)
    s, info = newton.newton_krylov(p, rtol=1e-8, max_newton=1)
    assert info["status"] == "not_converged" and info["newton_its"] == 1


@pytest.mark.parametrize("name", ["bias256", "sel256"])
def test_preconditioner_changes_path_not_map(name):
    # the workloads' recipes at 32^3: the 25th-percentile preconditioner
    # constant takes a different (shorter) CG path to the same MAP and the
    # same adjoint solution as the mean-diagonal one (H is positive definite)
    from oracle import adjoint
    inst = synth.config_instance(name, n=32)
    p = oracle_problem(inst)
    s1, i1 = newton.newton_krylov(p, rtol=1e-11, max_cg=5000, precond="mean")
    s2, i2 = newton.newton_krylov(p, rtol=1e-11, max_cg=5000, precond="p25")
    assert i1["status"] == "ok" and i2["status"] == "ok"
    assert i1["cg_its"] != i2["cg_its"]
    assert np.linalg.norm(s1 - s2) <= 1e-9 * np.linalg.norm(s1)
    dL = 2.0 * (s1 - inst["s_true"])
    l1, _ = adjoint.adjoint_pcg(p, s1, dL, rtol=1e-12, max_cg=20000, precond="mean")
    l2, _ = adjoint.adjoint_pcg(p, s1, dL, rtol=1e-12, max_cg=20000, precond="p25")
    assert np.linalg.norm(l1 - l2) <= 1e-9 * np.linalg.norm(l1)
