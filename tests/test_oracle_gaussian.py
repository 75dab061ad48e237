"""Pins for the oracle's Gaussian-prior MAP (section 2.2, unit bias,
eq. MAPG)."""
import numpy as np
import pytest
from scipy.stats import poisson

from conftest import oracle_problem
from oracle import gaussian
from oracle.grid import Problem
from paper_0911_1407_amd import synth


def _prob(n=(8, 8, 8), box=(64.0,) * 3, seed=3, mask=0.25, nbar=1.5, inv_p0=0.5):
    inst = synth.make_instance(n, box, 1.0, nbar, 1.0, radius=box[0] * 0.6, mask_frac=mask, seed=seed, block=2)
    inst["inv_p0"] = inv_p0
    return oracle_problem(inst)


def _white(n, box, sigma2, nbar, seed, mask=0.3):
    inst = synth.make_instance(n, box, 1.0, nbar, 1.0, radius=box[0] * 0.5, mask_frac=mask, seed=seed, block=2)
    pk = np.full(inst["pk"].shape, sigma2 * np.prod(box) / np.prod(n))
    return Problem(n, box, inst["w"], inst["counts"], pk, 1.0, 0.0, nbar, 1.0, 1.0 / sigma2)


def test_likelihood_matches_poisson_logpmf(rng):
    # -ln L = sum_i [lam_i - N_i ln lam_i + ln N_i!] with lam = nbar w (1 + delta);
    # differences in delta of the oracle's likelihood part equal those of logpmf
    p = _prob()
    d1 = 0.3 * rng.standard_normal(p.n)
    d2 = 0.3 * rng.standard_normal(p.n)
    pos = p.w > 0

    def nll(d):
        return -np.sum(poisson.logpmf(p.counts[pos], (p.nbar * p.w * (1.0 + d))[pos]))

    def lik(d):
        return gaussian.objective(p, d) - 0.5 * float(np.sum(d * gaussian.model.prior_apply(p, d)))

    assert lik(d1) - lik(d2) == pytest.approx(nll(d1) - nll(d2), rel=1e-10)


def test_gradient_matches_fd(rng):
    p = _prob()
    d = 0.2 * rng.standard_normal(p.n)
    g = gaussian.gradient(p, d)
    for _ in range(3):
        v = rng.standard_normal(p.n)
        h = 1e-6
        fd = (gaussian.objective(p, d + h * v) - gaussian.objective(p, d - h * v)) / (2 * h)
        assert fd == pytest.approx(float(np.sum(g * v)), rel=1e-6)
    # Hessian diagonal term = central FD of the likelihood gradient
    e = np.zeros(p.n)
    e[1, 2, 3] = 1.0
    h = 1e-6
    fd = (gaussian.gradient(p, d + h * e) - gaussian.gradient(p, d - h * e)) / (2 * h)
    from oracle import model
    assert fd[1, 2, 3] == pytest.approx(model.prior_apply(p, e)[1, 2, 3] + gaussian.hess_diag(p, d)[1, 2, 3],
                                        rel=1e-6)


@pytest.mark.parametrize("n", [(8, 8, 8), (32, 32, 32)])
def test_white_prior_closed_form(n):
    p = _white(n, tuple(2.0 * v for v in n), 0.6, 1.2, seed=4)
    ref = gaussian.white_prior_map(0.6, p.nbar, p.w, p.counts)
    d, _ = gaussian.newton_spectral(p, rtol=1e-13)
    assert np.abs(d - ref).max() <= 1e-11 * np.abs(ref).max()
    if n[0] == 8:
        dd, _ = gaussian.newton_dense(p)
        assert np.abs(dd - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n", [(8, 8, 8), (16, 16, 16)])
def test_map_solves_eq_mapg_and_solvers_agree(n):
    p = _prob(n=n, box=(4.0 * n[0],) * 3, mask=0.3, seed=5)
    dd, _ = gaussian.newton_dense(p)
    ds, _ = gaussian.newton_spectral(p, rtol=1e-13)
    assert np.linalg.norm(ds - dd) <= 1e-9 * np.linalg.norm(dd)
    # the paper's form of the MAP equation, applied through S itself
    assert np.linalg.norm(gaussian.mapg_residual(p, dd)) <= 1e-9 * np.linalg.norm(dd)
    assert np.all((1.0 + dd)[p.counts > 0] > 0)
