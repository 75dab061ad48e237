"""Pins for the oracle's objective, gradient and Hessian (section 2.1 eqs. 1-3,
section 2.3 log-prior, section 2.4 chain rule, section 3.1.2 gradient and
Hessian of the quadratic form)."""
import numpy as np
import pytest
from scipy.stats import poisson

from conftest import oracle_problem
from oracle import model
from paper_0911_1407_amd import synth


def _prob(beta=1.0, seed=3, n=(8, 8, 8), box=(64.0,) * 3, mask=0.25):
    inst = synth.make_instance(n, box, 1.0, 1.5, beta, radius=box[0] * 0.6, mask_frac=mask,
                               seed=seed, block=2)
    return oracle_problem(inst), inst


def test_likelihood_matches_poisson_logpmf():
    # eq. 1-3: -ln L = sum_i [<N_i> - N_i ln <N_i> + ln N_i!]; the oracle drops
    # sum_i [ln N_i! - N_i ln(nbar w_i)], which does not depend on s
    p, inst = _prob(beta=1.4)
    s = inst["s_true"]
    lam = p.nbar * p.w * np.exp(p.beta * s)
    pos = p.w > 0
    full = -np.sum(poisson.logpmf(p.counts[pos], lam[pos]))
    from scipy.special import gammaln
    const = np.sum(gammaln(p.counts[pos] + 1) - p.counts[pos] * np.log(p.nbar * p.w[pos]))
    assert abs(model.neg_log_likelihood(p, s) - (full - const)) <= 1e-10 * abs(full)


@pytest.mark.parametrize("beta", [1.0, 1.5, 0.7])
def test_gradient_matches_fd_of_objective(beta, rng):
    p, inst = _prob(beta=beta)
    s = inst["s_true"] + 0.1 * rng.standard_normal(p.n)
    g = model.gradient(p, s)
    for _ in range(3):
        v = rng.standard_normal(p.n)
        h = 1e-5
        fd = (model.objective(p, s + h * v) - model.objective(p, s - h * v)) / (2 * h)
        assert abs(fd - np.sum(g * v)) <= 1e-7 * (abs(fd) + np.linalg.norm(g) * np.linalg.norm(v) * 1e-3)


@pytest.mark.parametrize("beta", [1.0, 1.5])
def test_hessvec_matches_fd_of_gradient(beta, rng):
    p, inst = _prob(beta=beta)
    s = inst["s_true"]
    v = rng.standard_normal(p.n)
    h = 1e-6
    fd = (model.gradient(p, s + h * v) - model.gradient(p, s - h * v)) / (2 * h)
    hv = model.hessvec(p, s, v)
    assert np.linalg.norm(fd - hv) <= 1e-7 * np.linalg.norm(hv)


def test_hessian_symmetric_positive(rng):
    p, inst = _prob(beta=1.2)
    s = inst["s_true"]
    u, v = rng.standard_normal(p.n), rng.standard_normal(p.n)
    a = np.sum(u * model.hessvec(p, s, v))
    b = np.sum(v * model.hessvec(p, s, u))
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    assert np.sum(v * model.hessvec(p, s, v)) > 0
    H = model.hessian_dense(p, s)
    assert np.allclose(H @ v.ravel(), model.hessvec(p, s, v).ravel(), rtol=1e-11, atol=1e-11 * np.abs(H).max())
    assert np.linalg.eigvalsh(H).min() > 0


def test_unity_bias_reduces_to_map_equation_of_section_2_4_2(rng):
    # for beta = 1 the likelihood derivative is N - nbar w exp(s) (eq. MAPLNUB)
    p, inst = _prob(beta=1.0)
    s = inst["s_true"]
    np.testing.assert_allclose(model.dloglike_ds(p, s), p.counts - p.nbar * p.w * np.exp(s),
                               rtol=1e-13, atol=1e-13)


def test_dense_and_fft_objective_agree(rng):
    p, inst = _prob(beta=1.3)
    s = inst["s_true"]
    assert abs(model.objective(p, s) - model.objective(p, s, dense=True)) <= 1e-11 * abs(model.objective(p, s))
    np.testing.assert_allclose(model.gradient(p, s), model.gradient(p, s, dense=True), rtol=1e-9, atol=1e-10)
