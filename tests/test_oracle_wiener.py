"""Pins for the oracle's comparison estimators and quality measures
(section 4.1.1: inverse weighting, LSQ-Wiener filter; section 4.1.2:
correlation coefficient, Euclidean distance)."""
import numpy as np
import pytest
from scipy.spatial.distance import euclidean
from scipy.stats import poisson

from conftest import oracle_problem
from oracle import model, wiener
from oracle.grid import Problem
from paper_0911_1407_amd import synth


def _prob(n=(8, 8, 8), box=(64.0,) * 3, seed=3, mask=0.25, nbar=1.5):
    inst = synth.make_instance(n, box, 1.0, nbar, 1.0, radius=box[0] * 0.6, mask_frac=mask, seed=seed, block=2)
    return oracle_problem(inst), inst


def _white(n, box, sigma2, nbar, seed, mask=0.3):
    inst = synth.make_instance(n, box, 1.0, nbar, 1.0, radius=box[0] * 0.5, mask_frac=mask, seed=seed, block=2)
    ncell = n[0] * n[1] * n[2]
    vol = box[0] * box[1] * box[2]
    pk = np.full(inst["pk"].shape, sigma2 * vol / ncell)
    return Problem(n, box, inst["w"], inst["counts"], pk, 1.0, 0.0, nbar, 1.0, 1.0 / sigma2)


def test_inverse_weight_is_the_poisson_maximum_likelihood():
    # IW is the per-cell maximum of the Poisson likelihood of N_i given the
    # expected count nbar w_i (1 + delta_i): d/d delta of logpmf vanishes
    p, _ = _prob(mask=0.2)
    d = wiener.inverse_weight(p)
    cells = np.flatnonzero((p.w > 0).ravel() & (p.counts > 0).ravel())[:40]
    h = 1e-6
    for c in cells:
        i = np.unravel_index(c, p.n)
        lam = lambda x: p.nbar * p.w[i] * (1.0 + x)
        g = (poisson.logpmf(p.counts[i], lam(d[i] + h)) - poisson.logpmf(p.counts[i], lam(d[i] - h))) / (2 * h)
        assert abs(g) <= 1e-5 * p.counts[i]
    assert np.all(d[p.w == 0] == 0.0)


def test_lsq_white_prior_closed_form():
    # S = sigma^2 I: the system is diagonal in real space,
    # delta_i = (N_i - nbar w_i) / (1/sigma^2 + nbar w_i)
    p = _white((8, 8, 8), (16.0,) * 3, 0.7, 1.3, seed=2)
    ref = (p.counts - p.nbar * p.w) / (1.0 / 0.7 + p.nbar * p.w)
    assert np.abs(wiener.lsq_dense(p) - ref).max() <= 1e-12 * np.abs(ref).max()
    d, _ = wiener.lsq_pcg(p, rtol=1e-14)
    assert np.abs(d - ref).max() <= 1e-11 * np.abs(ref).max()


def test_lsq_uniform_completeness_is_diagonal_in_fourier_space():
    # w = w0 everywhere: (1/lambda_k + nbar w0) delta_k = F(N - nbar w0)_k
    p, _ = _prob(n=(16, 16, 16), box=(80.0,) * 3, mask=0.0)
    p = p.replace(w=np.full(p.n, 0.8), inv_p0=0.5)
    from oracle.grid import inv_lambda_half
    rhs = np.fft.rfftn(p.counts - p.nbar * 0.8)
    ref = np.fft.irfftn(rhs / (inv_lambda_half(p) + p.nbar * 0.8), s=p.n, axes=(0, 1, 2))
    assert np.linalg.norm(wiener.lsq_dense(p) - ref) <= 1e-11 * np.linalg.norm(ref)
    d, _ = wiener.lsq_pcg(p, rtol=1e-14)
    assert np.linalg.norm(d - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("n", [(8, 8, 8), (16, 16, 16)])
def test_lsq_is_the_gaussian_posterior_mode(n, rng):
    # the LSQ filter is the MAP of a Gaussian prior (covariance S) and a
    # Gaussian likelihood of delta_o = N/nbar - w with mean W delta and
    # covariance diag(w/nbar): the gradient of
    #   J(delta) = 1/2 delta^T S^-1 delta + 1/2 (delta_o - W delta)^T Nn^-1 (delta_o - W delta)
    # vanishes at the filtered field (all w > 0 here so Nn is invertible)
    p, _ = _prob(n=n, box=(4.0 * n[0],) * 3, mask=0.0)
    Sinv = model.prior_matrix(p)
    w = p.w.ravel()
    do = (p.counts / p.nbar - p.w).ravel()

    def J(x):
        r = do - w * x
        return 0.5 * x @ (Sinv @ x) + 0.5 * np.sum(r * r * p.nbar / w)

    d = wiener.lsq_dense(p).ravel()
    for _ in range(3):
        v = rng.standard_normal(d.shape)
        h = 1e-4
        slope = (J(d + h * v) - J(d - h * v)) / (2 * h)
        scale = np.sqrt(np.sum(v * v)) * np.sqrt(np.sum((Sinv @ d) ** 2))
        assert abs(slope) <= 1e-8 * scale
    dp, _ = wiener.lsq_pcg(p, rtol=1e-14)
    assert np.linalg.norm(dp.ravel() - d) <= 1e-10 * np.linalg.norm(d)


def test_lsq_dense_matches_pcg_masked(rng):
    p, _ = _prob(n=(16, 16, 16), box=(48.0,) * 3, mask=0.3, seed=7)
    dd = wiener.lsq_dense(p)
    dp, _ = wiener.lsq_pcg(p, rtol=1e-14)
    assert np.linalg.norm(dp - dd) <= 1e-9 * np.linalg.norm(dd)


def test_quality_measures(rng):
    x = rng.standard_normal((6, 7, 5))
    x -= x.mean()
    y = rng.standard_normal((6, 7, 5))
    y -= y.mean()
    assert wiener.corr_coeff(x, x) == pytest.approx(1.0, abs=1e-15)
    assert wiener.corr_coeff(3.0 * x, x) == pytest.approx(1.0, abs=1e-15)
    assert wiener.corr_coeff(-x, x) == pytest.approx(-1.0, abs=1e-15)
    # zero-mean fields: the Pearson coefficient of numpy
    assert wiener.corr_coeff(y, x) == pytest.approx(np.corrcoef(x.ravel(), y.ravel())[0, 1], abs=1e-14)
    assert wiener.euclidean_distance(x, x) == 0.0
    assert wiener.euclidean_distance(x + 0.25, x) == pytest.approx(0.25, rel=1e-14)
    assert wiener.euclidean_distance(y, x) == pytest.approx(euclidean(x.ravel(), y.ravel()) / np.sqrt(x.size),
                                                            rel=1e-14)
