"""Pins for the oracle's linear-bias MAP (sections 2.2.1 and 2.4.1): reduction
to the unit-bias models, brute force from dense DFT matrices, finite
differences, and a per-cell closed form under a white prior."""
import numpy as np
import pytest

from conftest import oracle_problem
from oracle import gaussian, linbias, model
from oracle.grid import Problem
from paper_0911_1407_amd import synth

LN, GA = linbias.LOGNORMAL, linbias.GAUSSIAN


def _prob(n=(8, 8, 8), box=(32.0,) * 3, seed=3, mask=0.25, nbar=1.5, inv_p0=0.5, sigma=0.8):
    inst = synth.make_instance(n, box, sigma, nbar, 1.0, radius=box[0] * 0.6, mask_frac=mask, seed=seed, block=2)
    inst["inv_p0"] = inv_p0
    return oracle_problem(inst)


def _bk(p, b0=1.0, smooth=4.0):
    return synth.bias_multiplier_half(p.n, p.box, b0, smooth)


def _start(p, kind, rng, scale=0.2):
    return linbias.prior_mean(p, kind) + scale * rng.standard_normal(p.n)


@pytest.mark.parametrize("kind", [LN, GA])
def test_unit_multiplier_reduces_to_unit_bias_models(kind, rng):
    # b_hat = 1 is delta_g = delta_M: the lognormal model with beta = 1 and the
    # unit-bias Gaussian-prior model, whose oracles are pinned on their own
    p = _prob()
    one = np.ones(synth.hermitian_multiplicity(p.n).shape)
    x1, x2 = _start(p, kind, rng), _start(p, kind, rng)
    v = rng.standard_normal(p.n)
    if kind == LN:
        g_ref, hv_ref = model.gradient(p, x1), model.hessvec(p, x1, v)
        df_ref = model.objective(p, x1) - model.objective(p, x2)
    else:
        g_ref = gaussian.gradient(p, x1)
        hv_ref = model.prior_apply(p, v) + gaussian.hess_diag(p, x1) * v
        df_ref = gaussian.objective(p, x1) - gaussian.objective(p, x2)
    g = linbias.gradient(p, one, x1, kind)
    hv = linbias.hessvec(p, one, x1, v, kind)
    df = linbias.objective(p, one, x1, kind) - linbias.objective(p, one, x2, kind)
    assert np.abs(g - g_ref).max() <= 1e-11 * np.abs(g_ref).max()
    assert np.abs(hv - hv_ref).max() <= 1e-11 * np.abs(hv_ref).max()
    assert df == pytest.approx(df_ref, rel=1e-10, abs=1e-9)


@pytest.mark.parametrize("kind", [LN, GA])
def test_objective_matches_dense_dft_brute_force(kind, rng):
    # the FFT form against dense matrices of S^-1 and B built from the DFT
    # definition, at 4 x 6 x 4 (uneven axes catch a transposed kernel)
    p = _prob(n=(4, 6, 4), box=(16.0, 24.0, 16.0), mask=0.0)
    bk = _bk(p, 0.9, 3.0)
    x = _start(p, kind, rng)
    f = linbias.objective(p, bk, x, kind)
    fd = linbias.objective_dense(p, bk, x, kind)
    assert f == pytest.approx(fd, rel=1e-12)
    # B applied through the FFT equals the dense matrix (real, even kernel)
    B = linbias.bias_matrix(bk, p.n)
    assert np.allclose(B, B.T, atol=1e-14)
    z = rng.standard_normal(p.n)
    assert np.abs(linbias.bias_apply(bk, z).ravel() - B @ z.ravel()).max() <= 1e-13


@pytest.mark.parametrize("kind", [LN, GA])
def test_gradient_and_hessvec_match_finite_differences(kind, rng):
    p = _prob(n=(4, 6, 4), box=(16.0, 24.0, 16.0), mask=0.0)
    bk = _bk(p, 0.9, 3.0)
    x = _start(p, kind, rng)
    g = linbias.gradient(p, bk, x, kind)
    h = 1e-5
    for _ in range(3):
        v = rng.standard_normal(p.n)
        fd = (linbias.objective_dense(p, bk, x + h * v, kind) - linbias.objective_dense(p, bk, x - h * v, kind)) / (2 * h)
        assert fd == pytest.approx(float(np.sum(g * v)), rel=1e-7)
        hv = linbias.hessvec(p, bk, x, v, kind)
        fdg = (linbias.gradient(p, bk, x + h * v, kind) - linbias.gradient(p, bk, x - h * v, kind)) / (2 * h)
        assert np.abs(fdg - hv).max() <= 1e-6 * np.abs(hv).max()
        u = rng.standard_normal(p.n)
        assert float(np.sum(u * hv)) == pytest.approx(float(np.sum(v * linbias.hessvec(p, bk, x, u, kind))), rel=1e-12)


def _white(n, box, sigma2, nbar, seed, mu):
    inst = synth.make_instance(n, box, 1.0, nbar, 1.0, radius=box[0] * 0.5, mask_frac=0.3, seed=seed, block=2)
    pk = np.full(inst["pk"].shape, sigma2 * np.prod(box) / np.prod(n))
    return Problem(n, box, inst["w"], inst["counts"], pk, 1.0, mu, nbar, 1.0, 1.0 / sigma2)


@pytest.mark.parametrize("kind,b0", [(LN, 1.0), (LN, 1.4), (GA, 0.7), (GA, 1.3)])
def test_white_prior_local_bias_closed_form(kind, b0):
    # S = sigma2 I and b_hat = b0 decouple the cells: each MAP value is the
    # root of a scalar equation, found by bisection
    p = _white((8, 8, 8), (16.0,) * 3, 0.6, 1.2, seed=4, mu=-0.3)
    bk = np.full(synth.hermitian_multiplicity(p.n).shape, b0)
    ref = linbias.white_prior_map(kind, 0.6, linbias.prior_mean(p, kind), b0, p.nbar, p.w, p.counts)
    x, info = linbias.newton_spectral(p, bk, kind, rtol=1e-13)
    assert info["status"] == "ok"
    assert np.abs(x - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max())
    xd, res = linbias.map_dense(p, bk, kind, gtol_rel=1e-13)
    assert np.abs(xd - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("kind", [LN, GA])
def test_spectral_newton_matches_dense_trust_region(kind):
    # non-local multiplier, masked selection: the truncated-PCG Newton against
    # scipy's dense trust-region Newton on the same objective
    p = _prob(n=(8, 8, 8), box=(24.0,) * 3, mask=0.3, seed=5)
    bk = _bk(p, 0.95, 3.0)
    xs, info = linbias.newton_spectral(p, bk, kind, rtol=1e-11)
    assert info["status"] == "ok"
    xd, res = linbias.map_dense(p, bk, kind, gtol_rel=1e-12)
    assert np.linalg.norm(xs - xd) <= 1e-9 * np.linalg.norm(xd)
    y = linbias.galaxy_field(p, bk, xs, kind)
    assert np.all(y[p.counts > 0] > 0)
    # the MAP equations of sections 2.2.1 / 2.4.1: prior side equals likelihood side
    g = linbias.gradient(p, bk, xs, kind)
    lhs = model.prior_apply(p, xs - linbias.prior_mean(p, kind))
    assert np.linalg.norm(g) <= 1e-10 * np.linalg.norm(lhs)


def test_likelihood_is_poisson_with_biased_rate(rng):
    # differences of the likelihood part equal those of -sum log Poisson(N | nbar w y)
    from scipy.stats import poisson
    p = _prob()
    bk = _bk(p)
    pos = p.w > 0
    x1, x2 = _start(p, LN, rng), _start(p, LN, rng)

    def nll(x):
        y = linbias.galaxy_field(p, bk, x, LN)
        return -np.sum(poisson.logpmf(p.counts[pos], (p.nbar * p.w * y)[pos]))

    assert linbias.likelihood(p, linbias.galaxy_field(p, bk, x1, LN)) - linbias.likelihood(
        p, linbias.galaxy_field(p, bk, x2, LN)) == pytest.approx(nll(x1) - nll(x2), rel=1e-10)


def test_white_prior_root_at_unit_bias_matches_closed_forms():
    # b0 = 1 is the unit bias: the bisection root equals the Lambert-W closed
    # form of the lognormal model and the quadratic root of the Gaussian one
    from oracle import closed_form
    rng = np.random.default_rng(7)
    shape = (6, 5, 4)
    w = rng.uniform(0.05, 1.0, shape)
    w[0, 0, :] = 0.0
    counts = np.where(w > 0, rng.poisson(3.0, shape), 0).astype(np.float64)
    sigma2, mu, nbar = 0.7, -0.35, 1.4
    ln = linbias.white_prior_map(LN, sigma2, mu, 1.0, nbar, w, counts)
    ref_ln = closed_form.white_prior_map(mu=mu, sigma2=sigma2, beta=1.0, nbar=nbar, w=w, counts=counts)
    assert np.abs(ln - ref_ln).max() <= 1e-12 * max(1.0, np.abs(ref_ln).max())
    ga = linbias.white_prior_map(GA, sigma2, 0.0, 1.0, nbar, w, counts)
    ref_ga = gaussian.white_prior_map(sigma2, nbar, w, counts)
    assert np.abs(ga - ref_ga).max() <= 1e-12 * max(1.0, np.abs(ref_ga).max())


def test_bias_multiplier_is_even_so_B_is_symmetric():
    # b_hat(-k) = b_hat(k) on the stored half spectrum (kz = 0 and Nyquist
    # planes hold both k and -k), which makes B a symmetric matrix
    for n in ((8, 8, 8), (6, 10, 4)):
        bk = synth.bias_multiplier_half(n, tuple(3.0 * v for v in n), 0.8, 2.5)
        full = linbias.bias_full(bk, n)
        neg = full[(-np.arange(n[0])) % n[0]][:, (-np.arange(n[1])) % n[1]][:, :, (-np.arange(n[2])) % n[2]]
        assert np.array_equal(full, neg)
        B = linbias.bias_matrix(bk, n)
        assert np.abs(B - B.T).max() <= 1e-14
