"""Pins for the oracle's spectral-form operators (section 3.1.2 gradient and
Hessian with the iterate held as its half spectrum; section 2.3: S_L^-1 is
diagonal in Fourier space), which are the reference of every full-size GPU
operator parity test.

``SpectralOps.grad`` and ``SpectralOps.hessvec`` are pinned three ways:
against the real-space ``model.gradient`` / ``model.hessvec`` (themselves
pinned by central differences of the objective and the gradient, and by the
dense DFT), transformed to the half spectrum; against central differences of
``SpectralOps.grad`` taken in spectral coordinates; and by symmetry and
positivity of the Hessian in the Parseval inner product.  A scale error, a
dropped 1/lambda term, a missing beta factor or a transposed operand fails
each of them by orders of magnitude more than the tolerances.

The linear-bias oracle's minimiser (a non-convex posterior, where the
iteration path could in principle pick the minimum) is shown not to depend
on its preconditioner constant on the selection recipe the GPU parity test
uses.
"""
import numpy as np
import pytest

from conftest import oracle_problem
from oracle import linbias, model
from oracle.newton import SpectralOps
from paper_0911_1407_amd import synth

# a cubic grid and a ragged one (three different axis lengths, odd nz/2+1)
GRIDS = [((16, 16, 16), 1.0), ((16, 24, 32), 1.4), ((12, 8, 20), 0.8)]


def _prob(n, beta, seed=11, cell=6.0, mask=0.25):
    box = tuple(cell * v for v in n)
    inst = synth.make_instance(n, box, 1.1, 1.2, beta, radius=0.45 * box[0], mask_frac=mask, seed=seed, block=2)
    inst["inv_p0"] = 0.3
    return oracle_problem(inst), inst


def _relmax(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("n,beta", GRIDS)
def test_spectral_grad_equals_transformed_real_space_gradient(n, beta, rng):
    P, inst = _prob(n, beta)
    ops = SpectralOps(P)
    s = inst["s_true"] + 0.1 * rng.standard_normal(n)
    s_back, e, g_hat = ops.grad(np.fft.rfftn(s))
    assert np.abs(s_back - s).max() <= 1e-13 * np.abs(s).max()
    np.testing.assert_allclose(e, P.nbar * P.w * np.exp(beta * s), rtol=1e-13, atol=0)
    ref = np.fft.rfftn(model.gradient(P, s))
    assert _relmax(g_hat, ref) <= 1e-12


@pytest.mark.parametrize("n,beta", GRIDS)
def test_spectral_hessvec_equals_transformed_real_space_hessvec(n, beta, rng):
    P, inst = _prob(n, beta)
    ops = SpectralOps(P)
    s = inst["s_true"] + 0.1 * rng.standard_normal(n)
    v = rng.standard_normal(n)
    got = ops.hessvec(model.hess_diag(P, s), np.fft.rfftn(v))
    ref = np.fft.rfftn(model.hessvec(P, s, v))
    assert _relmax(got, ref) <= 1e-12


@pytest.mark.parametrize("n,beta", GRIDS)
def test_spectral_hessvec_matches_fd_of_spectral_grad(n, beta, rng):
    # central differences of the spectral gradient along a spectral direction
    P, inst = _prob(n, beta)
    ops = SpectralOps(P)
    s_hat = np.fft.rfftn(inst["s_true"] + 0.1 * rng.standard_normal(n))
    v_hat = np.fft.rfftn(rng.standard_normal(n))
    s, _, _ = ops.grad(s_hat)
    h = 1e-6
    fd = (ops.grad(s_hat + h * v_hat)[2] - ops.grad(s_hat - h * v_hat)[2]) / (2 * h)
    hv = ops.hessvec(model.hess_diag(P, s), v_hat)
    assert np.linalg.norm(fd - hv) <= 1e-7 * np.linalg.norm(hv)


def test_spectral_hessvec_symmetric_positive(rng):
    P, inst = _prob((16, 24, 32), 1.3)
    ops = SpectralOps(P)
    d = model.hess_diag(P, inst["s_true"])
    u_hat = np.fft.rfftn(rng.standard_normal(P.n))
    v_hat = np.fft.rfftn(rng.standard_normal(P.n))
    a = ops.dot(u_hat, ops.hessvec(d, v_hat))
    b = ops.dot(v_hat, ops.hessvec(d, u_hat))
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    assert ops.dot(v_hat, ops.hessvec(d, v_hat)) > 0.0
    # Parseval: the spectral dot is the real-space one
    u, v = ops.inv(u_hat), ops.inv(v_hat)
    assert ops.dot(u_hat, v_hat) == pytest.approx(float(np.sum(u * v)), rel=1e-12)


def test_spectral_hessvec_fine_cells_plane_wave():
    # fine cells (1/lambda spans many decades) on a non-cubic grid and box,
    # with d = 0 (w = 0 everywhere): a plane wave given exactly as a
    # half-spectrum delta comes back multiplied by 1/lambda of its own mode
    # (a transposed axis or a wrong fold would pick another mode's lambda)
    n, box = (32, 24, 16), (64.0, 48.0, 40.0)
    inst = synth.make_instance(n, box, 1.5, 0.5, 1.0, seed=2)
    inst["w"] = np.zeros(n)
    inst["counts"] = np.zeros(n)
    P = oracle_problem(inst)
    ops = SpectralOps(P)
    for m in ((3, -5, 7), (-9, 2, 1), (1, 11, 5)):
        v_hat = np.zeros(ops.inv_lam.shape, dtype=np.complex128)
        v_hat[m[0] % n[0], m[1] % n[1], m[2]] = 0.5 * P.ncells
        kmag = 2 * np.pi * np.sqrt(sum((c / L) ** 2 for c, L in zip(m, box)))
        lam = P.amp * kmag ** -1.5 * np.exp(-(2 * kmag) ** 2) * P.ncells / P.volume
        got = ops.hessvec(np.zeros(n), v_hat)
        np.testing.assert_allclose(got, v_hat / lam, rtol=1e-13, atol=0)
        # in real space: cos(k.x) / lambda_k
        x = np.arange(n[0])[:, None, None] * m[0] / n[0] + np.arange(n[1])[None, :, None] * m[1] / n[1] \
            + np.arange(n[2])[None, None, :] * m[2] / n[2]
        wave = np.cos(2 * np.pi * x)
        np.testing.assert_allclose(ops.inv(got), wave / lam, rtol=0, atol=1e-12 * abs(1.0 / lam))


@pytest.mark.parametrize("kind", [linbias.LOGNORMAL, linbias.GAUSSIAN])
def test_linear_bias_minimiser_does_not_depend_on_preconditioner(kind):
    # the recipe of the GPU linear-bias parity test at 64^3: the selection
    # workload's cells, radial selection and masked 8^3 blocks, nbar 0.5,
    # with a 1.5-cell smoothing multiplier; two Newton paths whose
    # preconditioner constants differ (25th percentile vs mean of the
    # curvature) reach the same minimiser
    inst = synth.config_instance("sel256", n=64)
    P = oracle_problem(inst)
    cell = inst["box"][0] / inst["n"][0]
    bk = synth.bias_multiplier_half(inst["n"], inst["box"], 1.0, 1.5 * cell)
    x1, i1 = linbias.newton_spectral(P, bk, kind, rtol=1e-10, precond="p25")
    x2, i2 = linbias.newton_spectral(P, bk, kind, rtol=1e-10, precond="mean")
    assert i1["status"] == "ok" and i2["status"] == "ok", (i1, i2)
    assert i1["cg_its"] != i2["cg_its"] or i1["newton_its"] != i2["newton_its"]  # different paths
    assert np.linalg.norm(x1 - x2) <= 1e-9 * np.linalg.norm(x1)
    # and the same objective value (a different local minimum would differ)
    f1 = linbias.objective(P, bk, x1, kind)
    f2 = linbias.objective(P, bk, x2, kind)
    assert abs(f1 - f2) <= 1e-12 * abs(f1)
