"""Pins for the oracle adjoint (implicit-function derivative of the MAP)."""
import numpy as np
import pytest

from conftest import oracle_problem
from oracle import adjoint, closed_form, newton
from oracle.grid import Problem
from paper_0911_1407_amd import synth
from test_oracle_newton import white_problem


def _small(beta=1.3):
    inst = synth.make_instance((8, 8, 8), (25.0,) * 3, 1.0, 1.0, beta, radius=10.0, mask_frac=0.2,
                               seed=7, block=2)
    return oracle_problem(inst), inst


def _loss(p, s_true):
    s, info = newton.newton_dense(p)
    return adjoint.squared_error_loss(s, s_true)[0]


def test_pcg_adjoint_matches_dense():
    p, inst = _small()
    s, _ = newton.newton_dense(p)
    _, dL = adjoint.squared_error_loss(s, inst["s_true"])
    lam_d = adjoint.adjoint_dense(p, s, dL)
    lam_k, its = adjoint.adjoint_pcg(p, s, dL, rtol=1e-13)
    assert np.linalg.norm(lam_d - lam_k) <= 1e-10 * np.linalg.norm(lam_d)


def test_adjoint_grads_match_central_fd():
    p, inst = _small()
    s, _ = newton.newton_dense(p)
    _, dL = adjoint.squared_error_loss(s, inst["s_true"])
    lam = adjoint.adjoint_dense(p, s, dL)
    gr = adjoint.param_grads(p, s, lam)
    st = inst["s_true"]
    for name, attr in [("A", "amp"), ("beta", "beta"), ("nbar", "nbar")]:
        v = getattr(p, attr)
        h = 1e-5 * v
        fd = (_loss(p.replace(**{attr: v + h}), st) - _loss(p.replace(**{attr: v - h}), st)) / (2 * h)
        assert abs(fd - gr[name]) <= 1e-6 * abs(fd), name
    rng = np.random.default_rng(11)
    for name, attr in [("N", "counts"), ("w", "w")]:
        u = rng.choice([-1.0, 1.0], size=p.n)
        if name == "w":
            u = u * (p.w > 0)
        base = getattr(p, attr)
        h = 1e-5 * (1.0 if name == "N" else float(np.mean(p.w[p.w > 0])))
        fd = (_loss(p.replace(**{attr: base + h * u}), st) - _loss(p.replace(**{attr: base - h * u}), st)) / (2 * h)
        assert abs(fd - np.sum(gr[name] * u)) <= 1e-6 * abs(fd), name


@pytest.mark.parametrize("beta", [1.0, 1.5])
def test_white_prior_closed_form_derivatives(beta):
    sigma2 = 0.9
    p = white_problem((8, 8, 8), (16.0,) * 3, sigma2, 1.1, beta, seed=6)
    s, _ = newton.newton_dense(p)
    s_true = np.random.default_rng(2).standard_normal(p.n)
    _, dL = adjoint.squared_error_loss(s, s_true)
    lam = adjoint.adjoint_dense(p, s, dL)
    gr = adjoint.param_grads(p, s, lam)
    ds = closed_form.white_prior_derivs(s, mu=p.mu, sigma2=sigma2, beta=beta, nbar=p.nbar, w=p.w,
                                        counts=p.counts)
    for name in ("beta", "nbar", "mu"):
        expect = float(np.sum(dL * ds[name]))
        assert abs(gr[name] - expect) <= 1e-10 * abs(expect), name
    for name in ("N", "w"):
        np.testing.assert_allclose(gr[name], dL * ds[name], rtol=1e-9, atol=1e-12 * np.abs(dL * ds[name]).max())


def test_pcg_adjoint_matches_fd_ill_conditioned():
    # 2 Mpc/h cells (cond(H) ~ 1e16): the spectral PCG adjoint still matches
    # central differences of the loss, which a dense real-space solve does not
    inst = synth.make_instance((16, 16, 16), (32.0,) * 3, 1.2, 1.1, 1.5, radius=12.8, mask_frac=0.2,
                               seed=0, block=4)
    p = oracle_problem(inst)
    s, _ = newton.newton_krylov(p, rtol=1e-13)
    _, dL = adjoint.squared_error_loss(s, inst["s_true"])
    lam, _ = adjoint.adjoint_pcg(p, s, dL, rtol=1e-13, max_cg=5000)
    gr = adjoint.param_grads(p, s, lam)

    def L(q):
        sv, _ = newton.newton_krylov(q, rtol=1e-13)
        return adjoint.squared_error_loss(sv, inst["s_true"])[0]

    for name, attr in [("beta", "beta"), ("A", "amp")]:
        v = getattr(p, attr)
        h = 1e-5 * v
        fd = (L(p.replace(**{attr: v + h})) - L(p.replace(**{attr: v - h}))) / (2 * h)
        assert abs(fd - gr[name]) <= 1e-7 * abs(fd), name
