"""Adjoint derivatives of a scalar loss of the MAP field.

Test infrastructure only (see the package docstring).

The MAP s* is the root of g(s; theta) = S_L^-1 (s - mu) + beta (nbar w
exp(beta s) - N) (section 3.1.2 with the power-law bias of section 2.4).  By
the implicit function theorem, ds*/dtheta = -H^-1 dg/dtheta with H the
Hessian of section 3.1.2, so for a loss L(s*)

    dL/dtheta = -lambda^T dg/dtheta,   H(s*) lambda = dL/ds*.

Partial derivatives of g used here (mu held fixed):

    dg/dA     = -(1/A) S_L'^-1 (s - mu)   (S_L' = S_L without the k = 0 mode,
                                          whose inverse eigenvalue inv_p0 does
                                          not scale with A)
    dg/dbeta  = nbar w exp(beta s) (1 + beta s) - N
    dg/dnbar  = beta w exp(beta s)
    dg_i/dN_i = -beta
    dg_i/dw_i = beta nbar exp(beta s_i)
    dg/dmu    = -inv_p0 * 1
"""
import numpy as np

from .grid import inv_lambda_half
from .model import hessian_dense, prior_apply
from .newton import SpectralOps, pcg
from .model import hess_diag


def adjoint_dense(prob, s_star, dL_ds):
    """lambda = H(s*)^-1 dL/ds* with the dense Hessian (small grids)."""
    H = hessian_dense(prob, s_star)
    return np.linalg.solve(H, np.asarray(dL_ds, dtype=np.float64).ravel()).reshape(prob.n)


def adjoint_pcg(prob, s_star, dL_ds, rtol=1e-12, max_cg=20000, precond="mean", progress=None):
    """lambda from spectral preconditioned CG on H(s*) lambda = dL/ds*
    (preconditioner as ``newton.precond_constant``; progress as ``pcg``'s)."""
    ops = SpectralOps(prob)
    d = hess_diag(prob, s_star)
    b_hat = ops.fwd(np.asarray(dL_ds, dtype=np.float64))
    x_hat, its, rn = pcg(ops, d, b_hat, rtol * ops.norm(b_hat), max_cg, precond, progress)
    return ops.inv(x_hat), its


def param_grads(prob, s_star, lam):
    """dL/dtheta = -lambda^T dg/dtheta for theta in (A, beta, nbar, N, w, mu)."""
    s = np.asarray(s_star, dtype=np.float64)
    beta, nbar, w = prob.beta, prob.nbar, prob.w
    ebs = np.exp(beta * s)
    p_noncst = prob.replace(inv_p0=0.0)
    Sr = prior_apply(p_noncst, s - prob.mu)
    out = {}
    out["A"] = float(np.sum(lam * Sr)) / prob.amp
    out["beta"] = -float(np.sum(lam * (nbar * w * ebs * (1.0 + beta * s) - prob.counts)))
    out["nbar"] = -float(np.sum(lam * (beta * w * ebs)))
    out["N"] = beta * lam
    out["w"] = -lam * beta * nbar * ebs
    out["mu"] = prob.inv_p0 * float(np.sum(lam))
    return out


def squared_error_loss(s_star, s_true):
    """L = sum (s* - s_true)^2 and its gradient 2 (s* - s_true)."""
    r = np.asarray(s_star) - np.asarray(s_true)
    return float(np.sum(r * r)), 2.0 * r
