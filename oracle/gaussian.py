"""MAP of the Gaussian-prior model (section 2.2, unit bias).

Test infrastructure only (see the package docstring).

The prior on the overdensity delta is Gaussian with covariance S (section
2.2, zero mean); with the unit bias of section 2.2.2 the Poisson likelihood
of section 2.1 has expected counts nbar w (1 + delta).  The negative
log-posterior without its constants is

    f(delta) = 1/2 delta^T S^-1 delta + sum_i [nbar w_i delta_i - N_i ln(1 + delta_i)],

its gradient S^-1 delta + nbar w - N / (1 + delta), and its root is eq.
MAPG, delta = S (N / (1 + delta) - nbar w).  The Hessian S^-1 + diag(N /
(1 + delta)^2) is symmetric positive definite on the domain 1 + delta > 0
(cells with counts).  Solvers: a dense Newton with a Cholesky solve (small
grids) and a spectral Newton with an inner PCG (``newton.pcg``), both with
an Armijo search that keeps 1 + delta > 0 where N > 0.
"""
import numpy as np
from scipy.linalg import cho_factor, cho_solve

from . import model
from .grid import inv_lambda_half
from .newton import SpectralOps, pcg


def objective(prob, d):
    lik = np.sum(prob.nbar * prob.w * d) - np.sum(np.where(prob.counts > 0, prob.counts * np.log1p(d), 0.0))
    return 0.5 * float(np.sum(d * model.prior_apply(prob, d))) + float(lik)


def gradient(prob, d):
    return model.prior_apply(prob, d) + prob.nbar * prob.w - np.where(prob.counts > 0, prob.counts / (1.0 + d), 0.0)


def hess_diag(prob, d):
    return np.where(prob.counts > 0, prob.counts / (1.0 + d) ** 2, 0.0)


def prior_cov_apply(prob, x):
    """S x = F^-1 diag(lambda) F x (needs inv_p0 > 0 for the k = 0 mode)."""
    return np.fft.irfftn(np.fft.rfftn(x) / inv_lambda_half(prob), s=prob.n, axes=(0, 1, 2))


def mapg_residual(prob, d):
    """delta - S (N / (1 + delta) - nbar w): zero at the MAP (eq. MAPG)."""
    return d - prior_cov_apply(prob, prob.counts / (1.0 + d) - prob.nbar * prob.w)


def _armijo(prob, d, p, g, c1=1e-4, max_halvings=60):
    """Armijo backtracking from a = 1, halving, on the decrease in difference
    form f(d + a p) - f(d) = a b + a^2 c / 2 + sum_i [nbar w_i a p_i - N_i
    log1p(a p_i / (1 + d_i))] (b = d^T S^-1 p, c = p^T S^-1 p), which stays
    accurate when the decrease is far below the size of f; a step that
    leaves 1 + delta > 0 in a cell with counts is rejected."""
    slope = float(np.sum(g * p))
    if slope >= 0:
        return None
    Sp = model.prior_apply(prob, p)
    b = float(np.sum(d * Sp))
    c = float(np.sum(p * Sp))
    pos = prob.counts > 0
    ratio = np.where(pos, p / (1.0 + d), 0.0)
    a = 1.0
    for _ in range(max_halvings):
        if np.all(1.0 + a * ratio[pos] > 0.0):
            lik = np.sum(prob.nbar * prob.w * a * p) - np.sum(prob.counts[pos] * np.log1p(a * ratio[pos]))
            if a * b + 0.5 * a * a * c + lik <= c1 * a * slope:
                return a
        a *= 0.5
    return None


def newton_dense(prob, rtol=1e-13, max_newton=100):
    """Dense Newton (grids up to 16^3), start delta = 0; returns (delta, its)."""
    Sinv = model.prior_matrix(prob)
    d = np.zeros(prob.n)
    g = gradient(prob, d)
    g0 = np.linalg.norm(g)
    its = 0
    while np.linalg.norm(g) > rtol * g0 and its < max_newton:
        H = Sinv + np.diag(hess_diag(prob, d).ravel())
        p = -cho_solve(cho_factor(H), g.ravel()).reshape(prob.n)
        a = _armijo(prob, d, p, g)
        if a is None:
            break
        d = d + a * p
        g = gradient(prob, d)
        its += 1
    return d, its


def newton_spectral(prob, rtol=1e-12, max_newton=200, max_cg=20000):
    """Spectral inexact Newton with inner PCG, start delta = 0."""
    ops = SpectralOps(prob)
    d = np.zeros(prob.n)
    g = gradient(prob, d)
    g0 = np.linalg.norm(g)
    its = 0
    while np.linalg.norm(g) > rtol * g0 and its < max_newton:
        gn = np.linalg.norm(g)
        eta = min(0.5, max(np.sqrt(gn / g0), 0.5 * rtol * g0 / gn))
        g_hat = ops.fwd(g)
        x, _, _ = pcg(ops, hess_diag(prob, d), -g_hat, eta * ops.norm(g_hat), max_cg)
        p = ops.inv(x)
        a = _armijo(prob, d, p, g)
        if a is None:
            break
        d = d + a * p
        g = gradient(prob, d)
        its += 1
    return d, its


def white_prior_map(sigma2, nbar, w, counts):
    """Per-cell closed form for S = sigma2 I: delta / sigma2 + nbar w - N / (1 + delta) = 0,
    i.e. delta^2 / sigma2 + (1/sigma2 + nbar w) delta + (nbar w - N) = 0 with
    1 + delta > 0 (the root with the + sign); delta = -sigma2 nbar w where N = 0."""
    a = 1.0 / sigma2
    b = a + nbar * w
    c = nbar * w - counts
    root = (-b + np.sqrt(b * b - 4.0 * a * c)) / (2.0 * a)
    return np.where(counts > 0, root, -sigma2 * nbar * w)
