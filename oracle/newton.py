"""MAP solvers for the Poisson-lognormal posterior.

Test infrastructure only (see the package docstring).

Section 3.1 finds the MAP as the root of the gradient of the quadratic form,
grad Q(s) = S_L^-1 (s - mu) + nbar w exp(s) - N (unity bias; the beta factors
of the power-law bias follow from the chain rule of section 2.4), with the
Newton-Raphson update x <- x - H^-1 grad Q and, in its practical form, a
Krylov step x <- x + tau xi whose length tau = -xi^T grad Q / xi^T H xi is
eq. (New5).  The search vectors are left to an earlier reference; here they
are the conjugate directions of a preconditioned conjugate-gradient solve of
the Newton system, for which eq. (New5) is exactly the CG step length on the
local quadratic model.

Two solvers:

* ``newton_dense``  -- plain Newton-Raphson with a dense Hessian and a
  Cholesky solve, for grids up to 16^3.
* ``newton_krylov`` -- inexact Newton with an inner preconditioned CG, the
  iterate held as its half-complex spectrum so that S_L^-1 is an exact
  pointwise product; FFTs come from numpy.

Both globalise with an Armijo backtracking line search on f (c1 = 1e-4,
halving, at most 30 halvings).  The decrease f(s + a p) - f(s) is evaluated
in difference form, a b + a^2 c / 2 + sum_i [e_i expm1(a beta p_i) - a beta
N_i p_i] with b = p^T S_L^-1 (s - mu), c = p^T S_L^-1 p and e_i the expected
counts, so that it stays accurate when it is far below the size of f.
Stopping rule: ||g(s_j)||_2 <= rtol * ||g(s_0)||_2; start s_0 = mu unless
given; forcing term eta_j = min(0.5, sqrt(||g_j|| / ||g_0||)).  The dense
solver also stops at its roundoff floor: once ||g|| < 1e-10 ||g_0||, a step
that fails to halve ||g|| ends the iteration (status "floor").
"""
import numpy as np
import scipy.linalg

from . import dft
from .grid import hermitian_weights, inv_lambda_half
from .model import expected_counts, gradient, hess_diag, objective, prior_matrix


class SolveInfo(dict):
    pass


def _armijo(delta_f, slope, c1=1e-4, max_halvings=30):
    """Backtracking from a = 1: the first a = 2^-h with
    delta_f(a) <= c1 a slope; None if none is found."""
    a = 1.0
    for _ in range(max_halvings + 1):
        if delta_f(a) <= c1 * a * slope:
            return a
        a *= 0.5
    return None


def newton_dense(prob, s0=None, rtol=1e-13, max_newton=60):
    """Dense-Hessian Newton-Raphson (section 3.1) with Armijo backtracking."""
    n = prob.n
    s = np.full(n, prob.mu) if s0 is None else np.array(s0, dtype=np.float64).reshape(n)
    Sinv = prior_matrix(prob)
    beta = prob.beta

    def grad(sv):
        return (Sinv @ (sv.ravel() - prob.mu)).reshape(n) + beta * (
            expected_counts(prob, sv) - prob.counts)

    g = grad(s)
    g0 = np.linalg.norm(g)
    info = SolveInfo(newton_its=0, status="ok", rel_grad=0.0, history=[1.0])
    if g0 == 0.0:
        return s, info
    for it in range(max_newton):
        gn = np.linalg.norm(g)
        info["rel_grad"] = gn / g0
        if gn <= rtol * g0:
            break
        H = Sinv.copy()
        H[np.diag_indices_from(H)] += hess_diag(prob, s).ravel()
        p = scipy.linalg.cho_solve(scipy.linalg.cho_factor(H), -g.ravel()).reshape(n)
        e = expected_counts(prob, s)
        b = float(p.ravel() @ (Sinv @ (s.ravel() - prob.mu)))
        c = float(p.ravel() @ (Sinv @ p.ravel()))
        slope = float(np.sum(g * p))

        def delta_f(a):
            # a trial step too long for exp overflows to +inf, which the
            # Armijo test rejects like any other increase of f
            with np.errstate(over="ignore"):
                return a * b + 0.5 * a * a * c + float(
                    np.sum(e * np.expm1(a * beta * p) - a * beta * prob.counts * p))

        a = _armijo(delta_f, slope)
        if a is None:
            info["status"] = "linesearch"
            break
        s = s + a * p
        g = grad(s)
        info["newton_its"] = it + 1
        gn_new = np.linalg.norm(g)
        info["history"].append(gn_new / g0)
        if gn_new < 1e-10 * g0 and gn_new > 0.5 * gn:
            info["status"] = "floor"
            break
    else:
        if np.linalg.norm(g) > rtol * g0:
            info["status"] = "not_converged"
    info["rel_grad"] = np.linalg.norm(g) / g0
    return s, info


class SpectralOps:
    """Spectral-space helpers for the half-complex iterate."""

    def __init__(self, prob):
        self.prob = prob
        self.n = prob.n
        self.N = prob.ncells
        self.inv_lam = inv_lambda_half(prob)
        self.c = hermitian_weights(prob.n)
        self.mu_hat = np.zeros(self.inv_lam.shape, dtype=np.complex128)
        self.mu_hat[0, 0, 0] = self.N * prob.mu

    def dot(self, a, b):
        """Real-space inner product x^T y from half spectra (Parseval)."""
        return float(np.sum(self.c * (np.conj(a) * b).real) / self.N)

    def norm(self, a):
        return np.sqrt(self.dot(a, a))

    def fwd(self, x):
        return dft.rfftn(x)

    def inv(self, X):
        return dft.irfftn(X, self.n)

    def grad(self, s_hat):
        """Gradient spectrum g_hat = (s_hat - mu_hat)/lambda + F[beta (e - N)]."""
        prob = self.prob
        s = self.inv(s_hat)
        e = expected_counts(prob, s)
        g_hat = self.inv_lam * (s_hat - self.mu_hat) + self.fwd(prob.beta * (e - prob.counts))
        return s, e, g_hat

    def hessvec(self, d, p_hat):
        """H p in spectral form: p_hat/lambda + F[d * F^-1 p_hat]."""
        return self.inv_lam * p_hat + self.fwd(d * self.inv(p_hat))


def precond_constant(d, kind="mean"):
    """The constant c of the preconditioner 1/lambda_k + c: the mean of the
    Hessian diagonal d ("mean": with it, 1/lambda_k + c is the exact diagonal
    of H in the Fourier basis) or its 25th percentile floored at 1e-3 of the
    mean ("p25", which takes far fewer CG steps where d spans decades, as
    under a radial selection).  The paper gives no preconditioner; H is
    positive definite, so the choice changes the iteration path, never the
    MAP or the solution of a linear system."""
    m = float(np.mean(d))
    if kind == "p25":
        return max(float(np.percentile(d, 25)), 1e-3 * m)
    return m


def pcg(ops, d, rhs_hat, tol_abs, max_cg, precond="mean", progress=None):
    """Preconditioned CG on H x = rhs in spectral coordinates, preconditioned by
    the Fourier-diagonal 1/lambda_k + c (c from ``precond_constant``).  Stops
    when ||r|| <= tol_abs.  progress (optional): called with (iteration,
    ||r||) every 100 iterations (reporting only)."""
    M = ops.inv_lam + precond_constant(d, precond)
    Minv = np.where(M > 0, 1.0 / np.where(M > 0, M, 1.0), 0.0)
    x = np.zeros_like(rhs_hat)
    r = rhs_hat.copy()
    its = 0
    if ops.norm(r) <= tol_abs:
        return x, its, ops.norm(r)
    z = Minv * r
    p = z.copy()
    rz = ops.dot(r, z)
    for k in range(max_cg):
        q = ops.hessvec(d, p)
        pq = ops.dot(p, q)
        if pq <= 0.0:
            break
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        its = k + 1
        if ops.norm(r) <= tol_abs:
            break
        if progress is not None and its % 100 == 0:
            progress(its, ops.norm(r))
        z = Minv * r
        rz_new = ops.dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, its, ops.norm(r)


def newton_krylov(prob, s0=None, rtol=1e-8, max_newton=100, max_cg=500,
                  eta_max=0.5, return_hat=False, precond="mean", progress=None):
    """Inexact Newton-Krylov MAP solver with the spectral iterate (inner PCG
    preconditioned as ``precond_constant`` says).  progress (optional): called
    with (Newton step, ||g|| / ||g0||, CG iterations so far) after each step
    (reporting only)."""
    ops = SpectralOps(prob)
    n = prob.n
    s0 = np.full(n, prob.mu) if s0 is None else np.array(s0, dtype=np.float64).reshape(n)
    s_hat = ops.fwd(s0)
    s, e, g_hat = ops.grad(s_hat)
    gnorm = ops.norm(g_hat)
    g0 = gnorm
    info = SolveInfo(newton_its=0, cg_its=0, hvps=0, status="ok", rel_grad=0.0,
                     history=[1.0])
    if g0 == 0.0:
        return (s, s_hat, info) if return_hat else (s, info)
    beta = prob.beta
    for it in range(max_newton):
        if gnorm <= rtol * g0:
            break
        eta = min(eta_max, np.sqrt(gnorm / g0))
        d = hess_diag(prob, s)
        p_hat, its, _ = pcg(ops, d, -g_hat, eta * gnorm, max_cg, precond)
        info["cg_its"] += its
        info["hvps"] += its
        p = ops.inv(p_hat)
        slope = ops.dot(g_hat, p_hat)
        b = ops.dot(p_hat, ops.inv_lam * (s_hat - ops.mu_hat))
        c = ops.dot(p_hat, ops.inv_lam * p_hat)

        def delta_f(a):
            # a trial step too long for exp overflows to +inf, which the
            # Armijo test rejects like any other increase of f
            with np.errstate(over="ignore"):
                return a * b + 0.5 * a * a * c + float(
                    np.sum(e * np.expm1(a * beta * p) - a * beta * prob.counts * p))

        a = _armijo(delta_f, slope) if slope < 0 else None
        if a is None:
            info["status"] = "linesearch"
            break
        s_hat = s_hat + a * p_hat
        s, e, g_hat = ops.grad(s_hat)
        gnorm = ops.norm(g_hat)
        info["newton_its"] = it + 1
        info["history"].append(gnorm / g0)
        if progress is not None:
            progress(it + 1, gnorm / g0, info["cg_its"])
    else:
        if gnorm > rtol * g0:
            info["status"] = "not_converged"
    info["rel_grad"] = gnorm / g0
    return (s, s_hat, info) if return_hat else (s, info)


def objective_of(prob, s):
    return objective(prob, s)


def gradient_of(prob, s):
    return gradient(prob, s)
