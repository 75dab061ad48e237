"""Negative log-posterior, gradient and Hessian of the Poisson-lognormal model.

Test infrastructure only (see the package docstring).

The unknown is the log-density s = ln(1 + delta_M) (section 2.3).  With the
power-law bias 1 + delta_g = (1 + delta_M)^beta (a local case of the general
nonlinear bias of section 2.4; beta = 1 is the unity bias of section 2.4.2),
the negative log-posterior is, up to terms that do not depend on s,

    f(s) = 1/2 (s - mu)^T S_L^-1 (s - mu)                  [log-prior, section 2.3]
         + sum_i [ nbar w_i exp(beta s_i) - beta N_i s_i ]  [eq. 3 with eq. 2]

(the dropped constants are sum_i [ln N_i! - N_i ln(nbar w_i)]).  Its gradient
is the gradient of the quadratic form of section 3.1.2 generalised to beta,

    g(s) = S_L^-1 (s - mu) + beta (nbar w exp(beta s) - N),

and its Hessian is S_L^-1 + diag(beta^2 nbar w exp(beta s)) (section 3.1.2,
Hessian, with the beta factors of the chain rule of section 2.4).
"""
import numpy as np

from . import dft
from .grid import inv_lambda_full, inv_lambda_half


# ---------------------------------------------------------------------------
# Prior operator S_L^-1 (section 2.3: a convolution, diagonal in Fourier space)
# ---------------------------------------------------------------------------

def prior_apply(prob, x):
    """S_L^-1 x through the library FFT: F^-1 diag(1/lambda) F x."""
    return dft.irfftn(dft.rfftn(x) * inv_lambda_half(prob), prob.n)


def prior_apply_dense_dft(prob, x):
    """S_L^-1 x through the dense DFT definition (small grids only)."""
    return np.real(dft.idftn(dft.dftn(x) * inv_lambda_full(prob)))


def prior_kernel(prob):
    """Real-space convolution kernel c(r) of S_L^-1, so (S_L^-1 x)(r) =
    sum_r' c(r - r') x(r') (section 2.3: S_L x is a convolution)."""
    return np.real(dft.idftn(inv_lambda_full(prob)))


def prior_matrix(prob):
    """Dense N_cells x N_cells matrix of S_L^-1 built from its convolution
    kernel: M[a, b] = c((a - b) mod n), per axis.  Small grids only."""
    n = prob.n
    c = prior_kernel(prob)
    ix = np.arange(n[0]); iy = np.arange(n[1]); iz = np.arange(n[2])
    dx = (ix[:, None] - ix[None, :]) % n[0]
    dy = (iy[:, None] - iy[None, :]) % n[1]
    dz = (iz[:, None] - iz[None, :]) % n[2]
    # M[(ax,ay,az),(bx,by,bz)] = c[dx[ax,bx], dy[ay,by], dz[az,bz]]
    M = c[dx[:, None, None, :, None, None],
          dy[None, :, None, None, :, None],
          dz[None, None, :, None, None, :]]
    N = prob.ncells
    return M.reshape(N, N)


# ---------------------------------------------------------------------------
# Likelihood pieces (section 2.1 eqs. 1-3, section 2.4 chain rule)
# ---------------------------------------------------------------------------

def expected_counts(prob, s):
    """<N_i> = nbar w_i (1 + delta_g,i) with 1 + delta_g = exp(beta s) (eq. 2)."""
    return prob.nbar * prob.w * np.exp(prob.beta * s)


def neg_log_likelihood(prob, s):
    """-ln L up to s-independent terms: sum_i <N_i> - N_i ln(1 + delta_g,i) (eq. 3)."""
    lam = expected_counts(prob, s)
    return float(np.sum(lam) - np.sum(prob.counts * prob.beta * s))


def dloglike_ds(prob, s):
    """d ln L / d s_k by the chain rule of section 2.4 (eq. der), for the local
    power-law bias: [d ln L / d ln(1+delta_g)] * [d ln(1+delta_g) / d s].

    First factor: N - nbar w (1 + B); second factor:
    dB/d delta * (1 + delta) / (1 + B) = beta (1+delta)^(beta-1) (1+delta) / (1+delta)^beta = beta.
    """
    one_plus_delta = np.exp(s)
    one_plus_b = one_plus_delta ** prob.beta
    first = prob.counts - prob.nbar * prob.w * one_plus_b
    dB_ddelta = prob.beta * one_plus_delta ** (prob.beta - 1.0)
    second = dB_ddelta * one_plus_delta / one_plus_b
    return first * second


# ---------------------------------------------------------------------------
# Objective, gradient, Hessian
# ---------------------------------------------------------------------------

def objective(prob, s, dense=False):
    """f(s) = -ln posterior up to a constant (see the module docstring)."""
    r = s - prob.mu
    Sr = prior_apply_dense_dft(prob, r) if dense else prior_apply(prob, r)
    return 0.5 * float(np.sum(r * Sr)) + neg_log_likelihood(prob, s)


def gradient(prob, s, dense=False):
    """g = S_L^-1 (s - mu) - d ln L / d s (eq. priorlog plus eq. der)."""
    r = s - prob.mu
    Sr = prior_apply_dense_dft(prob, r) if dense else prior_apply(prob, r)
    return Sr - dloglike_ds(prob, s)


def hess_diag(prob, s):
    """Likelihood part of the Hessian: beta^2 nbar w exp(beta s) per cell."""
    return prob.beta ** 2 * expected_counts(prob, s)


def hessvec(prob, s, v, dense=False):
    """H v = S_L^-1 v + diag(beta^2 nbar w exp(beta s)) v (section 3.1.2)."""
    Sv = prior_apply_dense_dft(prob, v) if dense else prior_apply(prob, v)
    return Sv + hess_diag(prob, s) * v


def hessian_dense(prob, s):
    """Dense Hessian (small grids only)."""
    H = prior_matrix(prob)
    H[np.diag_indices_from(H)] += hess_diag(prob, s).ravel()
    return H
