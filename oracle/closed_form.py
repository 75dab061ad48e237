"""Closed-form MAP fields for special cases, used to pin the solvers.

Test infrastructure only (see the package docstring).

White prior.  If every prior eigenvalue equals sigma2 (S_L = sigma2 * I,
including the k = 0 mode), the MAP equation of section 2.4 decouples into one
scalar equation per cell,

    (s - mu)/sigma2 + beta (nbar w exp(beta s) - N) = 0.

Writing y = mu + sigma2 beta N - s gives beta y exp(beta y) = X with
X = sigma2 beta^2 nbar w exp(beta mu + sigma2 beta^2 N), so

    s = mu + sigma2 beta N - W0(X) / beta                (principal branch)

and, by implicit differentiation of the scalar equation G(s; theta) = 0,
ds/dtheta = -(dG/dtheta) / (dG/ds) with dG/ds = 1/sigma2 + beta^2 nbar w exp(beta s).

Uniform data.  If w = w0 and N = c >= 1 in every cell and inv_p0 = 0, the
prior term vanishes on uniform fields and the likelihood term vanishes at
nbar w0 exp(beta s) = c, so s = ln(c / (nbar w0)) / beta in every cell.

Zero completeness.  If w = 0 everywhere (then N = 0), the likelihood term is
identically zero and the MAP is the prior mean: s = mu when inv_p0 > 0; when
inv_p0 = 0 the k = 0 mode is free and s = mu + mean(s0 - mu).
"""
import numpy as np

from .lambertw import lambertw_exp


def white_prior_map(prob_or_none=None, *, mu, sigma2, beta, nbar, w, counts):
    w = np.asarray(w, dtype=np.float64)
    N = np.asarray(counts, dtype=np.float64)
    s = mu + sigma2 * beta * N
    pos = w > 0
    # ln X = ln(sigma2 beta^2 nbar w) + beta mu + sigma2 beta^2 N
    lnX = np.log(sigma2 * beta * beta * nbar * w[pos]) + beta * mu + sigma2 * beta * beta * N[pos]
    s = np.array(s, dtype=np.float64)
    s[pos] = s[pos] - lambertw_exp(lnX) / beta
    return s


def white_prior_derivs(s, *, mu, sigma2, beta, nbar, w, counts):
    """ds/dtheta per cell for theta in (beta, nbar, N, w, mu)."""
    ebs = np.exp(beta * s)
    dGds = 1.0 / sigma2 + beta * beta * nbar * w * ebs
    out = {}
    out["beta"] = -(nbar * w * ebs * (1.0 + beta * s) - counts) / dGds
    out["nbar"] = -(beta * w * ebs) / dGds
    out["N"] = beta / dGds
    out["w"] = -(beta * nbar * ebs) / dGds
    out["mu"] = (1.0 / sigma2) / dGds
    return out


def uniform_data_map(c, nbar, w0, beta):
    return np.log(c / (nbar * w0)) / beta


def zero_completeness_map(s0, mu, inv_p0):
    s0 = np.asarray(s0, dtype=np.float64)
    if inv_p0 > 0:
        return np.full(s0.shape, mu)
    return np.full(s0.shape, mu + float(np.mean(s0 - mu)))
