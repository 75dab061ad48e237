"""The paper's comparison estimators and quality measures (section 4.1).

Test infrastructure only (see the package docstring).

* Inverse weighting (section 4.1.1, the IW definitions): the inverse-weighted
  count N_i / w_i and the overdensity N_i / (w_i nbar) - 1.  Cells without
  data (w_i = 0) have no estimate; they are set to the mean, 0.
* LSQ-Wiener filter (section 4.1.1, the LSQ equation with the mask operator,
  the noise covariance and the observed overdensity defined there):
      delta = B^-1 (S^-1 + W^T N^-1 W)^-1 W^T N^-1 delta_o,
  W = diag(w), N = diag(w / nbar), delta_o = counts / nbar - w, unit bias
  B = 1.  Written out: W^T N^-1 W = diag(nbar w) and W^T N^-1 delta_o =
  counts - nbar w, so delta solves (S^-1 + diag(nbar w)) delta = counts -
  nbar w.  ``lsq_dense`` forms that matrix (S^-1 from ``model.prior_matrix``)
  and solves it; ``lsq_pcg`` solves the same system by preconditioned CG in
  spectral coordinates (``newton.pcg`` with d = nbar w).
* Correlation coefficient r and Euclidean distance D_Euc (section 4.1.2),
  written out as defined.
"""
import numpy as np

from . import model
from .newton import SpectralOps, pcg


def inverse_weighted_counts(prob):
    """N_i / w_i (0 where w_i = 0)."""
    w = prob.w
    return np.where(w > 0, prob.counts / np.where(w > 0, w, 1.0), 0.0)


def inverse_weight(prob):
    """delta_IW = N_i / (w_i nbar) - 1, and 0 where w_i = 0."""
    return np.where(prob.w > 0, inverse_weighted_counts(prob) / prob.nbar - 1.0, 0.0)


def lsq_dense(prob):
    """LSQ-Wiener overdensity by a dense solve (grids up to 16^3)."""
    A = model.prior_matrix(prob) + np.diag((prob.nbar * prob.w).ravel())
    b = (prob.counts - prob.nbar * prob.w).ravel()
    return np.linalg.solve(A, b).reshape(prob.n)


def lsq_pcg(prob, rtol=1e-12, max_cg=20000):
    """LSQ-Wiener overdensity by spectral PCG; returns (delta, its)."""
    ops = SpectralOps(prob)
    rhs = ops.fwd(prob.counts - prob.nbar * prob.w)
    x, its, _ = pcg(ops, prob.nbar * prob.w, rhs, rtol * ops.norm(rhs), max_cg)
    return ops.inv(x), its


def corr_coeff(rec, ref):
    """r = sum_i ref_i rec_i / (sqrt(sum_i ref_i^2) sqrt(sum_j rec_j^2))."""
    rec = np.asarray(rec, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.sum(ref * rec) / (np.sqrt(np.sum(ref * ref)) * np.sqrt(np.sum(rec * rec))))


def euclidean_distance(rec, ref):
    """D_Euc = sqrt((1 / N_cells) sum_i (rec_i - ref_i)^2)."""
    rec = np.asarray(rec, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.sqrt(np.mean((rec - ref) ** 2)))
