"""The lognormal prior built from a matter spectrum (section 2.3).

Test infrastructure only (see the package docstring).

The covariance S of the overdensity has eigenvalues lambda_k = A pk_k N / V
(the normalisation under which S(0) is the cell variance).  Its correlation
function is S(r) = F^-1 lambda (inverse transform with 1/N); the signal
s = ln(1 + delta) has the correlation function S_L(r) = ln(1 + S(r)) (the
transformation equation of section 2.3), eigenvalues lambda^L = F S_L and
mean mu = -sigma0^2 / 2 with sigma0^2 = S_L(0) (the mean-field equation).

The log transform need not keep every eigenvalue positive; values at or
below 1e-10 S_L(0) (S_L(0) is their mean) are raised to it -- a reading, the
paper is silent.  The returned spectrum is P_L = lambda^L V / N (to be used
with amplitude 1).
"""
import numpy as np

from . import dft

FLOOR_REL = 1e-10


def correlation_function(n, box, pk, amp):
    """S(r) on the grid of separations from the half spectrum pk."""
    N = n[0] * n[1] * n[2]
    V = box[0] * box[1] * box[2]
    return dft.irfftn(amp * np.asarray(pk, dtype=np.float64) * N / V, n)


def lognormal_prior(n, box, pk, amp):
    """Returns (P_L half spectrum, mu, sigma0^2, number of raised k != 0 modes)."""
    N = n[0] * n[1] * n[2]
    V = box[0] * box[1] * box[2]
    S = correlation_function(n, box, pk, amp)
    if np.any(S <= -1.0):
        raise ValueError("the correlation function reaches -1")
    SL = np.log1p(S)
    lam_L = dft.rfftn(SL).real
    floor = FLOOR_REL * abs(SL[0, 0, 0])
    low = ~(lam_L > floor)
    k0 = np.zeros_like(low)
    k0[0, 0, 0] = True
    n_clipped = int(np.sum(low & ~k0))
    lam_L = np.where(low, floor, lam_L)
    return lam_L * V / N, -0.5 * SL[0, 0, 0], SL[0, 0, 0], n_clipped
