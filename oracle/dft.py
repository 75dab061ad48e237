"""Discrete Fourier transforms for the oracle.

Test infrastructure only (see the package docstring).

Convention (used for the prior operator of sections 2.2-2.3): the forward
transform is X_k = sum_x x_x exp(-2 pi i m.x / n), unnormalised; the inverse
carries the factor 1/N_cells.

``dftn`` / ``idftn`` write the transform out as dense DFT matrices applied
along each axis: this is the definition, O(n^4), usable up to n ~ 48.
``rfftn`` / ``irfftn`` call scipy's FFT (a library primitive, run on all host
cores) for the large grids; the tests pin them against the dense definition.
"""
import os

import numpy as np
import scipy.fft

_WORKERS = os.cpu_count() or 1


def dft_matrix(n, sign):
    """Dense matrix M[k, x] = exp(sign * 2 pi i k x / n)."""
    j = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / n)


def dftn(x):
    """Forward 3D DFT (unnormalised) of a real or complex array."""
    X = np.asarray(x, dtype=np.complex128)
    for axis in range(3):
        M = dft_matrix(X.shape[axis], -1)
        X = np.moveaxis(np.tensordot(M, X, axes=([1], [axis])), 0, axis)
    return X


def idftn(X):
    """Inverse 3D DFT with the 1/N normalisation."""
    x = np.asarray(X, dtype=np.complex128)
    for axis in range(3):
        M = dft_matrix(x.shape[axis], +1)
        x = np.moveaxis(np.tensordot(M, x, axes=([1], [axis])), 0, axis)
    return x / x.size


def rdftn(x):
    """Half spectrum (last axis 0..n/2) of the dense forward DFT of a real field."""
    n2 = x.shape[2]
    return dftn(x)[:, :, : n2 // 2 + 1]


def rfftn(x):
    return scipy.fft.rfftn(np.asarray(x, dtype=np.float64), workers=_WORKERS)


def irfftn(X, n):
    return scipy.fft.irfftn(X, s=n, axes=(0, 1, 2), workers=_WORKERS)
