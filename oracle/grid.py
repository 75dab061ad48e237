"""Periodic grid, Fourier-mode bookkeeping and the prior's eigenvalues.

Test infrastructure only (see the package docstring).

Section 2.2 states that applying the signal covariance S to a field is a
convolution over the cells of the periodic box, so S is diagonal in Fourier
space with the power spectrum on its diagonal; section 2.3 states the same for
the lognormal covariance S_L.  The discrete eigenvalue convention (the paper
defers it to an earlier reference that is not available) is taken as

    lambda_k = P(|k|) * N_cells / V,

so that the ensemble variance of a cell is (1/V) * sum_k P(k), the discrete
counterpart of the continuum statement FT(S) = (2 pi)^3 P delta_D.  The k = 0
mode's inverse eigenvalue is an explicit input ``inv_p0`` (0 by default: the
mean of s is then fixed by the data alone).
"""
import numpy as np


class Problem:
    """Inputs of the posterior (sections 2.1-2.4), as plain FP64 arrays.

    n      -- grid shape (nx, ny, nz), real fields are C-ordered [x][y][z]
    box    -- box side lengths (Lx, Ly, Lz) in Mpc/h
    w      -- completeness per cell, shape n (eq. 2)
    counts -- observed galaxy counts per cell (non-negative integers), shape n
    pk     -- power spectrum shape per half-spectrum mode, shape
              (nx, ny, nz//2+1), (Mpc/h)^3; multiplied by ``amp``; the k = 0
              entry is ignored
    amp    -- power spectrum amplitude A
    mu     -- uniform prior mean of s (eq. mu)
    nbar   -- mean count per cell (eq. 2)
    beta   -- power-law bias exponent: 1 + delta_g = (1 + delta_M)^beta
    inv_p0 -- inverse prior eigenvalue of the k = 0 mode
    """

    def __init__(self, n, box, w, counts, pk, amp, mu, nbar, beta=1.0, inv_p0=0.0):
        self.n = tuple(int(v) for v in n)
        self.box = tuple(float(v) for v in box)
        self.w = np.asarray(w, dtype=np.float64).reshape(self.n)
        self.counts = np.asarray(counts, dtype=np.float64).reshape(self.n)
        nh = (self.n[0], self.n[1], self.n[2] // 2 + 1)
        self.pk = np.asarray(pk, dtype=np.float64).reshape(nh)
        self.amp = float(amp)
        self.mu = float(mu)
        self.nbar = float(nbar)
        self.beta = float(beta)
        self.inv_p0 = float(inv_p0)

    def replace(self, **kw):
        d = dict(n=self.n, box=self.box, w=self.w, counts=self.counts, pk=self.pk,
                 amp=self.amp, mu=self.mu, nbar=self.nbar, beta=self.beta,
                 inv_p0=self.inv_p0)
        d.update(kw)
        return Problem(**d)

    @property
    def ncells(self):
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def volume(self):
        return self.box[0] * self.box[1] * self.box[2]


def folded_index(n):
    """Integer mode numbers of a length-n axis, folded to [-n/2, n/2)."""
    m = np.arange(n)
    return np.where(m >= (n + 1) // 2, m - n, m) if n % 2 else np.where(m >= n // 2, m - n, m)


def half_shape(n):
    return (n[0], n[1], n[2] // 2 + 1)


def mode_vectors_half(n, box):
    """Wave-vector components (kx, ky, kz) on the half spectrum, in h/Mpc."""
    mx = folded_index(n[0]).astype(np.float64)
    my = folded_index(n[1]).astype(np.float64)
    mz = np.arange(n[2] // 2 + 1, dtype=np.float64)
    kx = (2 * np.pi / box[0]) * mx[:, None, None]
    ky = (2 * np.pi / box[1]) * my[None, :, None]
    kz = (2 * np.pi / box[2]) * mz[None, None, :]
    return kx, ky, kz


def kmag_half(n, box):
    kx, ky, kz = mode_vectors_half(n, box)
    return np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)


def hermitian_weights(n):
    """Multiplicity of each stored half-spectrum mode in the full spectrum.

    The planes kz = 0 and kz = nz/2 hold both k and -k, so each of their
    entries counts once; every other stored entry stands for itself and its
    conjugate partner, so it counts twice.
    """
    c = np.full(half_shape(n), 2.0)
    c[:, :, 0] = 1.0
    if n[2] % 2 == 0:
        c[:, :, n[2] // 2] = 1.0
    return c


def inv_lambda_half(prob):
    """Inverse prior eigenvalues 1/lambda_k on the half spectrum (section 2.3:
    S_L acts as a convolution, so S_L^-1 is diagonal in Fourier space)."""
    lam = prob.amp * prob.pk * prob.ncells / prob.volume
    inv = np.full_like(lam, np.inf)
    pos = lam > 0
    inv[pos] = 1.0 / lam[pos]
    inv[0, 0, 0] = prob.inv_p0
    return inv


def inv_lambda_full(prob):
    """Same as ``inv_lambda_half`` on the full (nx, ny, nz) spectrum, using
    lambda(-k) = lambda(k) (the prior is a real, even convolution kernel)."""
    n = prob.n
    half = inv_lambda_half(prob)
    full = np.empty(n)
    nh = n[2] // 2 + 1
    full[:, :, :nh] = half
    # mode (mx, my, mz) with mz > nz/2 equals the conjugate of (-mx, -my, nz - mz)
    for mz in range(nh, n[2]):
        src = half[:, :, n[2] - mz]
        full[:, :, mz] = src[(-np.arange(n[0])) % n[0]][:, (-np.arange(n[1])) % n[1]]
    return full
