"""Seeded synthetic inputs for the Poisson-lognormal MAP filter.

This module only draws inputs: a Gaussian log-density field with a given
power spectrum, a completeness (selection) field and Poisson counts.  It holds
none of the MAP method's arithmetic (no posterior, gradient, Hessian or
solver); both the HIP path and the CPU oracle take its arrays as plain inputs.

The paper's experiments use Poisson samples of an N-body simulation on a
256^3 grid over a 500 Mpc/h box (section 4.2) with radial completeness models
(Fig. 1).  Those data are not available; these generators stand in for them
with the same shapes: a periodic grid, ~2 Mpc/h cells, an observer at the box
centre, radial selection, optional blocky holes, and a lognormal density with
peaks of 1 + delta ~ 10^2-10^4.

Recipe (every config):
 1. white = default_rng([seed, 0]).standard_normal(n)
 2. G_hat = rfftn(white) * sqrt(lambda_k), lambda_k = A pk(k) N_cells / V,
    G_hat[0] = 0; G = irfftn(G_hat)
 3. s_true = G - sigma^2/2 (so 1 + delta = exp(G - sigma^2/2)), mu = -sigma^2/2
 4. w = exp(-(r/R)^2) about the box centre (cell centres at (i+1/2) dx), times
    a mask that zeroes round(frac * (n/8)^3) whole 8^3 blocks drawn without
    replacement by default_rng([seed, 1]); w = 1 when no selection is given
 5. N ~ Poisson(nbar w exp(beta s_true)) from default_rng([seed, 2]), stored
    as float64
The spectrum shape is pk(k) = k^-1.5 exp(-(2 k)^2) (k in h/Mpc, pk(0) = 0) and
A is set so that the ensemble cell variance (1/V) sum_{k != 0} A pk(k) over
all grid modes equals sigma^2.
"""
import os

import numpy as np
import scipy.fft

_WORKERS = os.cpu_count() or 1

__all__ = ["power_shape_half", "amplitude_for_sigma", "make_instance", "CONFIGS",
           "config_instance", "batch_instances", "hermitian_multiplicity"]


def _fold(n):
    m = np.arange(n)
    return np.where(m >= n // 2, m - n, m)


def _kmag_half(n, box):
    if box[0] == box[1] == box[2]:
        # |k| from the exact integer m^2 = mx^2 + my^2 + mz^2: every mode of
        # a shell gets a bitwise identical |k|, so the spectrum is exactly
        # isotropic (no rounding differences between permuted components)
        m2 = (_fold(n[0])[:, None, None] ** 2 + _fold(n[1])[None, :, None] ** 2
              + np.arange(n[2] // 2 + 1)[None, None, :] ** 2)
        return (2 * np.pi / box[0]) * np.sqrt(m2.astype(np.float64))
    kx = (2 * np.pi / box[0]) * _fold(n[0]).astype(np.float64)
    ky = (2 * np.pi / box[1]) * _fold(n[1]).astype(np.float64)
    kz = (2 * np.pi / box[2]) * np.arange(n[2] // 2 + 1, dtype=np.float64)
    return np.sqrt(kx[:, None, None] ** 2 + ky[None, :, None] ** 2 + kz[None, None, :] ** 2)


def hermitian_multiplicity(n):
    """How many full-spectrum modes each stored half-spectrum entry stands for."""
    c = np.full((n[0], n[1], n[2] // 2 + 1), 2.0)
    c[:, :, 0] = 1.0
    c[:, :, n[2] // 2] = 1.0
    return c


def power_shape_half(n, box, slope=-1.5, smooth=2.0):
    """pk(k) = k^slope exp(-(smooth k)^2) on the half spectrum; pk(0) = 0."""
    k = _kmag_half(n, box)
    pk = np.zeros_like(k)
    nz = k > 0
    pk[nz] = k[nz] ** slope * np.exp(-(smooth * k[nz]) ** 2)
    return pk


def bias_multiplier_half(n, box, b0=1.0, smooth=3.0):
    """Linear-bias multiplier b_hat(k) = b0 exp(-(smooth k)^2 / 2) on the half
    spectrum: a galaxy field that is a smoothed copy of the matter field
    (smooth in Mpc/h).  Deterministic and even in k."""
    k = _kmag_half(n, box)
    return b0 * np.exp(-0.5 * (smooth * k) ** 2)


def amplitude_for_sigma(pk_shape, n, box, sigma):
    vol = box[0] * box[1] * box[2]
    total = float(np.sum(hermitian_multiplicity(n) * pk_shape)) / vol
    return sigma * sigma / total


def make_instance(n, box, sigma, nbar, beta=1.0, radius=None, mask_frac=0.0,
                  seed=0, block=8):
    n = tuple(int(v) for v in n)
    box = tuple(float(v) for v in box)
    ncell = n[0] * n[1] * n[2]
    vol = box[0] * box[1] * box[2]
    pk = power_shape_half(n, box)
    amp = amplitude_for_sigma(pk, n, box, sigma)
    white = np.random.default_rng([seed, 0]).standard_normal(n)
    lam = amp * pk * ncell / vol
    g_hat = scipy.fft.rfftn(white, workers=_WORKERS)
    g_hat *= np.sqrt(lam)
    g_hat[0, 0, 0] = 0.0
    G = scipy.fft.irfftn(g_hat, s=n, axes=(0, 1, 2), workers=_WORKERS)
    del white, g_hat, lam
    mu = -0.5 * sigma * sigma
    s_true = G - 0.5 * sigma * sigma
    del G
    if radius is None:
        w = np.ones(n)
    else:
        ax = [(np.arange(n[i]) + 0.5) * (box[i] / n[i]) - 0.5 * box[i] for i in range(3)]
        r2 = ax[0][:, None, None] ** 2 + ax[1][None, :, None] ** 2 + ax[2][None, None, :] ** 2
        w = np.exp(-r2 / (radius * radius))
        del r2
    if mask_frac > 0:
        nb = tuple(v // block for v in n)
        nblocks = nb[0] * nb[1] * nb[2]
        k = int(round(mask_frac * nblocks))
        pick = np.random.default_rng([seed, 1]).choice(nblocks, size=k, replace=False)
        bm = np.ones(nblocks)
        bm[pick] = 0.0
        bm = bm.reshape(nb)
        w = w * np.repeat(np.repeat(np.repeat(bm, block, 0), block, 1), block, 2)
    rate = nbar * w * np.exp(beta * s_true)
    counts = np.random.default_rng([seed, 2]).poisson(rate).astype(np.float64)
    return dict(n=n, box=box, w=w, counts=counts, pk=pk, amp=amp, mu=mu, nbar=float(nbar),
                beta=float(beta), inv_p0=0.0, s_true=s_true, sigma=float(sigma), seed=seed)


# Workloads (grid, box in Mpc/h, sigma_G, nbar, beta, selection radius, mask fraction)
CONFIGS = {
    "plain32": dict(n=(32, 32, 32), box=(100.0,) * 3, sigma=1.0, nbar=1.0, beta=1.0,
                    radius=None, mask_frac=0.0, rtol=1e-8),
    "sel256": dict(n=(256, 256, 256), box=(500.0,) * 3, sigma=1.5, nbar=0.5, beta=1.0,
                   radius=200.0, mask_frac=0.2, rtol=1e-6),
    "bias256": dict(n=(256, 256, 256), box=(500.0,) * 3, sigma=1.5, nbar=2.0, beta=1.5,
                    radius=200.0, mask_frac=0.2, rtol=1e-6),
    "big512": dict(n=(512, 512, 512), box=(1000.0,) * 3, sigma=2.0, nbar=0.2, beta=1.2,
                   radius=400.0, mask_frac=0.0, rtol=1e-6),
}


def config_instance(name, seed=0, n=None):
    """Instance of a named workload; ``n`` overrides the grid (same cell size)."""
    c = dict(CONFIGS[name])
    if n is not None:
        scale = n / c["n"][0]
        c["box"] = tuple(b * scale for b in c["box"])
        if c["radius"] is not None:
            c["radius"] = c["radius"] * scale
        c["n"] = (n, n, n)
    return make_instance(c["n"], c["box"], c["sigma"], c["nbar"], c["beta"],
                         radius=c["radius"], mask_frac=c["mask_frac"], seed=seed)


def batch_instances(count=64, sizes=(32, 48, 64, 96), master_seed=3):
    """Independent instances of uneven size: n from ``sizes`` uniformly,
    box 3.125 n Mpc/h, sigma ~ U[0.8, 1.8], nbar log-uniform on [0.1, 5],
    unit bias, w = 1; instance i uses seed i."""
    rng = np.random.default_rng([master_seed, 99])
    ns = rng.choice(np.asarray(sizes), size=count)
    sig = rng.uniform(0.8, 1.8, size=count)
    nb = np.exp(rng.uniform(np.log(0.1), np.log(5.0), size=count))
    out = []
    for i in range(count):
        n = int(ns[i])
        out.append(make_instance((n, n, n), (3.125 * n,) * 3, float(sig[i]), float(nb[i]),
                                 1.0, radius=None, mask_frac=0.0, seed=i))
    return out
