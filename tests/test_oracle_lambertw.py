"""Pins for the Lambert W implementation (Corless et al. 1996)."""
import numpy as np

from oracle.lambertw import lambertw, lambertw_exp


def test_special_values():
    # W(0) = 0, W(e) = 1, W(1) = Omega, W(2 ln 2) = ln 2, W(-1/e) excluded (x >= 0 only)
    vals = lambertw(np.array([0.0, np.e, 1.0, 2 * np.log(2.0)]))
    np.testing.assert_allclose(vals, [0.0, 1.0, 0.5671432904097838, np.log(2.0)], rtol=1e-15, atol=1e-300)


def test_defining_identity(rng):
    # w e^w = x; for large x the identity is checked in log form, since an
    # ulp of w is amplified by a factor w in e^w
    x = np.exp(rng.uniform(-30, 600, size=2000))
    w = lambertw(x)
    small = x < 150.0
    np.testing.assert_allclose(w[small] * np.exp(w[small]), x[small], rtol=4e-15)
    big = ~small
    np.testing.assert_allclose(w[big] + np.log(w[big]), np.log(x[big]), rtol=2e-15)


def test_log_space_branch(rng):
    L = rng.uniform(-20, 5000, size=2000)
    w = lambertw_exp(L)
    np.testing.assert_allclose(w + np.log(w), L, rtol=1e-14, atol=1e-14)
    small = L < 600
    np.testing.assert_allclose(w[small], lambertw(np.exp(L[small])), rtol=1e-14)
