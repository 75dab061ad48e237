"""Principal branch W0 of the Lambert W function (w e^w = x), for x >= 0.

Test infrastructure only (see the package docstring).

Halley's iteration as described by Corless, Gonnet, Hare, Jeffrey & Knuth
(1996), "On the Lambert W function", Adv. Comput. Math. 5, section 4:

    w_{j+1} = w_j - f / (e^{w_j}(w_j + 1) - (w_j + 2) f / (2 w_j + 2)),
    f = w_j e^{w_j} - x.

For arguments too large to represent, ``lambertw_exp(L)`` returns W(e^L) by
solving w + ln w = L with Newton's method in log space.
"""
import numpy as np


def lambertw(x, tol=1e-15, max_iter=100):
    x = np.asarray(x, dtype=np.float64)
    if np.any(x < 0):
        raise ValueError("lambertw: only x >= 0 is supported")
    # starting guess: log1p(x) is within a factor ~2 of W(x) for x >= 0,
    # refined by one asymptotic correction for large x
    w = np.log1p(x)
    big = x > 3.0
    lx = np.log(np.where(big, x, 3.0))
    w = np.where(big, lx - np.log(lx), w)
    for _ in range(max_iter):
        ew = np.exp(w)
        f = w * ew - x
        wp1 = w + 1.0
        denom = ew * wp1 - (w + 2.0) * f / (2.0 * wp1)
        step = f / denom
        w_new = w - step
        done = np.all(np.abs(step) <= tol * (1.0 + np.abs(w_new)))
        w = w_new
        if done:
            break
    return w


def lambertw_exp(L, tol=1e-15, max_iter=100):
    """W(e^L) for real L, robust for L far above the float overflow limit.

    Solves h(w) = w + ln w - L = 0 (the logarithm of w e^w = e^L) by Newton's
    method, h'(w) = 1 + 1/w; for L below 1 it falls back to ``lambertw``.
    """
    L = np.asarray(L, dtype=np.float64)
    out = np.empty_like(L)
    small = L < 1.0
    if np.any(small):
        out[small] = lambertw(np.exp(L[small]), tol, max_iter)
    if np.any(~small):
        Lb = L[~small]
        w = np.maximum(Lb - np.log(Lb), 0.5)
        for _ in range(max_iter):
            h = w + np.log(w) - Lb
            step = h / (1.0 + 1.0 / w)
            w_new = w - step
            done = np.all(np.abs(step) <= tol * (1.0 + np.abs(w_new)))
            w = w_new
            if done:
                break
        out[~small] = w
    return out
