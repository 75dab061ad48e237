"""MAP with the linear (non-local) bias of sections 2.2.1 and 2.4.1.

Test infrastructure only (see the package docstring).

The galaxy overdensity is a linear function of the matter overdensity,
delta_g,i = sum_j b_ij delta_M,j (section 2.2.1).  For a translation-invariant
b_ij the operator B is a convolution, diagonal in Fourier space with the real
multiplier b_hat(k) (section 2.2.1 gives b_hat(k) = sqrt(P_g(k) / P_M(k))), so
B is symmetric whenever b_hat(-k) = b_hat(k).  Expected counts are
nbar w_i (1 + (B delta_M)_i) (eq. 2).  Two priors:

* lognormal (section 2.3): the unknown is s = ln(1 + delta_M), so
  delta_M = exp(s) - 1, with prior 1/2 (s - mu)^T S_L^-1 (s - mu);
* Gaussian (section 2.2): the unknown is delta_M itself, prior
  1/2 delta^T S^-1 delta (zero mean).

Writing x for the unknown, phi(x) for delta_M as a function of it and
y = 1 + B phi(x), the negative log-posterior without its constants is

    f(x) = 1/2 (x - m)^T S^-1 (x - m) + sum_i [nbar w_i y_i - N_i ln y_i],

whose gradient is the left side minus the right side of the linear-bias MAP
equations (section 2.2.1 for the Gaussian prior, section 2.4.1 for the
lognormal one),

    g = S^-1 (x - m) + phi'(x) * B^T u,        u = nbar w - N / y,

and whose Hessian is

    H = S^-1 + diag(phi''(x) * B^T u) + diag(phi') B^T diag(N / y^2) B diag(phi').

For the Gaussian prior phi'' = 0 and H is positive semi-definite; for the
lognormal prior the middle term can be negative, so the Newton system can be
indefinite away from the MAP.  The domain is y > 0 in every cell with counts.
With b_hat = 1 both reduce to the unit-bias models (``model`` with beta = 1,
``gaussian``) up to the constant sum_i nbar w_i.
"""
import numpy as np
from scipy.optimize import minimize

from . import dft, model
from .grid import hermitian_weights, inv_lambda_half

LOGNORMAL = 0
GAUSSIAN = 1


def phi(kind, x):
    """delta_M as a function of the unknown (section 2.3: delta = exp(s) - 1)."""
    return np.expm1(x) if kind == LOGNORMAL else np.array(x, dtype=np.float64)


def dphi(kind, x):
    return np.exp(x) if kind == LOGNORMAL else np.ones_like(x)


def d2phi(kind, x):
    return np.exp(x) if kind == LOGNORMAL else np.zeros_like(x)


def prior_mean(prob, kind):
    return prob.mu if kind == LOGNORMAL else 0.0


def bias_apply(bk, x):
    """B x = F^-1 diag(b_hat) F x (B^T x for a real, even b_hat)."""
    return dft.irfftn(dft.rfftn(x) * bk, x.shape)


def bias_full(bk, n):
    """b_hat on the full (nx, ny, nz) spectrum from its half spectrum, using
    b_hat(-k) = b_hat(k)."""
    full = np.empty(n)
    nh = n[2] // 2 + 1
    full[:, :, :nh] = bk
    for mz in range(nh, n[2]):
        src = bk[:, :, n[2] - mz]
        full[:, :, mz] = src[(-np.arange(n[0])) % n[0]][:, (-np.arange(n[1])) % n[1]]
    return full


def bias_matrix(bk, n):
    """Dense N x N matrix of B from the DFT definition: B[a, b] = beta(a - b)
    with the kernel beta = F^-1 b_hat (small grids only)."""
    kern = np.real(dft.idftn(bias_full(bk, n)))
    ix, iy, iz = (np.arange(v) for v in n)
    dx = (ix[:, None] - ix[None, :]) % n[0]
    dy = (iy[:, None] - iy[None, :]) % n[1]
    dz = (iz[:, None] - iz[None, :]) % n[2]
    M = kern[dx[:, None, None, :, None, None], dy[None, :, None, None, :, None],
             dz[None, None, :, None, None, :]]
    N = n[0] * n[1] * n[2]
    return M.reshape(N, N)


def galaxy_field(prob, bk, x, kind):
    """y = 1 + B phi(x): the expected counts divided by nbar w (eq. 2)."""
    return 1.0 + bias_apply(bk, phi(kind, x))


def likelihood(prob, y):
    """sum_i [nbar w_i y_i - N_i ln y_i] (eq. 3 without its constants); +inf
    outside the domain (y <= 0 in a cell with counts)."""
    pos = prob.counts > 0
    if np.any(y[pos] <= 0.0):
        return np.inf
    return float(np.sum(prob.nbar * prob.w * y) - np.sum(prob.counts[pos] * np.log(y[pos])))


def objective(prob, bk, x, kind):
    xm = x - prior_mean(prob, kind)
    return 0.5 * float(np.sum(xm * model.prior_apply(prob, xm))) + likelihood(prob, galaxy_field(prob, bk, x, kind))


def gradient(prob, bk, x, kind):
    y = galaxy_field(prob, bk, x, kind)
    u = prob.nbar * prob.w - np.where(prob.counts > 0, prob.counts / y, 0.0)
    return model.prior_apply(prob, x - prior_mean(prob, kind)) + dphi(kind, x) * bias_apply(bk, u)


def lik_hessvec(prob, bk, x, v, kind):
    """Likelihood part of H v: phi'' (B u) v + phi' B [(N / y^2) B (phi' v)]."""
    y = galaxy_field(prob, bk, x, kind)
    u = prob.nbar * prob.w - np.where(prob.counts > 0, prob.counts / y, 0.0)
    W = np.where(prob.counts > 0, prob.counts / y ** 2, 0.0)
    a = dphi(kind, x)
    return d2phi(kind, x) * bias_apply(bk, u) * v + a * bias_apply(bk, W * bias_apply(bk, a * v))


def hessvec(prob, bk, x, v, kind):
    return model.prior_apply(prob, v) + lik_hessvec(prob, bk, x, v, kind)


# ---------------------------------------------------------------------------
# Dense forms (grids up to 8^3): brute force from the DFT definitions
# ---------------------------------------------------------------------------

def objective_dense(prob, bk, x, kind):
    """f from dense matrices of S^-1 and B (no FFT anywhere)."""
    Sinv = model.prior_matrix(prob)
    B = bias_matrix(bk, prob.n)
    xm = (x - prior_mean(prob, kind)).ravel()
    y = (1.0 + B @ phi(kind, x).ravel()).reshape(prob.n)
    return 0.5 * float(xm @ Sinv @ xm) + likelihood(prob, y)


def map_dense(prob, bk, kind, gtol_rel=1e-11):
    """MAP by scipy's trust-region Newton (exact dense Hessian) on ``objective``
    and ``gradient``: a library minimiser standing beside the spectral one."""
    n = prob.n
    x0 = np.full(n, prior_mean(prob, kind))
    g0 = np.linalg.norm(gradient(prob, bk, x0, kind))
    Sinv = model.prior_matrix(prob)
    B = bias_matrix(bk, n)

    def f(v):
        return objective(prob, bk, v.reshape(n), kind)

    def g(v):
        return gradient(prob, bk, v.reshape(n), kind).ravel()

    def h(v):
        x = v.reshape(n)
        y = galaxy_field(prob, bk, x, kind).ravel()
        cnt = prob.counts.ravel()
        u = prob.nbar * prob.w.ravel() - np.where(cnt > 0, cnt / y, 0.0)
        W = np.where(cnt > 0, cnt / y ** 2, 0.0)
        a = dphi(kind, x).ravel()
        return Sinv + np.diag(d2phi(kind, x).ravel() * (B.T @ u)) + (a[:, None] * B.T) @ (W[:, None] * B * a[None, :])

    res = minimize(f, x0.ravel(), jac=g, hess=h, method="trust-exact",
                   options={"gtol": gtol_rel * g0, "maxiter": 500})
    # the trust region stops once f no longer resolves the decrease; full
    # Newton steps with the dense Hessian take the gradient the rest of the way
    v = res.x
    gv = g(v)
    for _ in range(20):
        if np.linalg.norm(gv) <= gtol_rel * g0:
            break
        v_new = v - np.linalg.solve(h(v), gv)
        g_new = g(v_new)
        if not np.linalg.norm(g_new) < np.linalg.norm(gv):
            break
        v, gv = v_new, g_new
    return v.reshape(n), res


# ---------------------------------------------------------------------------
# Spectral inexact Newton with a truncated PCG (any grid size)
# ---------------------------------------------------------------------------

def _dot(c, N, a, b):
    return float(np.sum(c * (np.conj(a) * b).real) / N)


def truncated_pcg(prob, bk, x, kind, g_hat, tol_abs, max_cg, precond="p25"):
    """PCG on H p = -g in half-spectrum coordinates, stopped at ||r|| <= tol_abs
    or at the first direction of non-positive curvature.  If that happens
    before any step, the preconditioned steepest-descent direction M^-1 (-g)
    is returned.  Preconditioner M_k = 1/lambda_k + c with c, over the cells
    of deff = max(0, phi'^2 N / y^2 + phi'' B^T u), either the 25th
    percentile floored at 1e-3 times the mean (precond="p25") or the mean
    itself (precond="mean").  The paper gives no preconditioner; the constant
    changes the iteration path, and the tests check that the minimiser
    reached from the prior mean does not depend on it."""
    n, N = prob.n, prob.ncells
    cw = hermitian_weights(n)
    inv_lam = inv_lambda_half(prob)
    y = galaxy_field(prob, bk, x, kind)
    u = prob.nbar * prob.w - np.where(prob.counts > 0, prob.counts / y, 0.0)
    a = dphi(kind, x)
    deff = a * a * np.where(prob.counts > 0, prob.counts / y ** 2, 0.0) + d2phi(kind, x) * bias_apply(bk, u)
    deff = np.maximum(deff, 0.0)
    if precond == "mean":
        c = float(np.mean(deff))
    else:
        c = max(float(np.percentile(deff, 25)), 1e-3 * float(np.mean(deff)))
    M = inv_lam + c
    Minv = np.where(M > 0, 1.0 / np.where(M > 0, M, 1.0), 0.0)
    sol = np.zeros_like(g_hat)
    r = -g_hat
    z = Minv * r
    p = z.copy()
    rz = _dot(cw, N, r, z)
    its = 0
    for k in range(max_cg):
        if np.sqrt(_dot(cw, N, r, r)) <= tol_abs:
            break
        # H p with the prior term as an exact pointwise product (section 2.3)
        q = inv_lam * p + dft.rfftn(lik_hessvec(prob, bk, x, dft.irfftn(p, n), kind))
        pq = _dot(cw, N, p, q)
        if pq <= 0.0:
            if k == 0:
                sol = z
            break
        alpha = rz / pq
        sol = sol + alpha * p
        r = r - alpha * q
        its = k + 1
        z = Minv * r
        rz_new = _dot(cw, N, r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return sol, its


def _spectral_grad(prob, bk, x_hat, kind, inv_lam, m_hat):
    """Real field x = F^-1 x_hat and the gradient spectrum
    g_hat = (x_hat - m_hat) / lambda + F[phi'(x) B u]: with the iterate held
    as its spectrum the prior term is an exact pointwise product (section 2.3:
    S^-1 is diagonal in Fourier space), so the gradient has no FFT-roundoff
    floor from the large 1/lambda of high-k modes."""
    x = dft.irfftn(x_hat, prob.n)
    y = galaxy_field(prob, bk, x, kind)
    u = prob.nbar * prob.w - np.where(prob.counts > 0, prob.counts / y, 0.0)
    return x, inv_lam * (x_hat - m_hat) + dft.rfftn(dphi(kind, x) * bias_apply(bk, u))


def _armijo(prob, bk, x, p, b, c, slope, kind, c1=1e-4, max_halvings=60):
    """Armijo backtracking from a = 1 (halving) on the decrease in difference
    form: a b + a^2 c / 2 + sum_i [nbar w_i dy_i - N_i log1p(dy_i / y_i)] with
    b = p^T S^-1 (x - m), c = p^T S^-1 p and dy = B (phi(x + a p) - phi(x))
    (phi(x + a p) - phi(x) = exp(x) expm1(a p) for the lognormal prior); a step
    that leaves y <= 0 in a cell with counts is rejected."""
    if slope >= 0:
        return None
    y = galaxy_field(prob, bk, x, kind)
    pos = prob.counts > 0
    a = 1.0
    for _ in range(max_halvings):
        with np.errstate(over="ignore", invalid="ignore"):
            dphi_a = np.exp(x) * np.expm1(a * p) if kind == LOGNORMAL else a * p
            dy = bias_apply(bk, dphi_a)
            if np.all(np.isfinite(dy)) and np.all(y[pos] + dy[pos] > 0.0):
                lik = float(np.sum(prob.nbar * prob.w * dy) - np.sum(prob.counts[pos] * np.log1p(dy[pos] / y[pos])))
                if a * b + 0.5 * a * a * c + lik <= c1 * a * slope:
                    return a
        a *= 0.5
    return None


def newton_spectral(prob, bk, kind, rtol=1e-12, max_newton=200, max_cg=20000, eta_max=0.5, precond="p25"):
    """Inexact Newton with the truncated PCG (preconditioner constant as in
    ``truncated_pcg``), from x0 = m (uniform), the iterate held as its half
    spectrum.  Returns (x, info) with info =
    dict(newton_its, cg_its, status, rel_grad); norms are those of the
    spectral gradient (Parseval)."""
    n, N = prob.n, prob.ncells
    cw = hermitian_weights(n)
    inv_lam = inv_lambda_half(prob)
    m_hat = np.zeros(inv_lam.shape, dtype=np.complex128)
    m_hat[0, 0, 0] = N * prior_mean(prob, kind)
    x_hat = dft.rfftn(np.full(n, prior_mean(prob, kind)))
    x, g_hat = _spectral_grad(prob, bk, x_hat, kind, inv_lam, m_hat)
    gn = g0 = np.sqrt(_dot(cw, N, g_hat, g_hat))
    info = {"newton_its": 0, "cg_its": 0, "status": "ok", "rel_grad": 0.0}
    if g0 == 0.0:
        return x, info
    for it in range(max_newton):
        if gn <= rtol * g0:
            break
        eta = min(eta_max, max(np.sqrt(gn / g0), 0.5 * rtol * g0 / gn))
        p_hat, its = truncated_pcg(prob, bk, x, kind, g_hat, eta * gn, max_cg, precond)
        info["cg_its"] += its
        Sp = inv_lam * p_hat
        b = _dot(cw, N, Sp, x_hat - m_hat)
        c = _dot(cw, N, Sp, p_hat)
        slope = _dot(cw, N, g_hat, p_hat)
        a = _armijo(prob, bk, x, dft.irfftn(p_hat, n), b, c, slope, kind)
        if a is None:
            info["status"] = "linesearch"
            break
        x_hat = x_hat + a * p_hat
        x, g_hat = _spectral_grad(prob, bk, x_hat, kind, inv_lam, m_hat)
        gn = np.sqrt(_dot(cw, N, g_hat, g_hat))
        info["newton_its"] = it + 1
    else:
        if gn > rtol * g0:
            info["status"] = "not_converged"
    info["rel_grad"] = float(gn / g0)
    return x, info


# ---------------------------------------------------------------------------
# Closed form: white prior, local constant bias
# ---------------------------------------------------------------------------

def white_prior_map(kind, sigma2, m, b0, nbar, w, counts, iters=200):
    """Per-cell MAP for S = sigma2 I and b_hat = b0 (B = b0 I): the root of
    (x - m) / sigma2 + b0 phi'(x) (nbar w - N / (1 + b0 phi(x))) = 0, found by
    bisection over the domain 1 + b0 phi(x) > 0 (cells with counts).  The root
    is unique when the per-cell curvature is positive: b0 >= 1 for the
    lognormal prior, any b0 > 0 for the Gaussian one."""
    w = np.asarray(w, dtype=np.float64)
    counts = np.asarray(counts, dtype=np.float64)
    pos = counts > 0

    def h(x):
        with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
            y = 1.0 + b0 * phi(kind, x)
            out = (x - m) / sigma2 + b0 * dphi(kind, x) * (nbar * w - np.where(pos, counts / y, 0.0))
        # outside the domain (or on its edge) the gradient is taken as -inf
        return np.where(pos & ~(y > 0), -np.inf, out)

    # the domain edge 1 + b0 phi(x) = 0 bounds the root from below in cells
    # with counts; elsewhere (and for b0 <= 1, lognormal) a point far left
    # where h < 0 does
    if kind == LOGNORMAL:
        edge = np.log1p(-1.0 / b0) if b0 > 1.0 else -np.inf
    else:
        edge = -1.0 / b0
    far = m - 50.0 * sigma2 - 50.0
    lo = np.where(pos & np.isfinite(edge), edge if np.isfinite(edge) else far, far)
    hi = np.full(w.shape, m + 50.0)
    assert np.all(h(lo) < 0) and np.all(h(hi) > 0), "root not bracketed"
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        neg = h(mid) < 0
        lo = np.where(neg, mid, lo)
        hi = np.where(neg, hi, mid)
    return 0.5 * (lo + hi)
