"""torch.autograd face of the MAP reconstruction.

``map_reconstruct(plan, amp, beta, nbar, counts, w, pk, mu)`` returns the MAP
log-density s* of the Poisson-lognormal posterior (sections 2.1-2.4, 3.1) as a
differentiable function of the prior amplitude A, the bias exponent beta, the
mean count nbar, the counts N and the completeness w.  The forward pass is
the Newton-Krylov solve (pl_newton_krylov_solve); the backward pass is ONE
adjoint solve H(s*) lambda = dL/ds* (pl_solve_adjoint) followed by the
implicit-function products dL/dtheta = -lambda^T dg/dtheta, where
g(s*; theta) = 0 is the stationarity condition of the MAP.  Both run in the
library's kernels; this module only marshals tensors.
"""
import torch

from .binding import PLError

__all__ = ["MAPReconstruct", "map_reconstruct"]


def _scalar(x):
    return float(x.detach().item()) if torch.is_tensor(x) else float(x)


class MAPReconstruct(torch.autograd.Function):
    """forward(plan, amp, beta, nbar, counts, w, pk, mu, inv_p0, solve_opts, adjoint_opts) -> s*"""

    @staticmethod
    def forward(ctx, plan, amp, beta, nbar, counts, w, pk, mu, inv_p0, solve_opts, adjoint_opts):
        params = dict(amp=_scalar(amp), beta=_scalar(beta), nbar=_scalar(nbar), mu=float(mu),
                      inv_p0=float(inv_p0))
        counts_d = plan._dev(counts.detach())
        w_d = plan._dev(w.detach())
        pk_d = plan._dev(pk.detach() if torch.is_tensor(pk) else pk)
        plan.set_problem(w_d, counts_d, pk_d, **params)
        s, info = plan.solve(**solve_opts)
        if info["status"] != 0:
            raise PLError(info["status"], f"MAP solve: {info}")
        ctx.plan = plan
        ctx.params = params
        ctx.adjoint_opts = adjoint_opts
        ctx.fields = (w_d, counts_d, pk_d)
        ctx.save_for_backward(s)
        ctx.dtypes = (counts.dtype, w.dtype)
        return s

    @staticmethod
    def backward(ctx, grad_s):
        (s,) = ctx.saved_tensors
        plan = ctx.plan
        w_d, counts_d, pk_d = ctx.fields
        # the plan may have served other problems since the forward pass
        plan.set_problem(w_d, counts_d, pk_d, **ctx.params)
        want_fields = ctx.needs_input_grad[4] or ctx.needs_input_grad[5]
        grads, info = plan.adjoint(s, grad_s.contiguous(), want_fields=want_fields, **ctx.adjoint_opts)
        if info["status"] != 0:
            raise PLError(info["status"], f"adjoint solve: {info}")
        dev = s.device

        def sc(k):
            return torch.tensor(grads[k], dtype=torch.float64, device=dev)

        d_amp = sc("A") if ctx.needs_input_grad[1] else None
        d_beta = sc("beta") if ctx.needs_input_grad[2] else None
        d_nbar = sc("nbar") if ctx.needs_input_grad[3] else None
        d_counts = grads["N"].to(ctx.dtypes[0]) if ctx.needs_input_grad[4] else None
        d_w = grads["w"].to(ctx.dtypes[1]) if ctx.needs_input_grad[5] else None
        return None, d_amp, d_beta, d_nbar, d_counts, d_w, None, None, None, None, None


def map_reconstruct(plan, amp, beta, nbar, counts, w, pk, mu, inv_p0=0.0, solve_opts=None, adjoint_opts=None):
    """MAP log-density s* (device tensor) on `plan`'s grid, differentiable in
    amp, beta, nbar (0-d tensors or floats), counts and w (tensors of the
    grid's shape).  solve_opts / adjoint_opts: keyword options of Plan.solve
    and Plan.adjoint (rtol, max_newton, max_cg, precision, ...)."""
    solve_opts = dict(rtol=1e-10, max_newton=200, max_cg=5000) if solve_opts is None else dict(solve_opts)
    adjoint_opts = dict(rtol=1e-10, max_cg=20000) if adjoint_opts is None else dict(adjoint_opts)
    return MAPReconstruct.apply(plan, amp, beta, nbar, counts, w, pk, mu, inv_p0, solve_opts, adjoint_opts)
