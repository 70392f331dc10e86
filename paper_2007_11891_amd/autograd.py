"""torch.autograd.Function around the HDG solve and its adjoint.

Forward: u = U(lambda, f), the recovered element solution of the condensed
HDG system for a per-element lambda field and nodal forcing f (boundary data
fixed: g_D, and g_N on the Neumann sides of a context that has them).  Backward: one adjoint solve with the same symmetric condensed
operator plus the lambda-sensitivity kernel (``hdg_adjoint`` in the C ABI).
Both run in the HIP library; this file only marshals tensors.
"""
from __future__ import annotations

import torch

from .hdg import HdgContext, default_opts


class HdgSolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, lam, f, hdg: HdgContext, dirichlet_trace, opts):
        if lam.dtype != torch.float64 or f.dtype != torch.float64:
            raise TypeError("lambda and f must be float64")
        lam = lam.detach().contiguous()
        f = f.detach().contiguous()
        hdg.set_lambda(lam)
        if dirichlet_trace is None:
            trace = hdg.zeros_trace()
        else:
            trace = dirichlet_trace.detach().clone()
        trace, u, info = hdg.solve_forcing(f, trace, opts=opts)
        ctx.hdg = hdg
        ctx.opts = opts
        ctx.info = info
        ctx.save_for_backward(lam, f, trace)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        lam, f, trace = ctx.saved_tensors
        hdg = ctx.hdg
        hdg.set_lambda(lam)
        dl, df, _ = hdg.adjoint(f, trace, grad_u.detach().contiguous(), opts=ctx.opts)
        return dl, df, None, None, None


def hdg_solve(lam, f, hdg: HdgContext, dirichlet_trace=None, opts=None):
    """Differentiable u(lambda, f); gradients flow to lambda and f.
    ``dirichlet_trace``: a full trace vector whose tail holds the boundary
    data (g_D and the g_N block), or None for zero data."""
    return HdgSolveFn.apply(lam, f, hdg, dirichlet_trace, opts or default_opts())
