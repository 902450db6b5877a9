"""torch.autograd.Function around the Wilson-Clover solve x = D(U, kappa)^-1 b.

Forward: wcl_solve.  Backward (upstream gradient g = dL/dx in PyTorch's
complex convention): the adjoint solve y = D^-dag g = g5 D^-1 g5 g
(wcl_solve with adjoint=1), then wcl_grad for the link and kappa gradients;
grad_b = y.  All arithmetic runs in the HIP library.
"""
from __future__ import annotations

import torch

from . import wcl


class WilsonCloverSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, kappa, b, lat, csw, opts):
        kap = float(kappa)
        lat.set_gauge(U)
        lat.set_params(kap, csw)
        x, info, rc = lat.solve(b, **opts)
        ctx.save_for_backward(U, x)
        ctx.lat, ctx.kappa, ctx.csw, ctx.opts = lat, kap, csw, dict(opts)
        ctx.kappa_is_tensor = isinstance(kappa, torch.Tensor)
        return x

    @staticmethod
    def backward(ctx, g):
        U, x = ctx.saved_tensors
        lat = ctx.lat
        # the context may have been reused for another field since the forward
        lat.set_gauge(U)
        lat.set_params(ctx.kappa, ctx.csw)
        y, info, rc = lat.solve(g.contiguous(), adjoint=1, **ctx.opts)
        gU, gk = lat.grad(x, y)
        gkappa = torch.tensor(gk, dtype=torch.float64) if ctx.kappa_is_tensor else None
        return gU, gkappa, y, None, None, None


def solve(U, kappa, b, lat, csw=1.0, **opts):
    """x = D(U, kappa)^-1 b, differentiable in U, kappa and b."""
    return WilsonCloverSolve.apply(U, kappa, b, lat, csw, opts)
