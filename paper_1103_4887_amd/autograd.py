"""The action A(X, p) as a differentiable torch function.

Forward is the library's FP64 action reduction (the path action of
Section 2.1: measurement term plus model-error term over the discretised
map); backward is its hand-written adjoint, the local stencil of dA/dx_n
and the FP64 sums of dA/dp_l.  Both run in the library's kernels; this
module only routes tensors.
"""

from __future__ import annotations

import torch

from .api import Context, Window, pimc_action, pimc_grad

_PREC = {torch.float32: "fp32", torch.float64: "fp64"}


class PimcAction(torch.autograd.Function):
    """A = PimcAction.apply(X, p, y, I, ctx, spec) -> 0-d FP64 tensor.

    X [M+1][4] (FP32 or FP64), p [7] FP64, y and I [M+1] in X's precision,
    all on the context's device.  y and I receive no gradient.
    """

    @staticmethod
    def forward(fctx, X, p, y, I, ctx: Context, spec):
        if X.dtype not in _PREC:
            raise TypeError("X must be float32 or float64")
        win = Window(X=X.detach().contiguous(), p=p.detach().contiguous(), y=y.contiguous(), I=I.contiguous(),
                     prec=_PREC[X.dtype])
        out = pimc_action(ctx, spec, win)
        fctx.save_for_backward(win.X, win.p, win.y, win.I)
        fctx.pimc = (ctx, spec)
        return out[0].clone()

    @staticmethod
    def backward(fctx, g):
        X, p, y, I = fctx.saved_tensors
        ctx, spec = fctx.pimc
        win = Window(X=X, p=p, y=y, I=I, prec=_PREC[X.dtype])
        gX, gp = pimc_grad(ctx, spec, win)
        gX = gX * g.to(gX.dtype) if fctx.needs_input_grad[0] else None
        gp = gp * g if fctx.needs_input_grad[1] else None
        return gX, gp, None, None, None, None


def action(ctx: Context, spec, X: torch.Tensor, p: torch.Tensor, y: torch.Tensor, I: torch.Tensor) -> torch.Tensor:
    """Differentiable A(X, p) (see PimcAction)."""
    return PimcAction.apply(X, p, y, I, ctx, spec)
