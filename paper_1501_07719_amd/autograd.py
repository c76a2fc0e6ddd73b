"""torch.autograd.Function over rime_chi2_grad.

The forward pass runs the library's fused chi^2 + adjoint kernels once (the
gradient costs about as much as the visibilities it never stores) and keeps
d chi^2 / d theta; the backward pass scales it by the incoming gradient.
"""
from __future__ import annotations

import torch

from . import rime as _r


class RimeChi2(torch.autograd.Function):
    """chi^2(lm, stokes, alpha, gshape) for a fixed observation and data.

    Inputs are float64 CUDA tensors: lm [nsrc][2], stokes [nsrc][4],
    alpha [nsrc], gshape [ngsrc][3] (the trailing ngsrc sources are
    Gaussians).  Returns a float64 scalar tensor."""

    @staticmethod
    def forward(ctx, lm, stokes, alpha, gshape, plan, data, weight, prec, ws):
        nsrc = lm.shape[0]
        ngsrc = gshape.shape[0]
        sky = _r.DeviceSky(lm=lm.detach().contiguous(), stokes=stokes.detach().contiguous(),
                           alpha=alpha.detach().contiguous(),
                           gshape=gshape.detach().contiguous(), npsrc=nsrc - ngsrc, ngsrc=ngsrc)
        chi2 = torch.empty(1, dtype=torch.float64, device=lm.device)
        grad = torch.empty((nsrc, 10), dtype=torch.float64, device=lm.device)
        if ws is None:
            ws = _r.workspace(plan, _r.MODE_CHI2_GRAD, prec, 1, nsrc, device=lm.device)
        _r.rime_chi2_grad(plan, sky, prec, data, weight, chi2, grad, ws)
        ctx.save_for_backward(grad)
        ctx.ngsrc = ngsrc
        return chi2[0]

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        gg = grad * g
        nsrc = grad.shape[0]
        ng = ctx.ngsrc
        return (gg[:, 0:2], gg[:, 2:6], gg[:, 6], gg[nsrc - ng:, 7:10],
                None, None, None, None, None)


def rime_chi2_autograd(lm, stokes, alpha, gshape, plan, data, weight, prec=_r.MIXED, ws=None):
    """Differentiable chi^2 through the HIP adjoint."""
    return RimeChi2.apply(lm, stokes, alpha, gshape, plan, data, weight, prec, ws)
