"""torch.autograd integration of the operator (Sec. 2.2: the forward is differentiable and
its gradient updates every baseline attribute and deformation parameter).

`radiate(pb, balls, deform, frame_t, sensors)` returns the signals [F][S][T] as a
differentiable function of `balls` [5][B] and `deform` [5][M][B]; its backward is one
slingbag_adjoint launch with the incoming gradient as the residual.  Only the base
attributes and coefficients are saved for the backward pass: every frame's deformed
attributes are recomputed inside the adjoint kernel, never stored.
"""

from __future__ import annotations

import torch

from . import ops
from .binding import Problem


class _Radiate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, balls, deform, pb: Problem, frame_t, sensors):
        y = ops.forward(pb, balls.detach(), None if deform is None else deform.detach(), frame_t, sensors)
        ctx.pb = pb
        ctx.has_deform = deform is not None
        if deform is None:
            ctx.save_for_backward(balls, frame_t, sensors)
        else:
            ctx.save_for_backward(balls, deform, frame_t, sensors)
        return y

    @staticmethod
    def backward(ctx, grad_y):
        if ctx.has_deform:
            balls, deform, frame_t, sensors = ctx.saved_tensors
        else:
            balls, frame_t, sensors = ctx.saved_tensors
            deform = None
        gb, gd = ops.adjoint(ctx.pb, balls.detach(), None if deform is None else deform.detach(),
                             frame_t, sensors, grad_y.contiguous())
        return gb, gd, None, None, None


def radiate(pb: Problem, balls, deform, frame_t, sensors):
    """Differentiable signals of the batch (see module docstring)."""
    return _Radiate.apply(balls, deform, pb, frame_t, sensors)


def l2_loss(pb: Problem, signals, measured):
    """1/2 sum (signals - measured)^2 with its gradient; the value comes from slingbag_loss."""
    return _L2.apply(signals, measured, pb)


class _L2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, signals, measured, pb: Problem):
        L, r = ops.loss(pb, signals.detach().contiguous(), measured.detach().contiguous())
        ctx.save_for_backward(r)
        return L

    @staticmethod
    def backward(ctx, grad_L):
        (r,) = ctx.saved_tensors
        return r * grad_L.to(r.dtype), None, None
