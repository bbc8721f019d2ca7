"""torch.autograd binding of the forward model and its adjoint.

``SimulateFn.apply(x, y, z, p0, a, array, model, ball_off, ctx)`` runs
sbp_simulate_signals; its backward runs sbp_adjoint_gradients with the
incoming gradient as the cotangent v (only for the parameters that need a
gradient).  FP32 tensors use the FP32 kernels, FP64 tensors the FP64 twins
(the latter exist so that torch.autograd.gradcheck can be run on the GPU path).
"""
from __future__ import annotations

import torch

from . import api

_NAMES = ("x", "y", "z", "p0", "a")


class SimulateFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, z, p0, a, array, model, ball_off=None, sbp_ctx=None):
        dtype = x.dtype
        if dtype not in (torch.float32, torch.float64):
            raise TypeError("SimulateFn needs float32 or float64 ball tensors")
        balls = {k: t.contiguous() for k, t in zip(_NAMES, (x, y, z, p0, a))}
        arr = {k: v.to(dtype).contiguous() for k, v in array.items()}
        c = sbp_ctx if sbp_ctx is not None else api.context(x.device.index or 0)
        out = api.simulate_signals(c, arr, balls, model, ball_off=ball_off, dtype=dtype)
        ctx.save_for_backward(*balls.values())
        ctx.arr, ctx.model, ctx.ball_off, ctx.sbp = arr, model, ball_off, c
        return out

    @staticmethod
    def backward(ctx, grad_y):
        saved = ctx.saved_tensors
        mask = 0
        for i in range(5):
            if ctx.needs_input_grad[i]:
                mask |= 1 << i
        if mask == 0:
            return (None,) * 9
        balls = dict(zip(_NAMES, saved))
        dtype = saved[0].dtype
        g = api.adjoint_gradients(ctx.sbp, ctx.arr, balls, ctx.model, grad_y.contiguous().to(dtype),
                                  mask=mask, ball_off=ctx.ball_off, dtype=dtype)
        return (g["x"], g["y"], g["z"], g["p0"], g["a"], None, None, None, None)


def simulate(x, y, z, p0, a, array, model, ball_off=None, sbp_ctx=None):
    """Differentiable simulated signals [F, D, T] of the balls (x, y, z, p0, a)."""
    return SimulateFn.apply(x, y, z, p0, a, array, model, ball_off, sbp_ctx)
