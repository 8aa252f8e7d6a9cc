"""Differentiable shooting: torch.autograd.Function over lm_shoot and lm_shoot_adjoint.

The forward pass is lm_shoot; the backward pass is the hand-written discrete adjoint of the
RK4 map (lm_shoot_adjoint, with step checkpointing).  Both run in the HIP library; this
module only routes tensors and gradients.
"""

from __future__ import annotations

import torch

from . import _lib


class ShootFunction(torch.autograd.Function):
    """(q1, p1) = shoot(q0, p0) over [0, t1] with `steps` RK4 steps.

    The backward pass (the discrete adjoint) exists for double precision and every pair
    (params.dtype == F64, params.cutoff == 0): when an input requires a gradient under other
    settings, forward raises before any GPU work rather than after the shoot."""

    @staticmethod
    def forward(ctx, q0, p0, params, t1: float, steps: int, ckpt_every: int = 10):
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            if params.dtype != _lib.F64 or params.cutoff > 0.0:
                raise _lib.LmError(_lib.LM_EUNSUPPORTED,
                                   "the shooting adjoint needs dtype F64 and cutoff 0 (got dtype %d, cutoff %g)"
                                   % (params.dtype, params.cutoff))
        q0 = q0.contiguous()
        p0 = p0.contiguous()
        q1 = torch.empty_like(q0)
        p1 = torch.empty_like(p0)
        _lib.lm_shoot(params, q0, p0, t1, steps, q1, p1)
        ctx.save_for_backward(q0, p0)
        ctx.params, ctx.t1, ctx.steps, ctx.ckpt = params, t1, steps, ckpt_every
        return q1, p1

    @staticmethod
    def backward(ctx, gq1, gp1):
        q0, p0 = ctx.saved_tensors
        gq1 = torch.zeros_like(q0) if gq1 is None else gq1.contiguous()
        gp1 = torch.zeros_like(p0) if gp1 is None else gp1.contiguous()
        gq0 = torch.empty_like(q0)
        gp0 = torch.empty_like(p0)
        _lib.lm_shoot_adjoint(ctx.params, q0, p0, ctx.t1, ctx.steps, ctx.ckpt, gq1, gp1, gq0, gp0)
        return gq0, gp0, None, None, None, None


def shoot(q0, p0, params, t1: float = 1.0, steps: int = 100, ckpt_every: int = 10):
    return ShootFunction.apply(q0, p0, params, t1, steps, ckpt_every)
