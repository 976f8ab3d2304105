"""The imaging operator as a differentiable torch function.

A (degridding, the measurement equation Eq. 1 discretised the w-stacking
way) maps an image x to visibilities A x; its adjoint A^H (gridding, per-
plane FFT, w-screen and plane sum, Eq. 2) maps visibilities back to an
image.  ``ImagingOp`` wraps both HIP paths of a ``WStackPlan``:

  forward(x)    = A x           -> ws_degrid
  backward(g)   = A^H g         -> ws_grid_visibilities + ws_image_accumulate
                  (real part taken when x is real)

With L = ||A x - V||^2 torch passes g = 2 (A x - V), so the gradient is
2 Re(A^H (A x - V)).  Both directions run entirely in the library's
kernels; nothing here computes.
"""
from __future__ import annotations

import torch

from .api import WStackPlan


class ImagingOp(torch.autograd.Function):
    """y = A x for an image x ([nv, nu], real or complex) on a fixed plan,
    baseline set and weights."""

    @staticmethod
    def forward(ctx, x, plan: WStackPlan, uvw, weight=None):
        ctx.plan = plan
        ctx.real = not x.is_complex()
        ctx.save_for_backward(uvw, weight) if weight is not None else \
            ctx.save_for_backward(uvw)
        ctx.has_weight = weight is not None
        return plan.degrid(x.contiguous(), uvw, weight)

    @staticmethod
    def backward(ctx, grad):
        plan = ctx.plan
        if ctx.has_weight:
            uvw, weight = ctx.saved_tensors
        else:
            (uvw,) = ctx.saved_tensors
            weight = None
        gx = plan.dirty_image(uvw, grad.contiguous().to(plan.cdtype), weight)
        if ctx.real:
            gx = gx.real.contiguous()
        return gx, None, None, None


def imaging_op(x, plan: WStackPlan, uvw, weight=None):
    """Differentiable A x (see ``ImagingOp``)."""
    return ImagingOp.apply(x, plan, uvw, weight)
