"""torch.autograd.Function wrappers over the field and compositing kernels.

The adjoint of the field is the recompute kernel (nsl_field_bwd): it stores
no activations, re-deriving each sample's encoding and network activations
from its position.  The adjoint of compositing (nsl_composite_bwd) recomputes
transmittance and the per-ray prefix sums from sigma, colour and t.  The
mapping loss (nsl_loss_fwd / nsl_loss_bwd) forms the same per-ray terms and
seeds as the step's compositing kernel, so the loss differentiates down to
the field parameters through the step's own arithmetic; other losses
written in torch on the rendered outputs differentiate through the same
field and compositing kernels.

Positions and directions are inputs (the poses are fixed at this boundary),
so no gradient flows to them.
"""
from __future__ import annotations

import torch

from . import nsl


class FieldFunction(torch.autograd.Function):
    """(params, xn [S,3], dirs [S,3]) -> (sigma [S], rgb [S,3])."""

    @staticmethod
    def forward(ctx, params, xn, dirs, field, workspace):
        if xn.requires_grad or dirs.requires_grad:
            raise ValueError("no gradient with respect to sample positions or directions")
        sigma, rgb = field.fwd(params.detach(), xn, dirs, workspace)
        ctx.save_for_backward(params, xn, dirs)
        ctx.field, ctx.ws = field, workspace
        return sigma, rgb

    @staticmethod
    def backward(ctx, g_sigma, g_rgb):
        params, xn, dirs = ctx.saved_tensors
        grads = torch.zeros_like(params)
        g_sigma = torch.zeros(xn.shape[0], device=xn.device) if g_sigma is None else g_sigma.contiguous()
        g_rgb = torch.zeros(xn.shape[0], 3, device=xn.device) if g_rgb is None else g_rgb.contiguous()
        ctx.field.bwd(params.detach(), xn, dirs, g_sigma, g_rgb, grads, ctx.ws)
        return grads, None, None, None, None


class CompositeFunction(torch.autograd.Function):
    """(sigma [S], rgb [S,3], t [S], ray_off [R+1]) -> out [R,6] =
    (r, g, b, d*, V*, A) in ray units (Eq. 5, 6)."""

    @staticmethod
    def forward(ctx, sigma, rgb, t, ray_off, delta):
        out = nsl.composite_fwd(sigma.detach().contiguous(), rgb.detach().contiguous(), t, ray_off, delta)
        ctx.save_for_backward(sigma, rgb, t, ray_off)
        ctx.delta = delta
        return out

    @staticmethod
    def backward(ctx, g_out):
        sigma, rgb, t, ray_off = ctx.saved_tensors
        g = g_out.contiguous()
        g_sigma, g_rgb = nsl.composite_bwd(sigma.detach().contiguous(), rgb.detach().contiguous(), t, ray_off,
                                           ctx.delta, g[:, 0:3].contiguous(), g[:, 3].contiguous(),
                                           g[:, 4].contiguous(), g[:, 5].contiguous())
        return g_sigma, g_rgb, None, None, None


def render_samples(field, params, xn, dirs, t, ray_off, delta, workspace):
    """Differentiable rendering of rays whose samples are contiguous."""
    sigma, rgb = FieldFunction.apply(params, xn, dirs, field, workspace)
    return CompositeFunction.apply(sigma, rgb, t, ray_off, delta)


class LossFunction(torch.autograd.Function):
    """(out [R,6] ray units, targets) -> (L, L_rgb, L_D) (Eq. 3, 4, 7)."""

    @staticmethod
    def forward(ctx, out, scale, rgb_target, depth_target_z, depth_var_z, lambda_d):
        args = (scale.contiguous(), rgb_target.contiguous(), depth_target_z.contiguous(), depth_var_z.contiguous())
        loss = nsl.loss_fwd(out.detach().contiguous(), args[1], args[2], args[3], args[0], lambda_d)
        ctx.save_for_backward(out, *args)
        ctx.lambda_d = lambda_d
        return loss

    @staticmethod
    def backward(ctx, g_loss):
        out, scale, rgb_target, depth_z, depth_var = ctx.saved_tensors
        g = nsl.loss_bwd(out.detach().contiguous(), rgb_target, depth_z, depth_var, scale, ctx.lambda_d,
                         g_loss.contiguous())
        return g, None, None, None, None, None


def mapping_loss(out, scale, rgb_target, depth_target_z, depth_var_z, lambda_d=1.0):
    """L_M = L_rgb + lambda_D L_D (Eq. 3, 4, 7), mean over rays, computed by
    the library (nsl_loss_fwd; its adjoint nsl_loss_bwd).

    out: [R,6] ray units; scale: |d~| per ray; depth targets in z units.
    Unusable measurements (non-finite, non-positive variance) get weight 0.
    Returns (L, L_rgb, L_D) as 0-d tensors.
    """
    loss = LossFunction.apply(out, scale, rgb_target, depth_target_z, depth_var_z, lambda_d)
    return loss[0], loss[1], loss[2]
