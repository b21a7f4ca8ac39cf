"""torch.autograd.Function wrappers over the field and compositing kernels.

The adjoint of the field is the recompute kernel (nsl_field_bwd): it stores
no activations, re-deriving each sample's encoding and network activations
from its position.  The adjoint of compositing (nsl_composite_bwd) recomputes
transmittance and the per-ray prefix sums from sigma, colour and t.  Loss
functions written in torch on the rendered outputs therefore differentiate
down to the field parameters through the same kernels as nsl_train_step.

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


def mapping_loss(out, scale, rgb_target, depth_target_z, depth_var_z, lambda_d=1.0):
    """L_M = L_rgb + lambda_D L_D (Eq. 3, 4, 7) in torch, mean over rays.

    out: [R,6] ray units; scale: |d~| per ray; depth targets in z units.
    Unusable measurements (non-finite, non-positive variance) get weight 0.
    """
    ok = torch.isfinite(depth_target_z) & torch.isfinite(depth_var_z) & (depth_var_z > 0)
    prec = torch.where(ok, 1.0 / (torch.where(ok, depth_var_z, torch.ones_like(depth_var_z)) * scale * scale),
                       torch.zeros_like(scale))
    d_ray = torch.where(ok, depth_target_z * scale, torch.zeros_like(scale))
    l_rgb = ((out[:, :3] - rgb_target) ** 2).sum(-1).mean()
    l_d = (prec * (out[:, 3] - d_ray) ** 2).mean()
    return l_rgb + lambda_d * l_d, l_rgb, l_d
