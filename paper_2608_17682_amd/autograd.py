"""torch.autograd.Function over the HIP renderer.

``render(sites, density, texels, nbr_off, nbr_idx, o, d, tmax, start)``
returns (rgb [R,3], T [R]) and is differentiable with respect to the site
positions, the densities sigma and the texels; rays and adjacency are not.
The forward runs voro_prepare + voro_render_fwd; the backward runs
voro_render_bwd, which replays each ray's walk instead of storing it.
Parameterise sigma = exp(rho) in torch (Sec. 5.4) and autograd supplies
dL/drho = sigma dL/dsigma.
"""
from __future__ import annotations

import torch

from . import voro


class VoroRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sites, density, texels, nbr_off, nbr_idx, o, d, tmax, start, params):
        ds = voro.DeviceScene(sites.detach().contiguous(), density.detach().contiguous(),
                              nbr_off, nbr_idx, texels.detach().contiguous())
        voro.voro_prepare(ds)
        rgb, T = voro.voro_render_fwd(ds, o, d, tmax, start, params)
        ctx.ds = ds
        ctx.params = params
        ctx.tex_dtype = texels.dtype
        ctx.save_for_backward(o, d, tmax, start, rgb, T)
        return rgb, T

    @staticmethod
    def backward(ctx, g_rgb, g_T):
        o, d, tmax, start, rgb, T = ctx.saved_tensors
        ds = ctx.ds
        if g_rgb is None:
            g_rgb = torch.zeros_like(rgb)
        gs, gd, gt = voro.voro_render_bwd(
            ds, o, d, tmax, start, rgb, T, g_rgb.contiguous(),
            None if g_T is None else g_T.contiguous(), ctx.params)
        if ctx.tex_dtype != torch.float32:
            gt = gt.to(ctx.tex_dtype)
        return gs, gd, gt, None, None, None, None, None, None, None


def render(sites, density, texels, nbr_off, nbr_idx, o, d, tmax, start, params=None):
    """Differentiable render of explicit rays; see the module docstring."""
    if params is None:
        params = voro.default_params()
    if params.skip_w != 0.0 and torch.is_grad_enabled() and (
            sites.requires_grad or density.requires_grad or texels.requires_grad):
        raise ValueError("skip_w must be 0 when gradients are needed")
    return VoroRender.apply(sites, density, texels, nbr_off, nbr_idx, o, d, tmax, start, params)
