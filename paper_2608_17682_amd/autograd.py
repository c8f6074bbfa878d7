"""torch.autograd.Functions over the HIP renderer.

``render(sites, density, texels, nbr_off, nbr_idx, o, d, tmax, start)``
returns (rgb [R,3], T [R]) for explicit rays (and, with distortion=True,
each ray's distortion loss of Sec. 5.3); ``render_views(sites, density,
texels, nbr_off, nbr_idx, cameras)`` returns per-pixel (rgb [P,3], T [P])
for up to 16 cameras generated in-kernel (one launch each way).  Both are
differentiable with respect to the site positions, the densities sigma and
the texels; rays, cameras and adjacency are not.  The forward runs
voro_prepare + the forward walk; the backward replays each ray's walk,
searching every exit again or, with stored_exits = n > 0, reading the first n
exits of each ray that the forward stored (8 bytes per ray and step, held
until the backward).  Parameterise sigma = exp(rho) in torch (Sec. 5.4)
and autograd supplies dL/drho = sigma dL/dsigma.
"""
from __future__ import annotations

import torch

from . import voro


class VoroRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sites, density, texels, nbr_off, nbr_idx, o, d, tmax, start, params,
                with_dist, stored_exits):
        ds = voro.DeviceScene(sites.detach().contiguous(), density.detach().contiguous(),
                              nbr_off, nbr_idx, texels.detach().contiguous())
        voro.voro_prepare(ds)
        dist = (torch.empty((o.shape[0], 3), dtype=torch.float32, device=o.device)
                if with_dist else None)
        trace = (torch.empty((stored_exits, o.shape[0], 2), dtype=torch.int32, device=o.device)
                 if stored_exits > 0 else None)
        rgb, T = voro.voro_render_fwd(ds, o, d, tmax, start, params, dist=dist, trace=trace)
        ctx.trace = trace
        ctx.ds = ds
        ctx.params = params
        ctx.tex_dtype = texels.dtype
        ctx.with_dist = with_dist
        ctx.save_for_backward(o, d, tmax, start, rgb, T,
                              dist if with_dist else torch.empty(0, device=o.device))
        if with_dist:
            return rgb, T, dist[:, 0]
        return rgb, T

    @staticmethod
    def backward(ctx, g_rgb, g_T, g_dist=None):
        o, d, tmax, start, rgb, T, dist = ctx.saved_tensors
        ds = ctx.ds
        if g_rgb is None:
            g_rgb = torch.zeros_like(rgb)
        if ctx.with_dist and g_dist is not None:
            dist_in, g_dist = dist, g_dist.contiguous()
        else:
            dist_in, g_dist = None, None
        gs, gd, gt = voro.voro_render_bwd(
            ds, o, d, tmax, start, rgb, T, g_rgb.contiguous(),
            None if g_T is None else g_T.contiguous(), ctx.params, dist=dist_in, g_dist=g_dist,
            trace=ctx.trace)
        ctx.trace = None
        if ctx.tex_dtype != torch.float32:
            gt = gt.to(ctx.tex_dtype)
        return gs, gd, gt, None, None, None, None, None, None, None, None, None


class VoroRenderViews(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sites, density, texels, nbr_off, nbr_idx, cams, params_fwd, params_bwd,
                stored_exits):
        ds = voro.DeviceScene(sites.detach().contiguous(), density.detach().contiguous(),
                              nbr_off, nbr_idx, texels.detach().contiguous())
        voro.voro_prepare(ds)
        trace = None
        if stored_exits > 0:
            nr, _ = voro.voro_camera_counts(list(cams))
            trace = torch.empty((stored_exits, nr, 2), dtype=torch.int32, device=sites.device)
        rgb, T, ray_rgbT = voro.voro_render_views_fwd(ds, cams, params_fwd, trace=trace)
        ctx.trace = trace
        ctx.ds = ds
        ctx.cams = cams
        ctx.params = params_bwd
        ctx.tex_dtype = texels.dtype
        ctx.ray_rgbT = ray_rgbT
        ctx.save_for_backward(rgb, T)
        return rgb, T

    @staticmethod
    def backward(ctx, g_rgb, g_T):
        rgb, T = ctx.saved_tensors
        if g_rgb is None:
            g_rgb = torch.zeros_like(rgb)
        gs, gd, gt = voro.voro_render_views_bwd(
            ctx.ds, ctx.cams, rgb, T, ctx.ray_rgbT, g_rgb.contiguous(),
            None if g_T is None else g_T.contiguous(), ctx.params, trace=ctx.trace)
        ctx.trace = None
        if ctx.tex_dtype != torch.float32:
            gt = gt.to(ctx.tex_dtype)
        return gs, gd, gt, None, None, None, None, None, None


# walk parameters: they decide the cell sequence and the colour, so the
# adjoint's replay must use the forward's values
_WALK_FIELDS = ("t_stop", "skip_w", "max_steps", "tie_window", "appearance", "edge_fp16")
# launch shape: results do not depend on it, each direction may use its own
_LAUNCH_FIELDS = ("lanes_per_ray", "tile_w", "tile_h", "block", "schedule")


def _wants_grad(*ts) -> bool:
    return torch.is_grad_enabled() and any(t.requires_grad for t in ts)


def _check_differentiable(params):
    if params.skip_w != 0.0:
        raise ValueError("skip_w must be 0 when gradients are needed")
    if params.edge_fp16 != 0:
        raise ValueError("edge_fp16 is a forward-only inference variant: the adjoint replays "
                         "the exact walk, so gradients need edge_fp16 = 0")


def backward_params(params_fwd, params_bwd=None):
    """The adjoint's parameters: the forward's walk parameters with params_bwd's
    launch shape.  Raises ValueError if params_bwd sets a walk parameter
    (t_stop, skip_w, max_steps, tie_window, appearance, edge_fp16) other than
    the forward's: the replay would visit other cells."""
    q = voro.voro_params.from_buffer_copy(params_fwd)
    if params_bwd is not None:
        for f in _WALK_FIELDS:
            if getattr(params_bwd, f) != getattr(params_fwd, f):
                raise ValueError(f"params_bwd.{f} = {getattr(params_bwd, f)} differs from the "
                                 f"forward's {getattr(params_fwd, f)}; only the launch shape "
                                 f"({', '.join(_LAUNCH_FIELDS)}) may differ")
        for f in _LAUNCH_FIELDS:
            setattr(q, f, getattr(params_bwd, f))
    return q


def render_views(sites, density, texels, nbr_off, nbr_idx, cams, params_fwd=None,
                 params_bwd=None, stored_exits=0):
    """Differentiable render of camera views (voro_camera list or objects with
    the camera attributes); pixels of all views concatenated in order.
    params_bwd supplies only the adjoint's launch shape (see backward_params).
    stored_exits > 0: the forward keeps each ray's first stored_exits exits
    (8 bytes per ray and step, until the backward) and the adjoint reads them
    instead of searching those steps again."""
    cams = voro.camera_array(cams)
    params_fwd = params_fwd or voro.default_params()
    params_bwd = backward_params(params_fwd, params_bwd)
    wants = _wants_grad(sites, density, texels)
    if wants:
        _check_differentiable(params_fwd)
    if stored_exits < 0:
        raise ValueError("stored_exits must be >= 0")
    return VoroRenderViews.apply(sites, density, texels, nbr_off, nbr_idx, cams, params_fwd,
                                 params_bwd, int(stored_exits) if wants else 0)


def render(sites, density, texels, nbr_off, nbr_idx, o, d, tmax, start, params=None,
           distortion=False, stored_exits=0):
    """Differentiable render of explicit rays; see the module docstring.  With
    distortion=True also returns each ray's distortion loss (Sec. 5.3), [R],
    differentiable like the colour.  stored_exits: as for render_views."""
    if params is None:
        params = voro.default_params()
    wants = _wants_grad(sites, density, texels)
    if wants:
        _check_differentiable(params)
    if stored_exits < 0:
        raise ValueError("stored_exits must be >= 0")
    return VoroRender.apply(sites, density, texels, nbr_off, nbr_idx, o, d, tmax, start, params,
                            bool(distortion), int(stored_exits) if wants else 0)
