"""Piecewise-constant volume rendering along one ray (Sec. 3.2), FP64.

For the ordered segments k of the ray (one per visited cell i_k):

    delta_k = max(min(exit_k, tmax) - t_k, 0)          segment length
    alpha_k = 1 - exp(-sigma_{i_k} delta_k)             opacity (Sec. 3.2)
    w_k     = T_k alpha_k,  T_{k+1} = T_k (1 - alpha_k) compositing weight / transmittance
    C       = sum_k w_k c_k                             front-to-back colour

with c_k the octahedral bilinear colour of cell i_k at the ray direction
(Sec. 5.1; appearance 0), or, for the paper's full model (appearance 1,
Sec. 5.2), c_k = sigmoid(T_vi(oct(d_k)) + T_vd(oct(-w))) with texels laid
out [N, 2, R, R, 4] (map 0 = T_vi, map 1 = T_vd), d_k the unit direction from
the site to the hit point x_k and -w the direction from x_k back towards
the ray's origin.  Readings of what the paper leaves open:
* appearance 2 is the spherical-harmonic colour of Sec. 3.3 at the ray
  direction (``sh``; coefficients [N, 48]), the comparison model;
* the hit point is where the ray enters the cell, x_k = o + t_k w; in the
  start cell, which holds the origin, it is where the ray leaves it,
  o + min(exit_0, tmax) w; a hit point on the site itself (d undefined)
  uses d = w;
* early termination is tested strictly, T_{k+1} < t_stop, after segment k
  has been fully composited; the walk also ends at the first exit at or
  beyond tmax, and after max_steps segments (flagged);
* the low-contribution skip of Sec. 5.6 drops the colour of a segment whose
  weight is below skip_w (transmittance is still updated); skip_w = 0
  composites every segment;
* rays cover t in [0, tmax] with no near plane and no background colour
  (the returned colour is premultiplied).
The record also carries the ray's distortion loss (Sec. 5.3) over the
segments [t_k, t_k + delta_k] with their weights w_k.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from . import appearance as appearance_mod, distortion, sh, walk


@dataclasses.dataclass
class RayRecord:
    rgb: np.ndarray
    T: float
    cells: List[int]
    t_in: List[float]
    exit: List[float]        # exit parameter of each cell (may exceed tmax, or inf)
    nxt: List[int]           # the cell entered at that exit (-1: none)
    delta: List[float]
    alpha: List[float]
    T_before: List[float]
    weight: List[float]
    color: List[np.ndarray]
    skipped: List[bool]
    gaps: List[float]        # FP64 gap between best and second-best exit, per step
    stop: str                # "tstop" | "tmax" | "max_steps"
    start_gap: float = math.inf
    appearance: int = 0
    dist: float = 0.0        # distortion loss of the ray (Sec. 5.3)
    t_hit: List[float] = dataclasses.field(default_factory=list)    # appearance 1
    surf_dir: List[np.ndarray] = dataclasses.field(default_factory=list)

    @property
    def K(self) -> int:
        return len(self.cells)


def render_ray(sites, density, texels, o, w, tmax, t_stop=1e-4, skip_w=0.0,
               max_steps=4096, start=None, method="stepwise", appearance=0) -> RayRecord:
    """Render one ray by brute force.  method: 'stepwise' or 'interval'."""
    appearance_model = int(appearance)
    if appearance_model not in (0, 1, 2):
        raise ValueError(f"appearance {appearance}")
    sites = walk.as64(sites)
    sig = walk.as64(density)
    tex = np.asarray(texels)
    if appearance_model == 1 and (tex.ndim != 5 or tex.shape[1] != 2):
        raise ValueError("appearance 1 needs texels [N, 2, R, R, 4]")
    if appearance_model == 2 and (tex.ndim != 2 or tex.shape[1] != 48):
        raise ValueError("appearance 2 needs SH coefficients [N, 48]")
    o = walk.as64(o)
    w = walk.as64(w)
    tmax = float(tmax)
    start_gap = math.inf
    if start is None:
        start, start_gap = walk.nearest_site(sites, o)

    if method == "stepwise":
        steps = walk.walk_stepwise(sites, o, w, tmax, start)
    elif method == "interval":
        cells, a, b = walk.cell_intervals(sites, o, w, tmax)

        def _gen():
            for k in range(len(cells)):
                nxt = int(cells[k + 1]) if k + 1 < len(cells) else -1
                ex = float(b[k]) if k + 1 < len(cells) else math.inf
                yield int(cells[k]), ex, nxt, math.inf
        steps = _gen()
    else:
        raise ValueError(method)

    C = np.zeros(3)
    T = 1.0
    t = 0.0
    rec = RayRecord(C, T, [], [], [], [], [], [], [], [], [], [], [], "tmax", start_gap,
                    appearance)
    for k, (i, ex, j, gap) in enumerate(steps):
        t_out = min(ex, tmax)
        delta = max(t_out - t, 0.0)
        tau = sig[i] * delta
        alpha = -math.expm1(-tau)
        wk = T * alpha
        skipped = skip_w > 0.0 and wk < skip_w
        if appearance_model == 1:
            t_hit = t if k > 0 else t_out
            rel = o + t_hit * w - sites[i]
            r = float(np.linalg.norm(rel))
            d_surf = rel / r if r > 0.0 else w.copy()
            rec.t_hit.append(t_hit)
            rec.surf_dir.append(d_surf)
        if skipped:
            c = np.zeros(3)
        else:
            if appearance_model == 1:
                c = appearance_mod.full_colour(tex[i, 0], tex[i, 1], d_surf, -w)
            elif appearance_model == 2:
                c = sh.sh_colour(tex[i], w)
            else:
                c = appearance_mod.lookup(tex[i], w)
            C = C + wk * c
        T_next = T * math.exp(-tau)
        rec.cells.append(i)
        rec.t_in.append(t)
        rec.exit.append(ex)
        rec.nxt.append(j)
        rec.delta.append(delta)
        rec.alpha.append(alpha)
        rec.T_before.append(T)
        rec.weight.append(wk)
        rec.color.append(c)
        rec.skipped.append(skipped)
        rec.gaps.append(gap)
        T = T_next
        t = t + delta
        if T < t_stop:
            rec.stop = "tstop"
            break
        if not (ex < tmax) or j < 0:
            rec.stop = "tmax"
            break
        if k + 1 >= max_steps:
            rec.stop = "max_steps"
            break
    rec.rgb = C
    rec.T = T
    rec.dist = distortion.distortion(rec.weight, rec.t_in,
                                     [a + b for a, b in zip(rec.t_in, rec.delta)])
    return rec


def render_rays(sites, density, texels, origins, dirs, tmax, starts=None, **kw):
    """Render many rays one by one.  Returns (rgb[R,3], T[R], records)."""
    R = len(origins)
    rgb = np.zeros((R, 3))
    T = np.ones(R)
    recs = []
    tm = np.broadcast_to(np.asarray(tmax, np.float64), (R,))
    for r in range(R):
        st = None if starts is None else int(starts[r])
        if tm[r] <= 0.0:
            recs.append(None)
            continue
        rec = render_ray(sites, density, texels, origins[r], dirs[r], tm[r], start=st, **kw)
        rgb[r] = rec.rgb
        T[r] = rec.T
        recs.append(rec)
    return rgb, T, recs


# ------------------------------------------------------- process-pool helper
_POOL_SCENE = None


def _pool_init(scene_arrays, kw):
    global _POOL_SCENE
    _POOL_SCENE = (scene_arrays, kw)


def _pool_job(args):
    (sites, density, texels), kw = _POOL_SCENE
    o, d, tm, st = args
    return render_rays(sites, density, texels, o, d, tm, st, **kw)


def render_rays_parallel(sites, density, texels, origins, dirs, tmax, starts=None,
                         workers=None, chunk=64, **kw):
    """render_rays over a process pool (fork); same results, one ray at a time."""
    import multiprocessing as mp
    import os
    R = len(origins)
    tm = np.broadcast_to(np.asarray(tmax, np.float64), (R,))
    workers = workers or os.cpu_count() or 1
    jobs = []
    for s in range(0, R, chunk):
        e = min(R, s + chunk)
        jobs.append((origins[s:e], dirs[s:e], tm[s:e], None if starts is None else starts[s:e]))
    if workers <= 1 or len(jobs) == 1:
        return render_rays(sites, density, texels, origins, dirs, tm, starts, **kw)
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_pool_init,
                  initargs=((sites, density, texels), kw)) as pool:
        parts = pool.map(_pool_job, jobs)
    rgb = np.concatenate([p[0] for p in parts])
    T = np.concatenate([p[1] for p in parts])
    recs = [r for p in parts for r in p[2]]
    return rgb, T, recs
