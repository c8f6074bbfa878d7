"""Octahedral direction map and bilinear texel lookup (Sec. 5.1), FP64.

Readings of points the paper leaves open:
* sign(0) = +1 in the lower-hemisphere unfold (otherwise -z would collide
  with +z at (0,0));
* "rescaled to texel space" is corner-aligned: x = (u+1)/2*(R-1), the
  lower texel index is min(floor(x), R-2) and the fraction x - index, with
  no border wrap; texture columns follow u and rows follow v;
* single-texture form (appearance 0): the colour is the interpolated texel
  itself (identity activation), and the map is indexed by the ray's own unit
  direction.

The paper's full model (appearance 1, Sec. 5.1 and 5.2) gives each cell two
maps of RGB logits, a surface map T_vi indexed by the unit direction d from
the site to the point where the ray meets the cell, and a view map T_vd
indexed by the unit direction from that point towards the camera; the
colour is the logistic sigmoid of their sum.
"""
from __future__ import annotations

import math

import numpy as np


def sign_nz(x: float) -> float:
    return 1.0 if x >= 0.0 else -1.0


def octahedral(d):
    """Unit direction -> (u, v) in [-1,1]^2.

    q = d / (|dx|+|dy|+|dz|); upper hemisphere (dz >= 0): (qx, qy);
    lower: ((1-|qy|) sign qx, (1-|qx|) sign qy).
    """
    dx, dy, dz = (float(c) for c in d)
    s = abs(dx) + abs(dy) + abs(dz)
    qx, qy = dx / s, dy / s
    if dz >= 0.0:
        return qx, qy
    return (1.0 - abs(qy)) * sign_nz(qx), (1.0 - abs(qx)) * sign_nz(qy)


def texel_coords(u: float, v: float, res: int):
    """Corner-aligned texel coordinates: ((col0, fx), (row0, fy))."""
    x = (u + 1.0) * 0.5 * (res - 1)
    y = (v + 1.0) * 0.5 * (res - 1)
    c0 = min(int(math.floor(x)), res - 2)
    r0 = min(int(math.floor(y)), res - 2)
    return (c0, x - c0), (r0, y - r0)


def bilinear_weights(d, res: int):
    """The four (row, col, weight) taps of the lookup for direction d."""
    u, v = octahedral(d)
    (c0, fx), (r0, fy) = texel_coords(u, v, res)
    return [(r0, c0, (1.0 - fx) * (1.0 - fy)),
            (r0, c0 + 1, fx * (1.0 - fy)),
            (r0 + 1, c0, (1.0 - fx) * fy),
            (r0 + 1, c0 + 1, fx * fy)]


def lookup(tex_cell, d):
    """Bilinear RGB colour of one cell's [R,R,4] texture at direction d."""
    t = np.asarray(tex_cell, np.float64)
    res = t.shape[0]
    c = np.zeros(3)
    for r, col, wgt in bilinear_weights(d, res):
        c += wgt * t[r, col, :3]
    return c


def sigmoid(x):
    """Logistic function, evaluated without overflow for either sign."""
    x = np.asarray(x, np.float64)
    e = np.exp(-np.abs(x))
    return np.where(x >= 0.0, 1.0 / (1.0 + e), e / (1.0 + e))


def full_colour(tex_vi, tex_vd, d_surf, d_view):
    """Sec. 5.2: c = sigmoid(T_vi(oct(d_surf)) + T_vd(oct(d_view))) for one cell."""
    return sigmoid(lookup(tex_vi, d_surf) + lookup(tex_vd, d_view))


def octahedral_jacobian(d):
    """d(u, v)/d(d) of the octahedral map at a (not necessarily unit) direction.

    With s = |dx|+|dy|+|dz| and q = d/s: dq_a/dd = (e_a - q_a sgn(d))/s, using
    sgn(0) = +1 like the map itself.  Upper hemisphere: (u, v) = (qx, qy).
    Lower: u = (1-|qy|) sgn qx gives du = -sgn(qx) sgn(qy) dqy, and
    v = (1-|qx|) sgn qy gives dv = -sgn(qx) sgn(qy) dqx.
    """
    d = np.asarray(d, np.float64)
    sg = np.array([sign_nz(c) for c in d])
    s = float(np.abs(d).sum())
    q = d / s
    dqx = (np.array([1.0, 0.0, 0.0]) - q[0] * sg) / s
    dqy = (np.array([0.0, 1.0, 0.0]) - q[1] * sg) / s
    if d[2] >= 0.0:
        return dqx, dqy
    k = -sg[0] * sg[1]
    return k * dqy, k * dqx


def lookup_grad_uv(tex_cell, d):
    """(dc/du, dc/dv) of the bilinear RGB lookup at direction d (fixed taps)."""
    t = np.asarray(tex_cell, np.float64)
    res = t.shape[0]
    u, v = octahedral(d)
    (c0, fx), (r0, fy) = texel_coords(u, v, res)
    t00, t01 = t[r0, c0, :3], t[r0, c0 + 1, :3]
    t10, t11 = t[r0 + 1, c0, :3], t[r0 + 1, c0 + 1, :3]
    k = 0.5 * (res - 1)
    dcu = k * ((1.0 - fy) * (t01 - t00) + fy * (t11 - t10))
    dcv = k * ((1.0 - fx) * (t10 - t00) + fx * (t11 - t01))
    return dcu, dcv
