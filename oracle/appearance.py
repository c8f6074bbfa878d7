"""Octahedral direction map and bilinear texel lookup (Sec. 5.1), FP64.

Readings of points the paper leaves open:
* sign(0) = +1 in the lower-hemisphere unfold (otherwise -z would collide
  with +z at (0,0));
* "rescaled to texel space" is corner-aligned: x = (u+1)/2*(R-1), the
  lower texel index is min(floor(x), R-2) and the fraction x - index, with
  no border wrap; texture columns follow u and rows follow v;
* the colour is the interpolated texel itself (identity activation), and the
  map is indexed by the ray's own unit direction.
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
