"""Voronoi partition and per-ray cell intervals by brute force (FP64).

Follows Sec. 3.1: a cell V_i holds every point at least as close to p_i as
to any other site; the ray r(t) = o + t*w is advanced from the cell holding
the origin across the *nearest forward crossing* of the bisector planes
(Fig. "Adjacency-based ray traversal").

Conventions (readings of points the paper leaves open):
* exact ties in distance or in exit parameter go to the smaller site index;
* a cell with no forward bisector (unbounded hull cell) exits at +inf;
* the walk here tests *all* sites, never the Delaunay adjacency: since
  V_i is the intersection of the half-spaces H_ij over all j, only
  face-sharing neighbours can attain the minimum, so this equals the
  adjacency walk.
"""
from __future__ import annotations

import numpy as np


def as64(a):
    return np.asarray(a, dtype=np.float64)


def nearest_site(sites, x):
    """Index of the cell containing point x: argmin_i |x - p_i|^2, ties -> smallest i.

    Returns (index, gap) with gap = second-smallest minus smallest squared distance.
    """
    p = as64(sites)
    x = as64(x)
    d2 = np.sum((p - x) ** 2, axis=1)
    i = int(np.argmin(d2))          # first occurrence == smallest index
    if d2.shape[0] > 1:
        part = np.partition(d2, 1)
        gap = float(part[1] - part[0])
    else:
        gap = np.inf
    return i, gap


def exit_crossing(sites, i, o, w):
    """Nearest forward bisector crossing out of cell i along o + t*w.

    For every j != i: n = p_j - p_i, b = n.w; if b > 0 the ray crosses the
    bisector plane through m = (p_i + p_j)/2 at t_j = n.(m - o) / b.
    Returns (t_exit, j_next, gap) where gap = second-best minus best t
    (inf when fewer than two forward faces).  No forward face -> (inf, -1, inf).
    """
    p = as64(sites)
    o = as64(o)
    w = as64(w)
    pi = p[i]
    n = p - pi
    b = n @ w
    m = 0.5 * (p + pi)
    a = np.sum(n * (m - o), axis=1)
    fwd = b > 0.0
    fwd[i] = False
    if not np.any(fwd):
        return np.inf, -1, np.inf
    t = np.full(p.shape[0], np.inf)
    t[fwd] = a[fwd] / b[fwd]
    j = int(np.argmin(t))           # first occurrence == smallest index on exact ties
    if np.count_nonzero(fwd) > 1:
        part = np.partition(t[fwd], 1)
        gap = float(part[1] - part[0])
    else:
        gap = np.inf
    return float(t[j]), j, gap


class RayBisectors:
    """exit_crossing for one fixed ray, with the ray's dot products taken once.

    The bisector of p_i and p_j is the plane of points x with
    (p_j - p_i).x = (|p_j|^2 - |p_i|^2)/2 (equal distance to both sites,
    Sec. 3.1).  On the ray x = o + t w it is crossed where
        t = (h_j - h_i) / (s_j - s_i),   s = p.w,   h = |p|^2/2 - p.o,
    which is exit_crossing's n.(m - o)/(n.w) written out: n.w = s_j - s_i and
    n.(m - o) = (|p_j|^2 - |p_i|^2)/2 - n.o = h_j - h_i.  s and h are per-site
    numbers of this ray, so each step costs a few passes over N scalars
    instead of over N vectors.  Same candidates (every j != i with
    n.w > 0), same arg-min (first occurrence = smallest index), same gap.
    """

    def __init__(self, sites, o, w):
        p = as64(sites)
        self.o = as64(o)
        self.w = as64(w)
        self.s = p @ self.w
        self.h = 0.5 * np.einsum("ij,ij->i", p, p) - p @ self.o
        n = p.shape[0]
        self._b = np.empty(n)
        self._a = np.empty(n)
        self._t = np.empty(n)
        self._fwd = np.empty(n, bool)

    def exit(self, i):
        """(t_exit, j_next, gap) out of cell i, as exit_crossing returns them."""
        b, a, t, fwd = self._b, self._a, self._t, self._fwd
        np.subtract(self.s, self.s[i], out=b)
        np.greater(b, 0.0, out=fwd)
        fwd[i] = False
        nf = int(np.count_nonzero(fwd))
        if nf == 0:
            return np.inf, -1, np.inf
        np.subtract(self.h, self.h[i], out=a)
        t.fill(np.inf)
        np.divide(a, b, out=t, where=fwd)
        j = int(np.argmin(t))           # first occurrence == smallest index on exact ties
        tj = float(t[j])
        if nf > 1:
            t[j] = np.inf
            gap = float(np.min(t)) - tj
        else:
            gap = np.inf
        return tj, j, gap


def walk_stepwise(sites, o, w, tmax, start=None):
    """Generator over the ray's cells by repeated nearest forward crossing.

    Yields (cell, exit_t, next_cell, gap) for each cell in order; the caller
    decides when to stop (early termination lives in the compositing).
    The walk itself ends after the cell whose exit is at or beyond tmax.
    """
    if start is None:
        start, _ = nearest_site(sites, o)
    i = int(start)
    ray = RayBisectors(sites, o, w)
    while True:
        t_exit, j, gap = ray.exit(i)
        yield i, t_exit, j, gap
        if not (t_exit < tmax) or j < 0:
            return
        i = j


def cell_intervals(sites, o, w, tmax):
    """All non-empty intervals [a_i, b_i] of the segment t in [0, tmax] per cell.

    Independent of the stepwise walk: cell i's constraints over every j != i,
    (p_j - p_i).(o + t w) <= (|p_j|^2 - |p_i|^2)/2, cut the line in one
    interval (a line meets a convex set in an interval).  Returns the cells
    with positive-length intervals sorted by entry: (cells, starts, ends).
    O(N^2) per ray - for tiny scenes only.
    """
    p = as64(sites)
    o = as64(o)
    w = as64(w)
    nrm = np.sum(p * p, axis=1)
    N = p.shape[0]
    cells, starts, ends = [], [], []
    for i in range(N):
        n = p - p[i]
        b = n @ w
        rhs = 0.5 * (nrm - nrm[i]) - n @ o
        mask = np.ones(N, bool)
        mask[i] = False
        lo, hi = 0.0, float(tmax)
        pos = mask & (b > 0)
        neg = mask & (b < 0)
        zer = mask & (b == 0)
        if np.any(zer & (rhs < 0)):
            continue
        if np.any(pos):
            hi = min(hi, float(np.min(rhs[pos] / b[pos])))
        if np.any(neg):
            lo = max(lo, float(np.max(rhs[neg] / b[neg])))
        if hi > lo:
            cells.append(i)
            starts.append(lo)
            ends.append(hi)
    order = np.argsort(starts, kind="stable")
    return (np.asarray(cells, np.int64)[order], np.asarray(starts)[order],
            np.asarray(ends)[order])


def csr_contains(nbr_off, nbr_idx, i, j):
    """True when j is listed in row i of the adjacency (validation only)."""
    row = nbr_idx[int(nbr_off[i]):int(nbr_off[i + 1])]
    return bool(np.any(row == j))
