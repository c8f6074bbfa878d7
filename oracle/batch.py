"""Many-ray evaluation of the oracle over a process pool (test infrastructure).

``evaluate`` renders rays one by one with ``render.render_ray`` in forked
worker processes and returns, per ray, what the parity tests compare: colour,
transmittance, the number of visited cells, the visited-cell sequence and the
degeneracy flags of ``margins``; ``sparse_gradients`` sums the FP64 adjoint
(``adjoint.grad_ray``) of chosen rays into per-cell gradients of the cells
they touch.  Nothing here adds arithmetic of its own: the results are those
of ``render_rays`` / ``grad_rays``, in the same order, computed in parallel.

Workers are forked, so a caller that already holds a GPU must not call this
(run it from a process that has not initialised one).
"""
from __future__ import annotations

import os

import numpy as np

from . import adjoint, margins, render, walk

_G = None


def _init(sites, density, texels, kw):
    global _G
    _G = (sites, density, texels, kw)


def _job(args):
    lo, o, d, tm, st, keep = args
    sites, density, texels, kw = _G
    t_stop = kw.get("t_stop", 1e-4)
    out = []
    for r in range(len(o)):
        if tm[r] <= 0.0:
            out.append((np.zeros(3), 1.0, 0, np.zeros(0, np.int64), False, False, None))
            continue
        rec = render.render_ray(sites, density, texels, o[r], d[r], float(tm[r]),
                                start=None if st is None else int(st[r]), **kw)
        deg = margins.degenerate(rec, t_stop, float(tm[r]))
        sdeg = margins.stop_degenerate(rec, t_stop)
        out.append((rec.rgb, rec.T, rec.K, np.asarray(rec.cells, np.int64), deg, sdeg,
                    rec if keep[r] else None))
    return lo, out


def evaluate(sites, density, texels, o, d, tmax, starts=None, keep_records=None,
             workers=None, chunk=None, **kw):
    """Oracle results of R rays (FP64), in ray order.

    Returns a dict: rgb [R,3], T [R], K [R], cells (list of R int64 arrays),
    degenerate [R], stop_degenerate [R] and records (list: the RayRecord of
    each ray with keep_records[r] set, else None).  Rays with tmax <= 0 are
    empty (rgb 0, T 1, K 0).  ``kw`` goes to ``render.render_ray``.
    """
    import multiprocessing as mp
    sites = walk.as64(sites)
    density = walk.as64(density)
    R = len(o)
    tm = np.broadcast_to(np.asarray(tmax, np.float64), (R,))
    keep = np.zeros(R, bool) if keep_records is None else np.asarray(keep_records, bool)
    workers = workers or min(16, os.cpu_count() or 1)
    chunk = chunk or max(1, R // (4 * workers))
    jobs = [(s, o[s:s + chunk], d[s:s + chunk], tm[s:s + chunk],
             None if starts is None else starts[s:s + chunk], keep[s:s + chunk])
            for s in range(0, R, chunk)]
    if workers <= 1:
        _init(sites, density, texels, kw)
        parts = [_job(j) for j in jobs]
    else:
        ctx = mp.get_context("fork")
        with ctx.Pool(workers, initializer=_init, initargs=(sites, density, texels, kw)) as pool:
            parts = pool.map(_job, jobs, chunksize=1)
    res = [x for _, part in sorted(parts, key=lambda p: p[0]) for x in part]
    return {"rgb": np.array([x[0] for x in res]).reshape(R, 3),
            "T": np.array([x[1] for x in res], np.float64),
            "K": np.array([x[2] for x in res], np.int64),
            "cells": [x[3] for x in res],
            "degenerate": np.array([x[4] for x in res], bool),
            "stop_degenerate": np.array([x[5] for x in res], bool),
            "records": [x[6] for x in res]}


class _Sparse3:
    def __init__(self):
        self.d = {}

    def __getitem__(self, i):
        return self.d.setdefault(int(i), np.zeros(3))

    def __setitem__(self, i, v):
        self.d[int(i)] = np.asarray(v, np.float64)


class _Sparse1:
    def __init__(self):
        self.d = {}

    def __getitem__(self, i):
        return self.d.get(int(i), 0.0)

    def __setitem__(self, i, v):
        self.d[int(i)] = float(v)


class _SparseTex:
    """Indexable like g_texels[i, ...] for the accumulation in grad_ray; each
    touched cell holds a dense block shaped like one cell's texels ([R,R,4],
    or [2,R,R,4] for the two maps of the full appearance model)."""

    def __init__(self, cell_shape):
        self.cell_shape = tuple(cell_shape)
        self.d = {}

    def _cell(self, i):
        return self.d.setdefault(int(i), np.zeros(self.cell_shape))

    def __getitem__(self, key):
        return self._cell(key[0])[key[1:]]

    def __setitem__(self, key, v):
        self._cell(key[0])[key[1:]] = v


def sparse_gradients(sites, density, texels, o, d, tmax, records, g_rgb, g_T=None):
    """FP64 gradients of L = sum_r g_rgb[r].rgb[r] + g_T[r] T[r] over the rays
    whose record is given (records[r] None = ray left out), restricted to the
    cells they touch.  Texels [N,R,R,4] (single map) or [N,2,R,R,4] (the full
    appearance model; the records say which model rendered them).

    Returns (cells [C] sorted, g_sites [C,3], g_density [C], g_texels [C, ...]
    with one cell's texel shape); every cell not listed has zero gradient.
    """
    sites = walk.as64(sites)
    density = walk.as64(density)
    cell_shape = tuple(np.shape(texels)[1:])
    gs, gd, gt = _Sparse3(), _Sparse1(), _SparseTex(cell_shape)
    R = len(records)
    tm = np.broadcast_to(np.asarray(tmax, np.float64), (R,))
    for r, rec in enumerate(records):
        if rec is None:
            continue
        adjoint.grad_ray(sites, density, texels, o[r], d[r], float(tm[r]), rec, g_rgb[r],
                         0.0 if g_T is None else g_T[r], gs, gd, gt)
    ids = np.array(sorted(set(gs.d) | set(gd.d) | set(gt.d)), np.int64)
    return (ids,
            np.array([gs.d.get(int(i), np.zeros(3)) for i in ids]).reshape(-1, 3),
            np.array([gd.d.get(int(i), 0.0) for i in ids]),
            np.array([gt.d.get(int(i), np.zeros(cell_shape)) for i in ids]).reshape(
                (-1,) + cell_shape))
