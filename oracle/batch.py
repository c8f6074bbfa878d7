"""Batch evaluation of the oracle in its own process (test infrastructure).

    python -m oracle.batch SCENE.npz RAYS.npz OUT.npz [WORKERS]

SCENE.npz holds sites, density, texels (float32 arrays; the adjacency is not
read).  RAYS.npz holds o [R,3], d [R,3], tmax [R] (float32) and optionally
g_rgb [R,3], g_T [R] (upstream gradients), start [R], t_stop, skip_w,
texel_dtype = "float16" (texels rounded to binary16 before use) and
grad_skip_degenerate (sum gradients over the non-degenerate rays only).  Writes rgb [R,3],
T [R], K [R], cells [R,128] (-1 padded), degenerate [R] and stop_degenerate [R]
(oracle.margins), and
with upstream gradients the FP64 gradients restricted to the touched cells:
grad_cells [C], grad_sites [C,3], grad_density [C], grad_texels [C,R,R,4].

Running as a separate process lets a caller that already holds the GPU use
forked workers here without forking itself.
"""
from __future__ import annotations

import sys

import numpy as np

from . import adjoint, margins, render

_G = None


def _init(sites, density, texels, kw):
    global _G
    _G = (sites, density, texels, kw)


def _job(args):
    o, d, tm, st, gr, gt, skip_degenerate = args
    sites, density, texels, kw = _G
    out = []
    for r in range(len(o)):
        rec = render.render_ray(sites, density, texels, o[r], d[r], float(tm[r]),
                                start=None if st is None else int(st[r]), **kw)
        deg = margins.degenerate(rec, kw.get("t_stop", 1e-4), float(tm[r]))
        sdeg = margins.stop_degenerate(rec, kw.get("t_stop", 1e-4))
        grad = None
        if gr is not None and not (skip_degenerate and deg):
            g_sites = _Sparse3()
            g_den = _Sparse1()
            g_tex = _SparseTex(texels.shape[1])
            adjoint.grad_ray(sites, density, texels, o[r], d[r], float(tm[r]), rec, gr[r], gt[r],
                             g_sites, g_den, g_tex)
            grad = (g_sites.d, g_den.d, g_tex.d)
        out.append((rec.rgb, rec.T, rec.K, rec.cells[:128], deg, grad, sdeg))
    return out


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
    """Indexable like g_texels[i, r, c, :3] for the accumulation in grad_ray."""

    def __init__(self, res):
        self.res = res
        self.d = {}

    def __getitem__(self, key):
        i = int(key[0])
        cell = self.d.setdefault(i, np.zeros((self.res, self.res, 4)))
        return cell[key[1:]]

    def __setitem__(self, key, v):
        i = int(key[0])
        cell = self.d.setdefault(i, np.zeros((self.res, self.res, 4)))
        cell[key[1:]] = v


def main(argv):
    import multiprocessing as mp
    import os
    scene_path, rays_path, out_path = argv[:3]
    workers = int(argv[3]) if len(argv) > 3 else min(16, os.cpu_count() or 1)
    z = np.load(scene_path, allow_pickle=False)
    sites, density, texels = z["sites"], z["density"], z["texels"]
    rz = np.load(rays_path, allow_pickle=False)
    if "texel_dtype" in rz and str(rz["texel_dtype"]) == "float16":
        # the GPU stores binary16 texels: evaluate on their exact values
        texels = texels.astype(np.float16).astype(np.float32)
    o, d, tm = rz["o"], rz["d"], rz["tmax"]
    st = rz["start"] if "start" in rz else None
    gr = rz["g_rgb"] if "g_rgb" in rz else None
    gt = rz["g_T"] if "g_T" in rz else (None if gr is None else np.zeros(len(o)))
    skip_deg = bool(rz["grad_skip_degenerate"]) if "grad_skip_degenerate" in rz else False
    kw = {}
    for k in ("t_stop", "skip_w"):
        if k in rz:
            kw[k] = float(rz[k])
    R = len(o)
    chunk = max(1, R // (4 * workers))
    jobs = []
    for s in range(0, R, chunk):
        e = min(R, s + chunk)
        jobs.append((o[s:e], d[s:e], tm[s:e], None if st is None else st[s:e],
                     None if gr is None else gr[s:e], None if gt is None else gt[s:e], skip_deg))
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_init, initargs=(sites, density, texels, kw)) as pool:
        res = [x for part in pool.map(_job, jobs) for x in part]
    out = {"rgb": np.array([x[0] for x in res]), "T": np.array([x[1] for x in res]),
           "K": np.array([x[2] for x in res]), "degenerate": np.array([x[4] for x in res]),
           "stop_degenerate": np.array([x[6] for x in res])}
    cells = np.full((R, 128), -1, np.int64)
    for r, x in enumerate(res):
        cells[r, :len(x[3])] = x[3]
    out["cells"] = cells
    if gr is not None:
        acc_s, acc_d, acc_t = {}, {}, {}
        for x in res:
            if x[5] is None:
                continue
            gs, gd, gtx = x[5]
            for i, v in gs.items():
                acc_s[i] = acc_s.get(i, 0.0) + v
            for i, v in gd.items():
                acc_d[i] = acc_d.get(i, 0.0) + v
            for i, v in gtx.items():
                acc_t[i] = acc_t.get(i, 0.0) + v
        ids = np.array(sorted(set(acc_s) | set(acc_d) | set(acc_t)), np.int64)
        res_ = texels.shape[1]
        out["grad_cells"] = ids
        out["grad_sites"] = np.array([acc_s.get(int(i), np.zeros(3)) for i in ids]).reshape(-1, 3)
        out["grad_density"] = np.array([acc_d.get(int(i), 0.0) for i in ids])
        out["grad_texels"] = np.array([acc_t.get(int(i), np.zeros((res_, res_, 4)))
                                       for i in ids]).reshape(-1, res_, res_, 4)
    np.savez(out_path, **out)


if __name__ == "__main__":
    main(sys.argv[1:])
