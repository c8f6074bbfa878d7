"""Seeded synthetic scenes, cameras and upstream gradients.

This module only *draws inputs*: site positions, per-cell densities, texels,
camera descriptions (pose and lens parameters) and upstream gradients.  It
holds none of the rendering arithmetic (no ray generation, no walk, no
compositing), so both the FP64 oracle and the HIP path can be fed from it.

The Delaunay adjacency (the walk's only topology, Sec. 3.1 "Adjacency-Based
Traversal") is built here with scipy's Qhull as an input to the GPU path; the
oracle never reads it, it only validates it.

Scenes stand in for the paper's trained Mip-NeRF 360 models (Sec. 6.1), which
are not available: the shapes follow the paper's 2M-site budget (Sec. 5.5),
~1 Mpix views and surface-concentrated, bimodal opacity (Sec. 5.3).
Random draws use ``numpy.random.default_rng(config_no)`` in the order
sites -> density -> texels -> cameras -> upstream gradients.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# camera models (same numbering as the C ABI's voro_camera.model)
PINHOLE = 0
FISHEYE = 1          # equidistant fisheye, theta = r / f
ROLLING_SHUTTER = 2  # per-row camera centre c0 + s * delta, s = row / (H - 1)
THIN_LENS = 3        # depth of field, spp aperture samples per pixel
MOTION_BLUR = 4      # spp time samples over the exposure


@dataclasses.dataclass
class Scene:
    sites: np.ndarray      # [N,3] float32
    density: np.ndarray    # [N]   float32 (sigma, not rho)
    texels: np.ndarray     # [N,R,R,4] float32, RGBA with A = 0 (row = v, col = u)
    nbr_off: np.ndarray    # [N+1] int32 CSR offsets (Delaunay adjacency)
    nbr_idx: np.ndarray    # [M]   int32 CSR neighbour ids
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.sites.shape[0])

    @property
    def tex_res(self) -> int:
        return int(self.texels.shape[1])


@dataclasses.dataclass
class Camera:
    """A camera *description*; rays are generated from it by each side."""
    model: int
    width: int
    height: int
    c2w: np.ndarray            # [3,4] float64: columns = right, down, forward, centre
    fov: float                 # radians; pinhole: horizontal FOV, fisheye: full FOV
    tmax: float
    rs_delta: tuple = (0.0, 0.0, 0.0)   # rolling shutter / motion blur: centre shift over the frame / exposure
    lens_radius: float = 0.0           # thin lens
    focus_dist: float = 1.0            # thin lens, along the optical axis
    spp: int = 1                       # samples per pixel (thin lens: a square; motion blur: times)

    @property
    def n_pixels(self) -> int:
        return self.width * self.height

    @property
    def n_rays(self) -> int:
        return self.width * self.height * self.spp


def look_at(centre, target, up=(0.0, 1.0, 0.0)) -> np.ndarray:
    """Camera-to-world [3,4] with OpenCV axes (+x right, +y down, +z forward)."""
    c = np.asarray(centre, np.float64)
    f = np.asarray(target, np.float64) - c
    f /= np.linalg.norm(f)
    upv = np.asarray(up, np.float64)
    if abs(float(np.dot(f, upv))) > 0.999:
        upv = np.array([0.0, 0.0, 1.0])
    x = np.cross(f, upv)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    m = np.zeros((3, 4))
    m[:, 0], m[:, 1], m[:, 2], m[:, 3] = x, y, f, c
    return m


def orbit_pose(angle: float, radius: float = 3.0) -> np.ndarray:
    """Pose on a circle in the xz-plane looking at the origin."""
    c = (radius * math.sin(angle), 0.0, -radius * math.cos(angle))
    return look_at(c, (0.0, 0.0, 0.0))


# ----------------------------------------------------------------- adjacency

def delaunay_csr(sites: np.ndarray):
    """Symmetric Delaunay adjacency of the sites as CSR (int32 offsets, ids).

    Rows are sorted by neighbour id.  Built with scipy's Qhull on the CPU.
    """
    from scipy.spatial import Delaunay
    pts = np.asarray(sites, np.float64)
    tri = Delaunay(pts)
    indptr, indices = tri.vertex_neighbor_vertices
    off = np.asarray(indptr, np.int64)
    idx = np.asarray(indices, np.int64)
    # sort each row (Qhull order is arbitrary)
    row = np.repeat(np.arange(len(off) - 1), np.diff(off))
    order = np.lexsort((idx, row))
    idx = idx[order]
    if off[-1] >= 2**31:
        raise ValueError("adjacency too large for int32 offsets")
    return off.astype(np.int32), idx.astype(np.int32)


def adjacency(sites: np.ndarray):
    """delaunay_csr for small inputs, the parallel certified build above 300k sites."""
    if len(sites) > 300_000:
        return delaunay_csr_parallel(sites)
    return delaunay_csr(sites)


def _texels(rng, n, res):
    tex = np.zeros((n, res, res, 4), np.float32)
    tex[..., :3] = rng.uniform(0.0, 1.0, (n, res, res, 3)).astype(np.float32)
    return tex


def _unit_shell(rng, n, jitter=0.01):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v + rng.normal(scale=jitter, size=(n, 3))


# -------------------------------------------------------------------- configs

def scene_uniform(n=512, tex_res=4, seed=1, with_csr=True) -> Scene:
    """Config 1: uniform sites in [-1,1]^3, sigma = exp(N(0,1)), U[0,1] texels."""
    rng = np.random.default_rng(seed)
    sites = rng.uniform(-1.0, 1.0, (n, 3)).astype(np.float32)
    density = np.exp(rng.normal(0.0, 1.0, n)).astype(np.float32)
    tex = _texels(rng, n, tex_res)
    off, idx = delaunay_csr(sites) if with_csr else (None, None)
    return Scene(sites, density, tex, off, idx, name=f"uniform{n}")


def scene_shell(n=100_000, tex_res=8, seed=2, shell_frac=0.7, with_csr=True) -> Scene:
    """Config 2 (and 4/5 structure): jittered unit-sphere shell + uniform background.

    Density 50 on the shell, 0.01 elsewhere.
    """
    rng = np.random.default_rng(seed)
    n_shell = int(round(n * shell_frac))
    shell = _unit_shell(rng, n_shell)
    bg = rng.uniform(-2.0, 2.0, (n - n_shell, 3))
    sites = np.concatenate([shell, bg]).astype(np.float32)
    density = np.concatenate([np.full(n_shell, 50.0), np.full(n - n_shell, 0.01)]).astype(np.float32)
    tex = _texels(rng, n, tex_res)
    off, idx = adjacency(sites) if with_csr else (None, None)
    return Scene(sites, density, tex, off, idx, name=f"shell{n}")


def scene_ellipsoids(n_surface=1_800_000, n_background=200_000, n_ell=20, tex_res=8,
                     seed=3, with_csr=True):
    """Config 3: sites clustered on random ellipsoid surfaces plus uniform background.

    Returns (scene, ellipsoids) with ellipsoids = list of (centre, R, semi_axes).
    """
    rng = np.random.default_rng(seed)
    per = n_surface // n_ell
    pts, ells = [], []
    for k in range(n_ell):
        c = rng.uniform(-3.0, 3.0, 3)
        a = rng.uniform(0.2, 1.0, 3)
        q, r = np.linalg.qr(rng.normal(size=(3, 3)))
        q = q * np.sign(np.diag(r))
        u = rng.normal(size=(per, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        pts.append(c + (u * a) @ q.T + rng.normal(scale=0.01, size=(per, 3)))
        ells.append((c, q, a))
    n_surf = per * n_ell
    bg = rng.uniform(-4.0, 4.0, (n_background, 3))
    sites = np.concatenate(pts + [bg]).astype(np.float32)
    density = np.concatenate([np.full(n_surf, 50.0), np.full(n_background, 0.01)]).astype(np.float32)
    tex = _texels(rng, sites.shape[0], tex_res)
    off, idx = adjacency(sites) if with_csr else (None, None)
    return Scene(sites, density, tex, off, idx, name=f"ellipsoids{sites.shape[0]}"), ells, rng


def interior_camera(ells, rng, width=1280, height=840, fov_deg=60.0, tmax=14.0,
                    n_candidates=64) -> Camera:
    """Config 3 view: seeded interior point with the largest clearance from the
    ellipsoids (candidates: the origin plus seeded points), looking at the
    nearest ellipsoid centre."""
    cands = np.concatenate([np.zeros((1, 3)), rng.uniform(-3.0, 3.0, (n_candidates - 1, 3))])
    # clearance measured against densely sampled surface points
    surf = []
    for c, q, a in ells:
        u = rng.normal(size=(2000, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        surf.append(c + (u * a) @ q.T)
    surf = np.concatenate(surf)
    clear = np.array([np.min(np.linalg.norm(surf - p, axis=1)) for p in cands])
    pos = cands[int(np.argmax(clear))]
    centres = np.array([c for c, _, _ in ells])
    tgt = centres[int(np.argmin(np.linalg.norm(centres - pos, axis=1)))]
    return Camera(PINHOLE, width, height, look_at(pos, tgt), math.radians(fov_deg), tmax)


def config1():
    """512 uniform sites, 4x4 texels, 64x64 pinhole at (0,0,-3) looking +z."""
    scene = scene_uniform(512, 4, seed=1)
    cam = Camera(PINHOLE, 64, 64, look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0)),
                 math.radians(60.0), 6.0)
    return scene, [cam]


def config2(n=100_000, width=800, height=800, n_poses=8, with_csr=True):
    """100k shell scene, 8x8 texels, 800x800 pinholes on a radius-3 orbit."""
    scene = scene_shell(n, 8, seed=2, with_csr=with_csr)
    cams = [Camera(PINHOLE, width, height, orbit_pose(2.0 * math.pi * k / n_poses),
                   math.radians(60.0), 8.0) for k in range(n_poses)]
    return scene, cams


def config3(scale=1.0, with_csr=True, width=1280, height=840):
    """2M ellipsoid-surface scene, one 1280x840 pinhole from inside the volume."""
    scene, ells, rng = scene_ellipsoids(int(1_800_000 * scale), int(200_000 * scale),
                                        with_csr=with_csr)
    cam = interior_camera(ells, rng, width, height)
    return scene, [cam]


def config5_cameras(scale=1.0) -> List[Camera]:
    """Eight mixed views on the radius-3 orbit: 2 pinhole, 2 fisheye 180 deg,
    2 rolling shutter (0.1 units along camera +x over the frame), 2 thin lens
    (4 samples per pixel, lens radius 0.05, focus distance 3).

    ``scale`` shrinks the resolutions (1.0 = the full workload)."""
    def sz(w, h):
        return max(2, int(round(w * scale))), max(2, int(round(h * scale)))
    cams = []
    for k in range(8):
        pose = orbit_pose(2.0 * math.pi * k / 8)
        kind = k // 2
        if kind == 0:
            w, h = sz(1280, 840)
            cams.append(Camera(PINHOLE, w, h, pose, math.radians(60.0), 8.0))
        elif kind == 1:
            w, h = sz(1024, 1024)
            cams.append(Camera(FISHEYE, w, h, pose, math.pi, 8.0))
        elif kind == 2:
            w, h = sz(960, 540)
            delta = tuple(float(x) for x in 0.1 * pose[:, 0])
            cams.append(Camera(ROLLING_SHUTTER, w, h, pose, math.radians(60.0), 8.0,
                               rs_delta=delta))
        else:
            w, h = sz(640, 480)
            cams.append(Camera(THIN_LENS, w, h, pose, math.radians(60.0), 8.0,
                               lens_radius=0.05, focus_dist=3.0, spp=4))
    return cams


def motion_blur_cameras(scale=1.0, spp=5) -> List[Camera]:
    """Two motion-blurred pinhole views on the radius-3 orbit (960x540 at scale
    1), spp time samples over an exposure that moves the centre by 0.15 along
    the camera's +x and 0.05 along its +z."""
    cams = []
    for k in (1, 5):
        pose = orbit_pose(2.0 * math.pi * k / 8 + 0.2)
        w, h = max(2, int(round(960 * scale))), max(2, int(round(540 * scale)))
        delta = tuple(float(x) for x in 0.15 * pose[:, 0] + 0.05 * pose[:, 2])
        cams.append(Camera(MOTION_BLUR, w, h, pose, math.radians(60.0), 8.0, rs_delta=delta,
                           spp=spp))
    return cams


def config5(n=4_000_000, cam_scale=1.0, with_csr=True):
    scene = scene_shell(n, 8, seed=5, with_csr=with_csr)
    return scene, config5_cameras(cam_scale)


def upstream(n_rays: int, seed: int, with_gT: bool = True):
    """Upstream gradients dL/drgb ~ N(0,1) (and dL/dT ~ N(0,1) or zero)."""
    rng = np.random.default_rng(1000 + seed)
    g_rgb = rng.normal(size=(n_rays, 3)).astype(np.float32)
    g_T = rng.normal(size=n_rays).astype(np.float32) if with_gT else np.zeros(n_rays, np.float32)
    return g_rgb, g_T


def crop_pixels(cam: Camera, size: int, seed: int, centre: bool):
    """Pixel indices (row-major) of a size x size crop: the centre crop or a seeded one."""
    if centre:
        x0 = (cam.width - size) // 2
        y0 = (cam.height - size) // 2
    else:
        rng = np.random.default_rng(seed)
        x0 = int(rng.integers(0, cam.width - size + 1))
        y0 = int(rng.integers(0, cam.height - size + 1))
    ys, xs = np.meshgrid(np.arange(y0, y0 + size), np.arange(x0, x0 + size), indexing="ij")
    return (ys * cam.width + xs).reshape(-1)


def sample_pixels(n_total: int, k: int, seed: int):
    """k distinct pixel/ray indices out of n_total, seeded and sorted."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_total, size=min(k, n_total), replace=False))


def to_f16(tex: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even cast of f32 texels to IEEE binary16 (input preparation)."""
    return tex.astype(np.float16)


def lattice_sites(n_per_axis: int, spacing: float = 1.0, jitter: float = 0.0, seed: int = 0):
    """Cubic lattice sites centred on the origin (optionally jittered)."""
    rng = np.random.default_rng(seed)
    g = (np.arange(n_per_axis) - (n_per_axis - 1) / 2.0) * spacing
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    if jitter:
        pts = pts + rng.normal(scale=jitter, size=pts.shape)
    return pts.astype(np.float32)


def scene_from_arrays(sites, density, texels, with_csr=True, name="custom") -> Scene:
    sites = np.ascontiguousarray(sites, np.float32)
    off, idx = delaunay_csr(sites) if (with_csr and sites.shape[0] >= 5) else (None, None)
    return Scene(sites, np.ascontiguousarray(density, np.float32),
                 np.ascontiguousarray(texels, np.float32), off, idx, name=name)


def full_texels(n: int, res: int, seed: int, vi_scale: float = 1.5,
                vd_scale: float = 0.5) -> np.ndarray:
    """Seeded logits for the two-map appearance model, [n, 2, res, res, 4] f32:
    surface map N(0, vi_scale^2), view map a smaller residual N(0, vd_scale^2),
    A channel zero (Sec. 5.1, 5.2; the paper starts the view map at zero and
    keeps it small with a regulariser)."""
    rng = np.random.default_rng(5000 + seed)
    tex = np.zeros((n, 2, res, res, 4), np.float32)
    tex[:, 0, :, :, :3] = rng.normal(0.0, vi_scale, (n, res, res, 3))
    tex[:, 1, :, :, :3] = rng.normal(0.0, vd_scale, (n, res, res, 3))
    return tex


def sh_coeffs(n: int, seed: int) -> np.ndarray:
    """Seeded degree-3 spherical-harmonic colour coefficients [n, 48] f32
    (coefficient-major RGB): a base colour U[0.2, 0.8] in the l = 0 term and
    N(0, (0.15 / 2^l)^2) higher orders."""
    rng = np.random.default_rng(7000 + seed)
    k = np.zeros((n, 16, 3), np.float32)
    k[:, 0, :] = rng.uniform(0.2, 0.8, (n, 3)) * (2.0 * math.sqrt(math.pi))
    for l in range(1, 4):
        k[:, l * l:(l + 1) * (l + 1), :] = rng.normal(0.0, 0.15 / 2 ** l, (n, 2 * l + 1, 3))
    return k.reshape(n, 48)


def texels_rgb(n: int, res: int, rgb) -> np.ndarray:
    tex = np.zeros((n, res, res, 4), np.float32)
    tex[..., :3] = np.asarray(rgb, np.float32)
    return tex


# --------------------------------------------- parallel certified adjacency
#
# Qhull is single threaded (~30k sites/s).  For the 2M/4M-site scenes the
# adjacency is built on overlapping blocks in worker processes.  A point's
# neighbour set from the local triangulation of a block's points plus a halo
# is accepted only with a certificate: every local Delaunay tetrahedron
# around the point has an empty circumsphere with respect to *all* sites -
# either the sphere lies inside the region whose sites the block holds (the
# block grown by the halo, unbounded on sides beyond every site), or a k-d
# tree over all sites finds none strictly inside it.  Certified tetrahedra
# are global Delaunay tetrahedra, and a point's full star of them is its
# global star.  Points without a certificate are retried with a doubled halo.

_ADJ_TREE = None
_ADJ_HULL = None   # set of sorted global convex-hull facets (vertex-id triples)


def _circumspheres(pts, simp):
    a = pts[simp[:, 0]]
    A = 2.0 * (pts[simp[:, 1:]] - a[:, None, :])                    # [T,3,3]
    b = np.sum(pts[simp[:, 1:]] ** 2, axis=2) - np.sum(a * a, axis=1)[:, None]
    with np.errstate(all="ignore"):
        det = np.linalg.det(A)
        ok = np.abs(det) > 1e-300
        c = np.full(a.shape, np.inf)
        if np.any(ok):
            c[ok] = np.linalg.solve(A[ok], b[ok][..., None])[..., 0]
        r = np.linalg.norm(c - a, axis=1)
    r[~np.isfinite(r)] = np.inf
    return c, r


def _block_job(args):
    (pts, gidx, owned, lo, hi, open_lo, open_hi) = args
    from scipy.spatial import Delaunay
    tri = Delaunay(pts)
    simp = tri.simplices
    # only tetrahedra around owned points matter
    simp = simp[np.any(owned[simp], axis=1)]
    c, r = _circumspheres(pts, simp)
    finite = np.isfinite(r)
    inside = finite.copy()
    for ax in range(3):
        if not open_lo[ax]:
            inside &= (c[:, ax] - r) >= lo[ax]
        if not open_hi[ax]:
            inside &= (c[:, ax] + r) <= hi[ax]
    check = np.nonzero(finite & ~inside)[0]
    certified = inside.copy()
    if len(check):
        cnt = _ADJ_TREE.query_ball_point(c[check], r[check] * (1.0 - 1e-10), return_length=True)
        certified[check] = np.asarray(cnt) == 0
    bad = np.bincount(simp[~certified].ravel(), minlength=len(pts)) > 0
    # where to look next: the rejected spheres hold the sites this star lacks
    need_lo = np.full((len(pts), 3), np.inf)
    need_hi = np.full((len(pts), 3), -np.inf)
    rej = np.nonzero(~certified & np.isfinite(r))[0]
    for k in range(4):
        np.minimum.at(need_lo, simp[rej, k], c[rej] - r[rej, None])
        np.maximum.at(need_hi, simp[rej, k], c[rej] + r[rej, None])
    # a vertex of the local hull has a star cut open by its hull faces: it is
    # complete only where those faces are facets of the global hull too
    for f in tri.convex_hull:
        if not np.any(owned[f]):
            continue
        key = tuple(sorted(int(x) for x in gidx[f]))
        if key not in _ADJ_HULL:
            bad[f] = True
    indptr, indices = tri.vertex_neighbor_vertices
    ok = np.nonzero(owned & ~bad)[0]
    deg = indptr[ok + 1] - indptr[ok]
    take = np.concatenate([np.arange(indptr[i], indptr[i + 1]) for i in ok]) if len(ok) else \
        np.zeros(0, np.int64)
    fl = np.nonzero(owned & bad)[0]
    return gidx[ok], deg, gidx[indices[take]], gidx[fl], need_lo[fl], need_hi[fl]


def delaunay_csr_parallel(sites: np.ndarray, blocks_per_axis: int = 4, workers: int = None,
                          halo: float = None, max_rounds: int = 8, verbose: bool = False):
    """Same CSR as delaunay_csr (rows sorted), built on overlapping blocks in
    parallel worker processes with a per-point certificate (see above)."""
    import multiprocessing as mp
    import os
    import time
    pts = np.asarray(sites, np.float64)
    n = len(pts)
    workers = workers or min(16, os.cpu_count() or 1)
    glo, ghi = pts.min(0), pts.max(0)
    ext = np.maximum(ghi - glo, 1e-300)
    B = blocks_per_axis
    h = halo if halo is not None else 0.15 * float(ext.max()) / B
    cell = np.minimum(((pts - glo) / ext * B).astype(np.int64), B - 1)
    bid = (cell[:, 0] * B + cell[:, 1]) * B + cell[:, 2]
    todo = [(b, ix) for b in range(B ** 3) for ix in [np.nonzero(bid == b)[0]] if len(ix)]
    deg = np.zeros(n, np.int64)
    parts = []
    done = np.zeros(n, bool)

    # fork workers (they share the k-d tree): call this only from a process
    # that has not touched the GPU (scene_cached runs it in a child process)
    global _ADJ_TREE, _ADJ_HULL
    from scipy.spatial import ConvexHull, cKDTree
    _ADJ_TREE = cKDTree(pts)
    _ADJ_HULL = {tuple(sorted(int(x) for x in f)) for f in ConvexHull(pts).simplices}

    # Every job also holds the global hull vertices: sites just inside the
    # hull lie under hull facets whose far vertices are their neighbours.
    hull_vertices = np.unique(np.array(sorted(_ADJ_HULL), np.int64).ravel())

    def region_job(own, lo, hi):
        # sites in the box [lo, hi] (k-d tree, Chebyshev ball, then trimmed)
        ctr, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
        cand = np.asarray(_ADJ_TREE.query_ball_point(ctr, float(half.max()) * (1 + 1e-12), p=np.inf),
                          np.int64)
        cand = cand[np.all((pts[cand] >= lo) & (pts[cand] <= hi), axis=1)]
        sel = np.union1d(cand, np.union1d(hull_vertices, own))
        owned = np.zeros(len(sel), bool)
        owned[np.searchsorted(sel, own)] = True
        return (pts[sel], sel, owned, lo, hi, lo <= glo, hi >= ghi)

    def block_job(b, own):
        bx, by, bz = b // (B * B), (b // B) % B, b % B
        blo = glo + ext * np.array([bx, by, bz]) / B
        bhi = glo + ext * np.array([bx + 1, by + 1, bz + 1]) / B
        return region_job(own, np.maximum(blo - h, glo - h), np.minimum(bhi + h, ghi + h))

    # span of the global hull facets around each hull vertex: a hull
    # vertex's neighbours can lie anywhere on those facets
    hull_span = {}
    for f in _ADJ_HULL:
        fp = pts[list(f)]
        for v in f:
            lo_, hi_ = hull_span.get(v, (fp.min(0), fp.max(0)))
            hull_span[v] = (np.minimum(lo_, fp.min(0)), np.maximum(hi_, fp.max(0)))

    def point_region(i, nlo, nhi):
        lo, hi = pts[i] - h, pts[i] + h
        if i in hull_span:
            lo, hi = np.minimum(lo, hull_span[i][0] - h), np.maximum(hi, hull_span[i][1] + h)
        lo = np.maximum(np.minimum(lo, nlo), glo - h)
        hi = np.minimum(np.maximum(hi, nhi), ghi + h)
        return lo, hi

    def group_jobs(failed):
        # stragglers close together share one job whose region covers all of theirs
        G = 4 * B
        key = {}
        for i, nlo, nhi in failed:
            g = tuple(np.minimum(((pts[i] - glo) / ext * G).astype(np.int64), G - 1))
            lo, hi = point_region(i, nlo, nhi)
            if g in key:
                ids, glo_, ghi_ = key[g]
                ids.append(i)
                key[g] = (ids, np.minimum(glo_, lo), np.maximum(ghi_, hi))
            else:
                key[g] = ([i], lo, hi)
        return [region_job(np.array(sorted(ids), np.int64), lo, hi) for ids, lo, hi in key.values()]

    # Sites near a face of the bounding box have long, flat Delaunay
    # tetrahedra (nothing lies beyond the face), so each face gets one slab
    # job spanning the whole face; interior blocks own the remaining sites.
    dist = np.minimum(pts - glo, ghi - pts)                  # [n,3]
    face_axis = np.argmin(dist, axis=1)
    near = dist[np.arange(n), face_axis] < 2.0 * h
    side_hi = (ghi - pts)[np.arange(n), face_axis] < (pts - glo)[np.arange(n), face_axis]
    jobs = []
    for ax in range(3):
        for hi_side in (False, True):
            own = np.nonzero(near & (face_axis == ax) & (side_hi == hi_side))[0]
            if not len(own):
                continue
            lo, hi = glo - h, ghi + h
            if hi_side:
                lo = lo.copy()
                lo[ax] = ghi[ax] - 4.0 * h
            else:
                hi = hi.copy()
                hi[ax] = glo[ax] + 4.0 * h
            jobs.append(region_job(own, lo, hi))
    for b, own in todo:
        own = own[~near[own]]
        if len(own):
            jobs.append(block_job(b, own))

    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        for rnd in range(max_rounds):
            t0 = time.perf_counter()
            results = pool.map(_block_job, jobs)
            failed = []
            for ids, dg, nb, bad, nlo, nhi in results:
                deg[ids] = dg
                done[ids] = True
                parts.append((ids, dg, nb))
                failed.extend(zip(bad.tolist(), nlo, nhi))
            if verbose:
                print(f"[adjacency] round {rnd}: {len(jobs)} jobs, halo {h:.3f}, "
                      f"{len(failed)} uncertified, {time.perf_counter() - t0:.1f}s", flush=True)
            if not failed:
                break
            # the few uncertified points: one region each, covering the
            # spheres that rejected them; the halo doubles in case that fails
            h *= 2.0
            jobs = group_jobs(failed)
        else:
            raise RuntimeError("adjacency certificate did not converge")
    _ADJ_TREE = None
    _ADJ_HULL = None
    if not done.all():
        raise RuntimeError("adjacency incomplete")
    off = np.zeros(n + 1, np.int64)
    np.cumsum(deg, out=off[1:])
    if off[-1] >= 2 ** 31:
        raise ValueError("adjacency too large for int32 offsets")
    idx = np.empty(off[-1], np.int64)
    for ids, dg, nb in parts:
        src = np.concatenate([[0], np.cumsum(dg)])
        for k, i in enumerate(ids):
            idx[off[i]:off[i + 1]] = np.sort(nb[src[k]:src[k + 1]])
    return off.astype(np.int32), idx.astype(np.int32)


# ------------------------------------------------------------ scene cache

def _build_config(name: str):
    """(scene, camera extras) of a named workload."""
    if name == "config2":
        return config2()[0], {}
    if name == "config3":
        scene, cams = config3(with_csr=True)
        return scene, {"cam_c2w": cams[0].c2w}
    if name == "config5":
        return config5()[0], {}
    if name.startswith("shell"):
        return scene_shell(int(name[5:]), 8, seed=5), {}
    raise ValueError(name)


def save_scene(scene: Scene, path: str, extras=None):
    np.savez(path, sites=scene.sites, density=scene.density, texels=scene.texels,
             nbr_off=scene.nbr_off, nbr_idx=scene.nbr_idx, name=np.array(scene.name),
             **{f"x_{k}": v for k, v in (extras or {}).items()})


def load_scene(path: str) -> Scene:
    z = np.load(path, allow_pickle=False)
    s = Scene(z["sites"], z["density"], z["texels"], z["nbr_off"], z["nbr_idx"],
              name=str(z["name"]))
    s.extras = {k[2:]: z[k] for k in z.files if k.startswith("x_")}
    return s


def config3_camera(scene: Scene) -> Camera:
    """The config-3 interior view of a cached config-3 scene."""
    return Camera(PINHOLE, 1280, 840, np.asarray(scene.extras["cam_c2w"], np.float64),
                  math.radians(60.0), 14.0)


def scene_cache_path(name: str, cache_dir: str = None) -> str:
    import os
    cache_dir = cache_dir or os.environ.get("VORO_SCENE_CACHE", "/tmp/voro_scene_cache")
    return os.path.join(cache_dir, f"{name}.npz")


def scene_cached(name: str, cache_dir: str = None) -> Scene:
    """A named scene (config2, config3, config5, shell<N>) from an .npz cache,
    built on a miss by a child process (so the caller may already hold the GPU:
    the parallel adjacency build forks workers only inside that child)."""
    import os
    import subprocess
    import sys
    path = scene_cache_path(name, cache_dir)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    if not os.path.exists(path):
        tmp = path[:-4] + ".tmp.npz"
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        subprocess.run([sys.executable, "-m", "paper_2608_17682_amd.synth", name, tmp], check=True,
                       cwd=root)
        os.replace(tmp, path)
    return load_scene(path)


if __name__ == "__main__":
    import sys
    _scene, _extras = _build_config(sys.argv[1])
    save_scene(_scene, sys.argv[2], _extras)
