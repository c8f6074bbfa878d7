"""GPU edge cases against the FP64 oracle: texture resolutions at both limits,
the smallest scenes (one site, two sites), a cell of very high degree, tiny
ray extents, the largest multi-view launch (16 views, 64 samples per pixel),
and a malformed adjacency (neutralised and counted, never followed)."""
import math

import numpy as np
import pytest
import torch

from oracle import cameras, render, walk
from paper_2608_17682_amd import synth, voro
from helpers import f32, stop_degenerate

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    voro.lib()
    return torch.device("cuda:0")


def upload(dev, sites, density, tex, off, idx):
    ds = voro.DeviceScene(to_dev(np.asarray(sites, np.float32), dev),
                          to_dev(np.asarray(density, np.float32), dev),
                          to_dev(np.asarray(off, np.int32), dev),
                          to_dev(np.asarray(idx, np.int32), dev), to_dev(tex, dev))
    voro.voro_prepare(ds)
    return ds


def random_rays(n, seed, spread=0.9, tmax=3.0):
    rng = np.random.default_rng(seed)
    o = rng.uniform(-spread, spread, (n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return f32(o), f32(d), np.full(n, tmax, np.float32)


def check_against_oracle(dev, ds, sites, density, tex, o, d, tm, params=None, atol=1e-4):
    starts = np.array([walk.nearest_site(sites, x)[0] for x in o], np.int32)
    rgb_o, T_o, recs = render.render_rays(sites, density, tex, o, d, tm, starts=starts)
    rgb, T = voro.voro_render_fwd(ds, to_dev(o, dev), to_dev(d, dev), to_dev(tm, dev),
                                  to_dev(starts, dev), params or voro.default_params())
    keep = np.array([r is None or not stop_degenerate(r, 1e-4) for r in recs])
    np.testing.assert_allclose(rgb.cpu().numpy()[keep], rgb_o[keep], atol=atol, rtol=0)
    np.testing.assert_allclose(T.cpu().numpy()[keep], T_o[keep], atol=atol, rtol=0)
    return recs


@pytest.mark.parametrize("res", [2, 16])
def test_texture_resolution_limits(dev, res):
    scene = synth.scene_uniform(200, res, seed=11)
    announce(f"texture resolution {res}")
    ds = upload(dev, scene.sites, scene.density, scene.texels, scene.nbr_off, scene.nbr_idx)
    assert ds.tex_res == res
    o, d, tm = random_rays(300, 12)
    check_against_oracle(dev, ds, scene.sites, scene.density, scene.texels, o, d, tm)


def test_single_site_scene(dev):
    # one unbounded cell: every ray stays in it to tmax, T = exp(-sigma tmax)
    sites = np.array([[0.1, -0.2, 0.3]], np.float32)
    dens = np.array([0.7], np.float32)
    tex = synth.scene_uniform(8, 4, seed=3).texels[:1]
    announce("one-site scene")
    ds = upload(dev, sites, dens, tex, [0, 0], np.zeros(0, np.int32))
    o, d, tm = random_rays(64, 13)
    check_against_oracle(dev, ds, sites, dens, tex, o, d, tm)
    _, T = voro.voro_render_fwd(ds, to_dev(o, dev), to_dev(d, dev), to_dev(tm, dev),
                                torch.zeros(64, dtype=torch.int32, device=dev))
    np.testing.assert_allclose(T.cpu().numpy(), math.exp(-0.7 * 3.0), rtol=1e-5)


def test_two_site_scene_closed_form(dev):
    # the bisector z = 0 at t* = 3 for o = (0,0,-3), w = +z (the two-site pin)
    sites = np.array([[0.0, 0.0, -0.5], [0.0, 0.0, 0.5]], np.float32)
    dens = np.array([0.4, 1.3], np.float32)
    tex = synth.texels_rgb(2, 4, (0.25, 0.5, 0.75))
    tex[1, ..., :3] = (0.9, 0.1, 0.2)
    announce("two-site scene")
    ds = upload(dev, sites, dens, tex, [0, 1, 2], [1, 0])
    o = f32([[0.0, 0.0, -3.0]])
    d = f32([[0.0, 0.0, 1.0]])
    rgb, T = voro.voro_render_fwd(ds, to_dev(o, dev), to_dev(d, dev),
                                  to_dev(np.array([6.0], np.float32), dev),
                                  torch.zeros(1, dtype=torch.int32, device=dev))
    a0 = 1.0 - math.exp(-0.4 * 3.0)
    a1 = 1.0 - math.exp(-1.3 * 3.0)
    want = a0 * np.array([0.25, 0.5, 0.75]) + (1.0 - a0) * a1 * np.array([0.9, 0.1, 0.2])
    np.testing.assert_allclose(rgb.cpu().numpy()[0], want, atol=2e-6)
    assert float(T[0]) == pytest.approx(math.exp(-3.0 * (0.4 + 1.3)), rel=1e-5)


def test_high_degree_cell(dev):
    # a centre site inside a shell of 300 sites: its cell has hundreds of faces
    rng = np.random.default_rng(21)
    u = rng.normal(size=(300, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    sites = np.concatenate([[[0.0, 0.0, 0.0]], 0.5 * u, rng.uniform(-1.5, 1.5, (60, 3))])
    sites = sites.astype(np.float32)
    off, idx = synth.delaunay_csr(sites)
    deg0 = int(off[1] - off[0])
    assert deg0 > 100
    dens = np.full(len(sites), 0.5, np.float32)
    tex = synth.scene_uniform(len(sites), 4, seed=22, with_csr=False).texels
    announce(f"high-degree cell ({deg0} faces)")
    ds = upload(dev, sites, dens, tex, off, idx)
    rng2 = np.random.default_rng(23)
    o = f32(rng2.normal(0.0, 0.02, (128, 3)))   # rays from inside the centre cell
    d = rng2.normal(size=(128, 3))
    d = f32(d / np.linalg.norm(d, axis=1, keepdims=True))
    check_against_oracle(dev, ds, sites, dens, tex, o, d, np.full(128, 2.0, np.float32))


def test_tiny_ray_extents(dev):
    scene = synth.scene_uniform(150, 4, seed=31)
    ds = upload(dev, scene.sites, scene.density, scene.texels, scene.nbr_off, scene.nbr_idx)
    o, d, _ = random_rays(200, 32)
    tm = np.full(200, 1e-5, np.float32)
    announce("tmax 1e-5")
    check_against_oracle(dev, ds, scene.sites, scene.density, scene.texels, o, d, tm, atol=1e-6)


def test_sixteen_views_and_64_samples(dev):
    scene = synth.scene_uniform(300, 4, seed=41)
    ds = upload(dev, scene.sites, scene.density, scene.texels, scene.nbr_off, scene.nbr_idx)
    cams = (synth.config5_cameras(scale=0.02) + synth.motion_blur_cameras(scale=0.02, spp=64)
            + synth.config5_cameras(scale=0.015)[:6])
    cams[6].spp = 64                               # a thin-lens view with 8 x 8 samples
    for cm in cams:
        cm.tmax = 4.0
    assert len(cams) == voro.MAX_VIEWS
    announce(f"{len(cams)} views, 64 samples per pixel")
    rgb_v, T_v, ray_v = voro.voro_render_views_fwd(ds, cams, voro.default_params())
    rgb_v, T_v = rgb_v.cpu().numpy(), T_v.cpu().numpy()
    off = 0
    for vi, cm in enumerate(cams):
        o, d, tm, valid = cameras.camera_rays_of(cm)
        for p in synth.sample_pixels(cm.n_pixels, 4, vi):
            rs = slice(p * cm.spp, (p + 1) * cm.spp)
            rgb_o, T_o, recs = render.render_rays(scene.sites, scene.density, scene.texels,
                                                  f32(o[rs]), f32(d[rs]), f32(tm[rs]))
            if any(r is not None and stop_degenerate(r, 1e-4) for r in recs):
                continue
            np.testing.assert_allclose(rgb_v[off + p], rgb_o.mean(0), atol=1e-4, rtol=0)
        off += cm.n_pixels


def test_malformed_adjacency_is_neutralised(dev):
    scene = synth.scene_uniform(100, 4, seed=51)
    off = scene.nbr_off.astype(np.int64).copy()
    idx = scene.nbr_idx.astype(np.int64).copy()
    idx[off[3]] = -1                 # out-of-range ids
    idx[off[4]] = 100 + 7
    idx[off[5]] = 5                  # a self loop
    off[10] = off[11] + 2            # a row whose end precedes its start
    stats = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    ds = voro.DeviceScene(to_dev(scene.sites, dev), to_dev(scene.density, dev),
                          to_dev(off.astype(np.int32), dev), to_dev(idx.astype(np.int32), dev),
                          to_dev(scene.texels, dev))
    announce("malformed adjacency")
    voro.voro_prepare(ds, stats=stats)
    assert int(stats[voro.STAT_NAMES.index("bad_csr")]) >= 4
    o, d, tm = random_rays(256, 52)
    starts = np.array([walk.nearest_site(scene.sites, x)[0] for x in o], np.int32)
    rgb, T = voro.voro_render_fwd(ds, to_dev(o, dev), to_dev(d, dev), to_dev(tm, dev),
                                  to_dev(starts, dev))
    torch.cuda.synchronize()
    assert torch.isfinite(rgb).all() and torch.isfinite(T).all()
    assert float(T.min()) >= 0.0 and float(T.max()) <= 1.0


def test_morton_sort_is_stable_on_equal_codes(dev):
    # 10x10x10 grid positions, each taken by three cells (equal Morton codes);
    # distinct positions are far apart in the 1024^3 code grid.  The reorder
    # must keep each trio together and in its original order.
    announce("morton reorder: equal codes keep their order")
    g = (np.arange(10) + 0.5) / 10.0
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(3)
    order = rng.permutation(3 * len(pos))
    sites = np.repeat(pos, 3, axis=0)[order].astype(np.float32)
    n = len(sites)
    tex = np.zeros((n, 2, 2, 4), np.float32)
    tex[:, :, :, 0] = np.arange(n, dtype=np.float32)[:, None, None]
    off = np.zeros(n + 1, np.int32)
    ds = voro.DeviceScene(to_dev(sites, dev), to_dev(np.ones(n, np.float32), dev),
                          to_dev(off, dev), torch.zeros(0, dtype=torch.int32, device=dev),
                          to_dev(tex, dev))
    ds2, perm, inv = voro.voro_morton_reorder(ds)
    perm = perm.cpu().numpy()
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert np.array_equal(inv.cpu().numpy()[perm], np.arange(n))
    s2 = ds2.sites.cpu().numpy()
    np.testing.assert_array_equal(s2, sites[perm])
    np.testing.assert_array_equal(ds2.texels.cpu().numpy()[:, 0, 0, 0], perm.astype(np.float32))
    for k in range(0, n, 3):
        trio = perm[k:k + 3]
        assert np.all(sites[trio] == sites[trio[0]]), k
        assert trio[0] < trio[1] < trio[2], (k, trio)
