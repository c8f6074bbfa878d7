"""The oracle's pool runners return what the one-ray-at-a-time oracle returns,
ray for ray and in order (they add no arithmetic of their own)."""
import numpy as np

from oracle import adjoint, batch, cameras, render
from paper_2608_17682_amd import synth
from helpers import f32


def _rays():
    scene, cams = synth.config1()
    o, d, tm, _ = cameras.camera_rays_of(cams[0])
    pick = synth.sample_pixels(len(o), 96, 4)
    return scene, f32(o[pick]), f32(d[pick]), f32(tm[pick])


def test_evaluate_equals_render_rays():
    scene, o, d, tm = _rays()
    rgb, T, recs = render.render_rays(scene.sites, scene.density, scene.texels, o, d, tm)
    res = batch.evaluate(scene.sites, scene.density, scene.texels, o, d, tm, workers=3, chunk=7,
                         keep_records=np.arange(len(o)) % 2 == 0)
    assert np.array_equal(res["rgb"], rgb) and np.array_equal(res["T"], T)
    for r, rec in enumerate(recs):
        assert res["K"][r] == rec.K
        assert res["cells"][r].tolist() == rec.cells
        assert (res["records"][r] is not None) == (r % 2 == 0)


def test_render_rays_parallel_equals_render_rays():
    scene, o, d, tm = _rays()
    rgb, T, recs = render.render_rays(scene.sites, scene.density, scene.texels, o, d, tm)
    rgb2, T2, recs2 = render.render_rays_parallel(scene.sites, scene.density, scene.texels,
                                                  o, d, tm, workers=3, chunk=10)
    assert np.array_equal(rgb2, rgb) and np.array_equal(T2, T)
    assert [r.cells for r in recs2] == [r.cells for r in recs]


def test_sparse_gradients_equal_dense():
    scene, o, d, tm = _rays()
    rgb, T, recs = render.render_rays(scene.sites, scene.density, scene.texels, o, d, tm)
    g_rgb, _ = synth.upstream(len(o), 1)
    use = [r if k % 3 else None for k, r in enumerate(recs)]
    ids, gs, gd, gt = batch.sparse_gradients(scene.sites, scene.density, scene.texels, o, d, tm,
                                             use, g_rgb)
    kept = [r for r in use if r is not None]
    sel = [k for k, r in enumerate(use) if r is not None]
    ws, wd, wt = adjoint.grad_rays(scene.sites, scene.density, scene.texels, o[sel], d[sel],
                                   tm[sel], kept, g_rgb[sel], np.zeros(len(sel)))
    touched = np.nonzero(np.any(ws != 0, 1) | (wd != 0) | np.any(wt != 0, (1, 2, 3)))[0]
    assert set(touched.tolist()) <= set(ids.tolist())
    np.testing.assert_allclose(gs, ws[ids], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(gd, wd[ids], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(gt, wt[ids], rtol=1e-12, atol=1e-15)


def test_sparse_gradients_equal_dense_full_model():
    # the two-map texel blocks of the full appearance model accumulate like
    # the dense adjoint's [N, 2, R, R, 4] gradient
    scene, o, d, tm = _rays()
    tex = synth.full_texels(scene.n, scene.tex_res, seed=3)
    rgb, T, recs = render.render_rays(scene.sites, scene.density, tex, o, d, tm, appearance=1)
    res = batch.evaluate(scene.sites, scene.density, tex, o, d, tm, workers=2, chunk=11,
                         keep_records=np.ones(len(o), bool), appearance=1)
    assert np.array_equal(res["rgb"], rgb) and np.array_equal(res["T"], T)
    g_rgb, _ = synth.upstream(len(o), 2)
    ids, gs, gd, gt = batch.sparse_gradients(scene.sites, scene.density, tex, o, d, tm,
                                             res["records"], g_rgb)
    assert gt.shape[1:] == tex.shape[1:]
    ws, wd, wt = adjoint.grad_rays(scene.sites, scene.density, tex, o, d, tm, recs, g_rgb,
                                   np.zeros(len(o)))
    touched = np.nonzero(np.any(ws != 0, 1) | (wd != 0) | np.any(wt != 0, (1, 2, 3, 4)))[0]
    assert set(touched.tolist()) <= set(ids.tolist())
    assert np.abs(wt[:, 1]).max() > 0    # the view map is exercised
    np.testing.assert_allclose(gs, ws[ids], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(gd, wd[ids], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(gt, wt[ids], rtol=1e-12, atol=1e-15)


def test_evaluate_equals_render_rays_sh():
    scene, o, d, tm = _rays()
    k = synth.sh_coeffs(scene.n, seed=3)
    rgb, T, _ = render.render_rays(scene.sites, scene.density, k, o, d, tm, appearance=2)
    res = batch.evaluate(scene.sites, scene.density, k, o, d, tm, workers=2, chunk=13,
                         appearance=2)
    assert np.array_equal(res["rgb"], rgb) and np.array_equal(res["T"], T)
