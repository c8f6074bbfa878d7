"""GPU parity of the full appearance model (appearance 1: surface map at the
site-to-hit-point direction plus view map, sigmoid of the summed logits;
Sec. 5.1, 5.2) against the FP64 oracle: every ray of the config-1 scene
with two seeded logit maps, the adjoint over the non-degenerate rays, the
multi-view launch against explicit rays, and half-precision maps."""
import numpy as np
import pytest
import torch

from oracle import adjoint, cameras, render, walk
from paper_2608_17682_amd import synth, voro
from helpers import degenerate, f32, stop_degenerate

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


class Case:
    pass


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    voro.lib()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def cf(dev):
    c = Case()
    c.scene, c.cams = synth.config1()
    c.tex = synth.full_texels(c.scene.n, c.scene.tex_res, seed=1)
    o, d, tm, _ = cameras.camera_rays_of(c.cams[0])
    c.o, c.d, c.tm = f32(o), f32(d), f32(tm)
    c.start = np.array([walk.nearest_site(c.scene.sites, x)[0] for x in c.o[:1]] * len(c.o),
                       np.int32)
    c.rgb, c.T, c.recs = render.render_rays(c.scene.sites, c.scene.density, c.tex, c.o, c.d,
                                            c.tm, starts=c.start, appearance=1)
    c.ds = voro.DeviceScene(to_dev(c.scene.sites, dev), to_dev(c.scene.density, dev),
                            to_dev(c.scene.nbr_off, dev), to_dev(c.scene.nbr_idx, dev),
                            to_dev(c.tex, dev))
    assert c.ds.tex_maps == 2 and c.ds.tex_res == c.scene.tex_res
    announce("full appearance: prepare")
    voro.voro_prepare(c.ds)
    c.O, c.D, c.TM, c.S = (to_dev(c.o, dev), to_dev(c.d, dev), to_dev(c.tm, dev),
                           to_dev(c.start, dev))
    return c


@pytest.mark.parametrize("lpr", [1, 4])
def test_full_fwd_matches_oracle(dev, cf, lpr):
    p = voro.default_params(appearance=1, lanes_per_ray=lpr)
    nsteps = torch.empty(len(cf.o), dtype=torch.int32, device=dev)
    announce(f"full fwd lpr={lpr}")
    rgb, T = voro.voro_render_fwd(cf.ds, cf.O, cf.D, cf.TM, cf.S, p, nsteps=nsteps)
    rgb, T, K = rgb.cpu().numpy(), T.cpu().numpy(), nsteps.cpu().numpy()
    keep = np.array([not stop_degenerate(r, 1e-4) for r in cf.recs])
    assert keep.mean() > 0.99
    np.testing.assert_allclose(rgb[keep], cf.rgb[keep], atol=1e-4, rtol=0)
    np.testing.assert_allclose(T[keep], cf.T[keep], atol=1e-4, rtol=0)
    seq = np.array([not degenerate(r, 1e-4, float(cf.tm[0])) for r in cf.recs])
    assert np.array_equal(K[seq], [cf.recs[i].K for i in np.nonzero(seq)[0]])
    # the colour is not the single-map one: both maps matter
    assert np.abs(cf.rgb).max() > 0.05


def assert_grad_close(got, want, name):
    scale = max(1e-12, float(np.abs(want).max()))
    err = np.abs(got - want)
    assert err.max() <= 1e-4 * scale + 1e-6, (name, err.max(), scale)
    assert np.linalg.norm(got - want) <= 1e-4 * np.linalg.norm(want) + 1e-6, name


@pytest.mark.parametrize("lpr", [1, 4])
def test_full_bwd_matches_oracle_gradient(dev, cf, lpr):
    deg = np.array([degenerate(r, 1e-4, float(cf.tm[0])) for r in cf.recs])
    sel = np.nonzero(~deg)[0]
    g_rgb, g_T = synth.upstream(len(cf.o), 1)
    g_rgb, g_T = g_rgb[sel], g_T[sel]
    want = adjoint.grad_rays(cf.scene.sites, cf.scene.density, cf.tex, cf.o[sel], cf.d[sel],
                             cf.tm[sel], [cf.recs[i] for i in sel], g_rgb, g_T)
    announce(f"full bwd lpr={lpr}")
    p = voro.default_params(appearance=1, lanes_per_ray=lpr)
    si = torch.from_numpy(sel).to(dev)
    rgb, T = voro.voro_render_fwd(cf.ds, cf.O[si], cf.D[si], cf.TM[si], cf.S[si], p)
    got = voro.voro_render_bwd(cf.ds, cf.O[si], cf.D[si], cf.TM[si], cf.S[si], rgb, T,
                               to_dev(g_rgb, dev), to_dev(g_T, dev), p)
    got = [x.cpu().numpy() for x in got]
    assert got[2].shape == cf.tex.shape
    for g, w, name in zip(got, want, ("sites", "density", "texels")):
        assert_grad_close(g, w, name)
    assert np.all(got[2][..., 3] == 0)
    # both maps and the surface-direction position term are exercised
    assert np.abs(want[2][:, 0]).max() > 0 and np.abs(want[2][:, 1]).max() > 0


def test_full_model_with_distortion(dev, cf):
    deg = np.array([degenerate(r, 1e-4, float(cf.tm[0])) for r in cf.recs])
    sel = np.nonzero(~deg)[0][::2]
    g_rgb, g_T = synth.upstream(len(cf.o), 2)
    g_rgb, g_T = g_rgb[sel], g_T[sel]
    g_dist = np.random.default_rng(3).normal(0.0, 2.0, len(sel)).astype(np.float32)
    want = adjoint.grad_rays(cf.scene.sites, cf.scene.density, cf.tex, cf.o[sel], cf.d[sel],
                             cf.tm[sel], [cf.recs[i] for i in sel], g_rgb, g_T, g_dist)
    announce("full appearance + distortion bwd")
    p = voro.default_params(appearance=1)
    si = torch.from_numpy(sel).to(dev)
    dist = torch.empty((len(sel), 3), dtype=torch.float32, device=dev)
    rgb, T = voro.voro_render_fwd(cf.ds, cf.O[si], cf.D[si], cf.TM[si], cf.S[si], p, dist=dist)
    np.testing.assert_allclose(dist[:, 0].cpu().numpy(), [cf.recs[i].dist for i in sel],
                               atol=2e-6, rtol=1e-4)
    got = voro.voro_render_bwd(cf.ds, cf.O[si], cf.D[si], cf.TM[si], cf.S[si], rgb, T,
                               to_dev(g_rgb, dev), to_dev(g_T, dev), p, dist=dist,
                               g_dist=to_dev(g_dist, dev))
    for g, w, name in zip(got, want, ("sites", "density", "texels")):
        assert_grad_close(g.cpu().numpy(), w, name)


def test_full_views_equal_explicit(dev, cf):
    cams = synth.config5_cameras(scale=0.05)
    for cm in cams:
        cm.tmax = 4.0
    nr = [cm.n_rays for cm in cams]
    npx = sum(cm.n_pixels for cm in cams)
    p = voro.default_params(appearance=1)
    announce("full appearance: views vs explicit, fwd and bwd")
    rgb_v, T_v, ray_v = voro.voro_render_views_fwd(cf.ds, cams, p)
    O, D, TM = voro.voro_gen_rays(cams, dev)
    centres = to_dev(f32([cm.c2w[:, 3] for cm in cams]), dev)
    cc = voro.voro_locate_origins(cf.ds, centres)
    hint = torch.cat([cc[i:i + 1].expand(n) for i, n in enumerate(nr)]).contiguous()
    S = voro.voro_locate_origins(cf.ds, O, hint=hint)
    rgb_e, T_e = voro.voro_render_fwd(cf.ds, O, D, TM, S, p)
    off_r = off_p = 0
    rv, tv, re_ = rgb_v.cpu().numpy(), T_v.cpu().numpy(), rgb_e.cpu().numpy()
    for cm in cams:
        n, m = cm.n_rays, cm.n_pixels
        if cm.spp == 1:
            np.testing.assert_array_equal(rv[off_p:off_p + m], re_[off_r:off_r + n])
        else:
            mean = re_[off_r:off_r + n].reshape(m, cm.spp, 3).mean(1)
            np.testing.assert_allclose(rv[off_p:off_p + m], mean, atol=1e-6)
        off_r += n
        off_p += m
    g_rgb, g_T = synth.upstream(npx, 5)
    gv = voro.voro_render_views_bwd(cf.ds, cams, rgb_v, T_v, ray_v, to_dev(g_rgb, dev),
                                    to_dev(g_T, dev), p)
    # the same adjoint reading the forward's first 3 exits of each ray (the
    # rest searched): the full model reloads each cell's record itself
    trace = torch.empty((3, sum(nr), 2), dtype=torch.int32, device=dev)
    voro.voro_render_views_fwd(cf.ds, cams, p, trace=trace)
    gx = voro.voro_render_views_bwd(cf.ds, cams, rgb_v, T_v, ray_v, to_dev(g_rgb, dev),
                                    to_dev(g_T, dev), p, trace=trace)
    gr, gt_ = [], []
    off = 0
    for cm in cams:
        sl = slice(off, off + cm.n_pixels)
        gr.append(np.repeat(g_rgb[sl], cm.spp, 0) / cm.spp)
        gt_.append(np.repeat(g_T[sl], cm.spp, 0) / cm.spp)
        off += cm.n_pixels
    ge = voro.voro_render_bwd(cf.ds, O, D, TM, S, rgb_e, T_e, to_dev(np.concatenate(gr), dev),
                              to_dev(np.concatenate(gt_), dev), p)
    for a, x, b, name in zip(gv, gx, ge, ("sites", "density", "texels")):
        a, x, b = a.cpu().numpy(), x.cpu().numpy(), b.cpu().numpy()
        assert np.abs(a - b).max() <= 1e-5 * max(1.0, np.abs(b).max()), name
        assert np.abs(x - b).max() <= 1e-5 * max(1.0, np.abs(b).max()), name


@pytest.mark.parametrize("dtype", ["float16", "bfloat16"])
def test_full_half_maps_match_oracle_on_dequantised_logits(dev, cf, dtype):
    th = voro.voro_cast_texels(cf.ds.texels, dtype)
    assert tuple(th.shape) == cf.tex.shape
    dsh = cf.ds.with_arrays(texels=th)
    voro.voro_prepare(dsh)
    sel = np.arange(0, len(cf.o), 7)
    deq = th.float().cpu().numpy().astype(np.float64)
    rgb_o, T_o, recs = render.render_rays(cf.scene.sites, cf.scene.density, deq, cf.o[sel],
                                          cf.d[sel], cf.tm[sel], starts=cf.start[sel],
                                          appearance=1)
    announce(f"full appearance {dtype} maps")
    si = torch.from_numpy(sel).to(dev)
    rgb, T = voro.voro_render_fwd(dsh, cf.O[si], cf.D[si], cf.TM[si], cf.S[si],
                                  voro.default_params(appearance=1))
    keep = np.array([not stop_degenerate(r, 1e-4) for r in recs])
    np.testing.assert_allclose(rgb.cpu().numpy()[keep], rgb_o[keep], atol=1e-4, rtol=0)


def test_appearance_must_match_the_texel_layout(dev, cf):
    with pytest.raises(voro.VoroError):
        voro.voro_render_fwd(cf.ds, cf.O[:64], cf.D[:64], cf.TM[:64], cf.S[:64],
                             voro.default_params(appearance=0))
