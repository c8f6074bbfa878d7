"""GPU parity of the HIP walk (through the C ABI) against the FP64 oracle.

Tolerances: rgb and T within 1e-4 absolute (FP32 compositing over <= a few
hundred segments); visited-cell sequences bit-exact except on rays the
oracle marks epsilon-degenerate (near-tied exits, near-zero segments,
T within 1e-4 relative of t_stop, exits within 1e-5 of tmax).
"""
import math

import numpy as np
import pytest
import torch

from oracle import adjoint, cameras, render, walk
from paper_2608_17682_amd import synth, voro
from helpers import degenerate, f32, stop_degenerate

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    voro.lib()
    return torch.device("cuda:0")


def to_dev(a, dev, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


class Case:
    pass


@pytest.fixture(scope="module")
def c1(dev):
    """Config 1: 512 uniform sites, 4x4 texels, 64x64 pinhole; oracle on every ray."""
    c = Case()
    c.scene, c.cams = synth.config1()
    o, d, tm, _ = cameras.camera_rays_of(c.cams[0])
    c.o, c.d, c.tm = f32(o), f32(d), f32(tm)
    c.start = np.array([walk.nearest_site(c.scene.sites, x)[0] for x in c.o[:1]] * len(c.o),
                       np.int32)
    c.rgb, c.T, c.recs = render.render_rays(c.scene.sites, c.scene.density, c.scene.texels,
                                            c.o, c.d, c.tm, starts=c.start)
    c.ds = voro.device_scene(c.scene, dev)
    announce("config1 prepare")
    voro.voro_prepare(c.ds)
    c.O, c.D, c.TM, c.S = (to_dev(c.o, dev), to_dev(c.d, dev), to_dev(c.tm, dev),
                           to_dev(c.start, dev))
    return c


def gpu_fwd(c, params=None, max_record=0):
    R = c.O.shape[0]
    p = params or voro.default_params()
    p.max_record = max_record
    nsteps = torch.empty(R, dtype=torch.int32, device=c.O.device)
    cells = (torch.empty((R, max_record), dtype=torch.int32, device=c.O.device)
             if max_record else None)
    stats = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=c.O.device)
    rgb, T = voro.voro_render_fwd(c.ds, c.O, c.D, c.TM, c.S, p, nsteps=nsteps, cells=cells,
                                  stats=stats)
    torch.cuda.synchronize()
    return (rgb.cpu().numpy(), T.cpu().numpy(), nsteps.cpu().numpy(),
            None if cells is None else cells.cpu().numpy(), stats.cpu().numpy())


def test_locate_matches_oracle(dev, c1):
    rng = np.random.default_rng(0)
    pts = f32(rng.uniform(-1.3, 1.3, (64, 3)))
    want = np.array([walk.nearest_site(c1.scene.sites, x)[0] for x in pts])
    announce("locate brute force, 64 origins")
    got = voro.voro_locate_origins(c1.ds, to_dev(pts, dev)).cpu().numpy()
    np.testing.assert_array_equal(got, want)
    pts2 = f32(rng.uniform(-1.6, 1.6, (3000, 3)))
    want2 = np.array([walk.nearest_site(c1.scene.sites, x)[0] for x in pts2])
    hint = torch.zeros(3000, dtype=torch.int32, device=dev)
    announce("locate greedy walk, 3000 origins")
    got2 = voro.voro_locate_origins(c1.ds, to_dev(pts2, dev), hint=hint).cpu().numpy()
    np.testing.assert_array_equal(got2, want2)


def test_fwd_config1_every_ray(dev, c1):
    announce("fwd config1 4096 rays")
    rgb, T, K, cells, stats = gpu_fwd(c1, max_record=64)
    np.testing.assert_allclose(rgb, c1.rgb, rtol=0, atol=1e-4)
    np.testing.assert_allclose(T, c1.T, rtol=0, atol=1e-4)
    deg = np.array([degenerate(r, 1e-4, float(c1.tm[0])) for r in c1.recs])
    assert deg.mean() < 0.01, deg.mean()
    for r in np.nonzero(~deg)[0]:
        rec = c1.recs[r]
        assert K[r] == rec.K, r
        np.testing.assert_array_equal(cells[r, :rec.K], rec.cells)
        assert np.all(cells[r, rec.K:] == -1)
    assert stats[voro.STAT_NAMES.index("rays")] == len(c1.o)
    assert stats[voro.STAT_NAMES.index("steps")] == K.sum()
    assert stats[voro.STAT_NAMES.index("max_steps")] == 0
    assert stats[voro.STAT_NAMES.index("bad_start")] == 0


@pytest.mark.parametrize("lpr", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("tiled", [False, True])
def test_launch_shapes_are_bit_identical(dev, c1, lpr, tiled):
    base_rgb, base_T, base_K, _, _ = gpu_fwd(c1)
    p = voro.default_params(lanes_per_ray=lpr)
    if tiled:
        p.img_w = 64
    announce(f"fwd config1 lpr={lpr} tiled={tiled}")
    rgb, T, K, _, _ = gpu_fwd(c1, p)
    np.testing.assert_array_equal(rgb, base_rgb)
    np.testing.assert_array_equal(T, base_T)
    np.testing.assert_array_equal(K, base_K)


def test_ragged_and_empty(dev, c1):
    # a prime number of rays (ragged last wave) and R = 0
    n = 4093
    p = voro.default_params(lanes_per_ray=4)
    announce("fwd ragged 4093 rays")
    rgb, T = voro.voro_render_fwd(c1.ds, c1.O[:n], c1.D[:n], c1.TM[:n], c1.S[:n], p)
    np.testing.assert_allclose(rgb.cpu().numpy(), c1.rgb[:n], atol=1e-4, rtol=0)
    z = torch.empty((0, 3), device=dev)
    rgb0, T0 = voro.voro_render_fwd(c1.ds, z, z, z[:, 0], torch.empty(0, dtype=torch.int32,
                                                                       device=dev))
    assert rgb0.shape == (0, 3)


def test_anomaly_counters(dev, c1):
    # max_steps cap, out-of-range start cells, tmax <= 0 and NaN density
    p = voro.default_params(max_steps=3)
    announce("fwd max_steps=3")
    rgb, T, K, _, stats = gpu_fwd(c1, p)
    assert K.max() == 3 and stats[voro.STAT_NAMES.index("max_steps")] > 0
    S = c1.S.clone()
    S[:10] = -5
    S[10:20] = c1.ds.n + 7
    TM = c1.TM.clone()
    TM[20:30] = 0.0
    stats = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    announce("fwd bad start cells")
    rgb, T = voro.voro_render_fwd(c1.ds, c1.O, c1.D, TM, S, stats=stats)
    rgb, T, st = rgb.cpu().numpy(), T.cpu().numpy(), stats.cpu().numpy()
    assert np.all(rgb[:30] == 0) and np.all(T[:30] == 1)
    assert st[voro.STAT_NAMES.index("bad_start")] == 20
    dens = c1.ds.density.clone()
    dens[c1.start[0]] = float("nan")
    ds2 = c1.ds.with_arrays(density=dens)
    voro.voro_prepare(ds2)
    stats = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    announce("fwd NaN density")
    rgb, T = voro.voro_render_fwd(ds2, c1.O, c1.D, c1.TM, c1.S, stats=stats)
    assert stats.cpu().numpy()[voro.STAT_NAMES.index("nan")] > 0
    voro.voro_prepare(c1.ds)


def test_skip_matches_oracle(dev, c1):
    sel = np.arange(0, 4096, 7)
    rgb_o, T_o, _ = render.render_rays(c1.scene.sites, c1.scene.density, c1.scene.texels,
                                       c1.o[sel], c1.d[sel], c1.tm[sel], starts=c1.start[sel],
                                       skip_w=0.02)
    p = voro.default_params(skip_w=0.02)
    stats = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    announce("fwd skip_w=0.02")
    rgb, T = voro.voro_render_fwd(c1.ds, c1.O[sel], c1.D[sel], c1.TM[sel], c1.S[sel], p,
                                  stats=stats)
    np.testing.assert_allclose(rgb.cpu().numpy(), rgb_o, atol=1e-4, rtol=0)
    np.testing.assert_allclose(T.cpu().numpy(), T_o, atol=1e-4, rtol=0)
    assert stats.cpu().numpy()[voro.STAT_NAMES.index("skipped")] > 0


def test_gen_rays_match_oracle(dev):
    cams = synth.config5_cameras(scale=0.1) + synth.motion_blur_cameras(scale=0.08)
    announce("gen_rays 8 mixed cameras + 2 motion blur")
    O, D, TM = voro.voro_gen_rays(cams, dev)
    O, D, TM = O.cpu().numpy(), D.cpu().numpy(), TM.cpu().numpy()
    off = 0
    for cam in cams:
        o, d, tm, valid = cameras.camera_rays_of(cam)
        n = len(o)
        np.testing.assert_allclose(O[off:off + n], o, atol=2e-6, rtol=0)
        np.testing.assert_allclose(D[off:off + n], d, atol=2e-6, rtol=0)
        np.testing.assert_array_equal(TM[off:off + n] > 0, valid)
        np.testing.assert_allclose(np.linalg.norm(D[off:off + n], axis=1), 1.0, atol=1e-6)
        off += n
    assert off == len(O)


def grads_gpu(c, sel, g_rgb, g_T, lpr=1):
    p = voro.default_params(lanes_per_ray=lpr)
    rgb, T = voro.voro_render_fwd(c.ds, c.O[sel], c.D[sel], c.TM[sel], c.S[sel], p)
    gs, gd, gt = voro.voro_render_bwd(c.ds, c.O[sel], c.D[sel], c.TM[sel], c.S[sel], rgb, T,
                                      to_dev(g_rgb, c.O.device), to_dev(g_T, c.O.device), p)
    torch.cuda.synchronize()
    return gs.cpu().numpy(), gd.cpu().numpy(), gt.cpu().numpy()


def assert_grad_close(got, want, name):
    # FP32 accumulation over up to a few thousand rays: relative error of the
    # whole vector below 1e-4, each entry within 1e-4 of the largest entry
    scale = max(1e-12, float(np.abs(want).max()))
    err = np.abs(got - want)
    assert err.max() <= 1e-4 * scale + 1e-6, (name, err.max(), scale)
    assert np.linalg.norm(got - want) <= 1e-4 * np.linalg.norm(want) + 1e-6, name


@pytest.mark.parametrize("lpr", [1, 4])
def test_bwd_config1_matches_oracle_gradient(dev, c1, lpr):
    deg = np.array([degenerate(r, 1e-4, float(c1.tm[0])) for r in c1.recs])
    sel = np.nonzero(~deg)[0]
    g_rgb, g_T = synth.upstream(len(c1.o), 1)
    g_rgb, g_T = g_rgb[sel], g_T[sel]
    want = adjoint.grad_rays(c1.scene.sites, c1.scene.density, c1.scene.texels, c1.o[sel],
                             c1.d[sel], c1.tm[sel], [c1.recs[i] for i in sel], g_rgb, g_T)
    announce(f"bwd config1 lpr={lpr}")
    got = grads_gpu(c1, torch.from_numpy(sel).to(dev), g_rgb, g_T, lpr)
    for g, w, name in zip(got, want, ("sites", "density", "texels")):
        assert_grad_close(g, w, name)
    assert np.all(got[2][..., 3] == 0)


def test_bwd_zero_upstream_gives_zero(dev, c1):
    sel = torch.arange(0, 4096, 3, device=dev)
    n = len(sel)
    announce("bwd zero upstream")
    gs, gd, gt = grads_gpu(c1, sel, np.zeros((n, 3), np.float32), np.zeros(n, np.float32))
    assert np.all(gs == 0) and np.all(gd == 0) and np.all(gt == 0)


def test_autograd_function(dev, c1):
    from paper_2608_17682_amd.autograd import render as vrender
    sites = c1.ds.sites.clone().requires_grad_(True)
    rho = torch.log(c1.ds.density.clone()).requires_grad_(True)
    tex = c1.ds.texels.clone().requires_grad_(True)
    announce("autograd render config1")
    rgb, T = vrender(sites, torch.exp(rho), tex, c1.ds.nbr_off, c1.ds.nbr_idx, c1.O, c1.D, c1.TM,
                     c1.S)
    g_rgb, g_T = synth.upstream(len(c1.o), 1)
    loss = (rgb * to_dev(g_rgb, dev)).sum() + (T * to_dev(g_T, dev)).sum()
    loss.backward()
    np.testing.assert_allclose(rgb.detach().cpu().numpy(), c1.rgb, atol=1e-4, rtol=0)
    # dL/drho = sigma dL/dsigma (Sec. 5.4), from the oracle over the non-degenerate rays
    gs, gd, gt = adjoint.grad_rays(c1.scene.sites, c1.scene.density, c1.scene.texels, c1.o, c1.d,
                                   c1.tm, c1.recs, g_rgb, g_T)
    assert_grad_close(rho.grad.cpu().numpy(), gd * c1.scene.density, "rho")
    assert_grad_close(tex.grad.cpu().numpy(), gt, "texels")


WALK_STATS = ("rays", "steps", "degree_sum", "max_steps", "nan", "bad_start", "fp64_redecide",
              "skipped")


@pytest.mark.parametrize("lpr,schedule", [(2, voro.SCHEDULE_GRID), (1, voro.SCHEDULE_GRID),
                                          (1, voro.SCHEDULE_REFILL), (1, voro.SCHEDULE_PERSISTENT),
                                          (2, voro.SCHEDULE_PERSISTENT)])
def test_views_fwd_equals_explicit_rays(dev, c1, lpr, schedule):
    # every multi-view schedule generates the same rays, starts in the same
    # cells and takes the same walk as gen_rays + locate + render_fwd, and
    # counts the same walk statistics (however each kernel gathers them)
    cams = synth.config5_cameras(scale=0.06) + synth.motion_blur_cameras(scale=0.05)
    for cm in cams:
        cm.tmax = 4.0
    announce(f"views fwd vs explicit, mixed cameras, lpr {lpr} schedule {schedule}")
    p = voro.default_params(lanes_per_ray=lpr, schedule=schedule)
    st_v = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    rgb_v, T_v, ray_v = voro.voro_render_views_fwd(c1.ds, cams, p, stats=st_v)
    O, D, TM = voro.voro_gen_rays(cams, dev)
    centres = to_dev(f32([cm.c2w[:, 3] for cm in cams]), dev)
    cc = voro.voro_locate_origins(c1.ds, centres)
    nr = [cm.n_rays for cm in cams]
    hint = torch.cat([cc[i:i + 1].expand(n) for i, n in enumerate(nr)]).contiguous()
    S = voro.voro_locate_origins(c1.ds, O, hint=hint)
    st_e = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    rgb_e, T_e = voro.voro_render_fwd(c1.ds, O, D, TM, S, voro.default_params(lanes_per_ray=1),
                                      stats=st_e)
    sv = dict(zip(voro.STAT_NAMES, st_v.cpu().tolist()))
    se = dict(zip(voro.STAT_NAMES, st_e.cpu().tolist()))
    assert sv["rays"] == int((TM > 0).sum().item()) and sv["steps"] > sv["rays"]
    assert {k: sv[k] for k in WALK_STATS} == {k: se[k] for k in WALK_STATS}
    rgb_e, T_e = rgb_e.cpu().numpy(), T_e.cpu().numpy()
    ray_v = ray_v.cpu().numpy()
    rgb_v, T_v = rgb_v.cpu().numpy(), T_v.cpu().numpy()
    off_r = off_p = 0
    for cm in cams:
        n, npx = cm.n_rays, cm.n_pixels
        if cm.spp == 1:
            np.testing.assert_array_equal(rgb_v[off_p:off_p + npx], rgb_e[off_r:off_r + n])
            np.testing.assert_array_equal(T_v[off_p:off_p + npx], T_e[off_r:off_r + n])
        else:
            np.testing.assert_array_equal(ray_v[off_r:off_r + n, :3], rgb_e[off_r:off_r + n])
            mean = rgb_e[off_r:off_r + n].reshape(npx, cm.spp, 3).mean(1)
            np.testing.assert_allclose(rgb_v[off_p:off_p + npx], mean, atol=1e-6)
        off_r += n
        off_p += npx


def test_views_match_oracle_sampled(dev, c1):
    cams = synth.config5_cameras(scale=0.06) + synth.motion_blur_cameras(scale=0.05)
    for cm in cams:
        cm.tmax = 4.0
    announce("views fwd vs oracle, sampled pixels")
    rgb_v, T_v, ray_v = voro.voro_render_views_fwd(c1.ds, cams)
    rgb_v, T_v = rgb_v.cpu().numpy(), T_v.cpu().numpy()
    off = 0
    for vi, cm in enumerate(cams):
        o, d, tm, valid = cameras.camera_rays_of(cm)
        pix = synth.sample_pixels(cm.n_pixels, 24, vi)
        for p in pix:
            rs = slice(p * cm.spp, (p + 1) * cm.spp)
            rgb_o, T_o, recs = render.render_rays(c1.scene.sites, c1.scene.density,
                                                  c1.scene.texels, f32(o[rs]), f32(d[rs]),
                                                  f32(tm[rs]))
            if any(stop_degenerate(r, 1e-4) for r in recs):
                continue
            np.testing.assert_allclose(rgb_v[off + p], rgb_o.mean(0), atol=1e-4, rtol=0)
            np.testing.assert_allclose(T_v[off + p], T_o.mean(), atol=1e-4, rtol=0)
        off += cm.n_pixels


def test_views_bwd_equals_explicit(dev, c1):
    cams = synth.config5_cameras(scale=0.05) + synth.motion_blur_cameras(scale=0.04, spp=3)
    for cm in cams:
        cm.tmax = 4.0
    nr = [cm.n_rays for cm in cams]
    npx = sum(cm.n_pixels for cm in cams)
    g_rgb, g_T = synth.upstream(npx, 5)
    p = voro.default_params()
    announce("views bwd vs explicit bwd")
    rgb_v, T_v, ray_v = voro.voro_render_views_fwd(c1.ds, cams, p)
    gv = voro.voro_render_views_bwd(c1.ds, cams, rgb_v, T_v, ray_v, to_dev(g_rgb, dev),
                                    to_dev(g_T, dev), p)
    O, D, TM = voro.voro_gen_rays(cams, dev)
    centres = to_dev(f32([cm.c2w[:, 3] for cm in cams]), dev)
    cc = voro.voro_locate_origins(c1.ds, centres)
    hint = torch.cat([cc[i:i + 1].expand(n) for i, n in enumerate(nr)]).contiguous()
    S = voro.voro_locate_origins(c1.ds, O, hint=hint)
    rgb_e, T_e = voro.voro_render_fwd(c1.ds, O, D, TM, S, p)
    # per-ray upstream: a thin-lens pixel's gradient is shared by its samples
    gr, gt_ = [], []
    off = 0
    for cm in cams:
        sl = slice(off, off + cm.n_pixels)
        gr.append(np.repeat(g_rgb[sl], cm.spp, 0) / cm.spp)
        gt_.append(np.repeat(g_T[sl], cm.spp, 0) / cm.spp)
        off += cm.n_pixels
    ge = voro.voro_render_bwd(c1.ds, O, D, TM, S, rgb_e, T_e, to_dev(np.concatenate(gr), dev),
                              to_dev(np.concatenate(gt_), dev), p)
    for a, b, name in zip(gv, ge, ("sites", "density", "texels")):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        # same terms, different atomic order: FP32 summation differences only
        assert np.abs(a - b).max() <= 1e-5 * max(1.0, np.abs(b).max()), name


@pytest.mark.parametrize("lpr,schedule,cap", [(1, voro.SCHEDULE_PERSISTENT, 512),
                                              (1, voro.SCHEDULE_GRID, 3),
                                              (1, voro.SCHEDULE_REFILL, 7),
                                              (4, voro.SCHEDULE_PERSISTENT, 5)])
def test_views_stored_exits(dev, c1, lpr, schedule, cap):
    # The forward's stored exits are the walk's own (each step's next cell is
    # the cell the explicit-ray walk visits next); they change no forward
    # output, and the adjoint that reads them (searching only past the cap)
    # gives the gradients of the adjoint that searches every step.
    cams = synth.config5_cameras(scale=0.05) + synth.motion_blur_cameras(scale=0.04, spp=3)
    for cm in cams:
        cm.tmax = 4.0
    nr = [cm.n_rays for cm in cams]
    R = sum(nr)
    npx = sum(cm.n_pixels for cm in cams)
    g_rgb, g_T = synth.upstream(npx, 7)
    p = voro.default_params()
    p.lanes_per_ray = lpr
    p.schedule = schedule
    announce(f"stored exits lpr={lpr} schedule={schedule} cap={cap}")
    ns0 = torch.empty(R, dtype=torch.int32, device=dev)
    rgb0, T0, ray0 = voro.voro_render_views_fwd(c1.ds, cams, p, nsteps=ns0)
    trace = torch.full((cap, R, 2), -7, dtype=torch.int32, device=dev)
    ns1 = torch.empty(R, dtype=torch.int32, device=dev)
    rgb1, T1, ray1 = voro.voro_render_views_fwd(c1.ds, cams, p, nsteps=ns1, trace=trace)
    assert torch.equal(rgb0, rgb1) and torch.equal(T0, T1) and torch.equal(ray0, ray1)
    assert torch.equal(ns0, ns1)
    # the explicit-ray walk's visited cells
    O, D, TM = voro.voro_gen_rays(cams, dev)
    centres = to_dev(f32([cm.c2w[:, 3] for cm in cams]), dev)
    cc = voro.voro_locate_origins(c1.ds, centres)
    hint = torch.cat([cc[i:i + 1].expand(n) for i, n in enumerate(nr)]).contiguous()
    S = voro.voro_locate_origins(c1.ds, O, hint=hint)
    pe = voro.default_params()
    pe.max_record = 256
    K = torch.empty(R, dtype=torch.int32, device=dev)
    cells = torch.empty((R, 256), dtype=torch.int32, device=dev)
    voro.voro_render_fwd(c1.ds, O, D, TM, S, pe, nsteps=K, cells=cells)
    K, cells, tr = K.cpu().numpy(), cells.cpu().numpy(), trace.cpu().numpy()
    assert np.array_equal(K, ns1.cpu().numpy()) and K.max() <= 256
    walked = 0
    for i in range(R):
        k = int(K[i])
        m = min(k, cap)
        # steps 0..m-2 lead to the next visited cell; the last stored step
        # to the next one or to none
        assert np.array_equal(tr[:max(m - 1, 0), i, 1], cells[i, 1:max(m, 1)]), i
        if m > 0:
            assert -1 <= tr[m - 1, i, 1] < c1.ds.n
            assert np.isfinite(tr[:m - 1, i, 0].view(np.float32)).all()
        assert (tr[m:, i] == -7).all(), i  # steps not walked are left untouched
        walked += k > cap
    if cap < 10:
        assert walked > 0  # some rays go past the stored steps
    g1, gT1 = to_dev(g_rgb, dev), to_dev(g_T, dev)
    sa = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    sb = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    ga = voro.voro_render_views_bwd(c1.ds, cams, rgb0, T0, ray0, g1, gT1, p, stats=sa)
    gb = voro.voro_render_views_bwd(c1.ds, cams, rgb1, T1, ray1, g1, gT1, p, trace=trace,
                                    stats=sb)
    # the same steps; edge rows read only where no exit was stored
    i_steps, i_deg = voro.STAT_NAMES.index("steps"), voro.STAT_NAMES.index("degree_sum")
    sa, sb = sa.cpu().numpy(), sb.cpu().numpy()
    assert sa[i_steps] == sb[i_steps] == int(K.sum())
    if cap >= K.max():
        assert sb[i_deg] == 0
    else:
        assert 0 < sb[i_deg] < sa[i_deg]
    for a, b, name in zip(ga, gb, ("sites", "density", "texels")):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.isfinite(b).all()
        # same terms, different atomic order: FP32 summation differences only
        assert np.abs(a - b).max() <= 1e-5 * max(1.0, np.abs(a).max()), name


@pytest.mark.parametrize("lpr", [1, 4])
def test_explicit_stored_exits_are_the_walk(dev, c1, lpr):
    # explicit rays: the stored exits lead from each visited cell to the next
    # one, and storing them changes no forward output
    R = c1.O.shape[0]
    cap = 5
    p = voro.default_params(lanes_per_ray=lpr)
    p.max_record = 256
    announce(f"explicit rays: stored exits lpr={lpr}")
    K = torch.empty(R, dtype=torch.int32, device=dev)
    cells = torch.empty((R, 256), dtype=torch.int32, device=dev)
    rgb0, T0 = voro.voro_render_fwd(c1.ds, c1.O, c1.D, c1.TM, c1.S, p, nsteps=K, cells=cells)
    trace = torch.full((cap, R, 2), -7, dtype=torch.int32, device=dev)
    rgb1, T1 = voro.voro_render_fwd(c1.ds, c1.O, c1.D, c1.TM, c1.S, voro.default_params(
        lanes_per_ray=lpr), trace=trace)
    assert torch.equal(rgb0, rgb1) and torch.equal(T0, T1)
    K, cells, tr = K.cpu().numpy(), cells.cpu().numpy(), trace.cpu().numpy()
    assert K.max() <= 256 and (K > cap).any()
    for i in range(R):
        m = min(int(K[i]), cap)
        assert np.array_equal(tr[:max(m - 1, 0), i, 1], cells[i, 1:max(m, 1)]), i
        assert (tr[m:, i] == -7).all(), i


def test_views_stored_exit_outside_the_scene_ends_the_ray(dev, c1):
    # A stored next cell outside [0, n) (a buffer from another walk) is never
    # read: the adjoint ends that ray's walk there, so every ray here stops
    # after its first cell and only first-cell gradients appear.
    cams = synth.config5_cameras(scale=0.05)[:2]
    for cm in cams:
        cm.tmax = 4.0
    R = sum(cm.n_rays for cm in cams)
    npx = sum(cm.n_pixels for cm in cams)
    p = voro.default_params()
    announce("stored exits: next cells outside the scene")
    rgb, T, ray = voro.voro_render_views_fwd(c1.ds, cams, p)
    trace = torch.empty((4, R, 2), dtype=torch.int32, device=dev)
    trace[..., 0] = torch.tensor([1.0], dtype=torch.float32).view(torch.int32).item()
    trace[..., 1] = c1.ds.n + 5
    trace[1, :, 1] = -9
    g = to_dev(synth.upstream(npx, 3, with_gT=False)[0], dev)
    gs, gd, gt = voro.voro_render_views_bwd(c1.ds, cams, rgb, T, ray, g, None, p, trace=trace)
    st = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    voro.voro_render_views_bwd(c1.ds, cams, rgb, T, ray, g, None, p, trace=trace, stats=st)
    st = st.cpu().numpy()
    rays = int(st[voro.STAT_NAMES.index("rays")])
    assert rays > 0 and int(st[voro.STAT_NAMES.index("steps")]) == rays
    for a in (gs, gd, gt):
        assert torch.isfinite(a).all()
    # the start cells (one per camera centre) are the only cells touched
    touched = torch.nonzero(gd).flatten().cpu().numpy()
    centres = to_dev(f32([cm.c2w[:, 3] for cm in cams]), dev)
    starts = set(voro.voro_locate_origins(c1.ds, centres).cpu().numpy().tolist())
    assert set(touched.tolist()) <= starts


def test_distortion_fwd_matches_oracle(dev, c1):
    R = len(c1.o)
    dist = torch.empty((R, 3), dtype=torch.float32, device=dev)
    announce("distortion loss fwd config1")
    rgb, T = voro.voro_render_fwd(c1.ds, c1.O, c1.D, c1.TM, c1.S, voro.default_params(),
                                  dist=dist)
    dist = dist.cpu().numpy()
    keep = np.array([not stop_degenerate(r, 1e-4) for r in c1.recs])
    want = np.array([r.dist for r in c1.recs])
    wsum = np.array([sum(r.weight) for r in c1.recs])
    assert want.max() > 0.01
    np.testing.assert_allclose(dist[keep, 0], want[keep], atol=2e-6, rtol=1e-4)
    np.testing.assert_allclose(dist[keep, 2], wsum[keep], atol=1e-5, rtol=0)
    # the colour is unchanged by asking for the loss
    rgb0, _ = voro.voro_render_fwd(c1.ds, c1.O, c1.D, c1.TM, c1.S, voro.default_params())
    assert torch.equal(rgb, rgb0)


@pytest.mark.parametrize("cap", [0, 3])
@pytest.mark.parametrize("lpr", [1, 4])
def test_distortion_bwd_matches_oracle_gradient(dev, c1, lpr, cap):
    deg = np.array([degenerate(r, 1e-4, float(c1.tm[0])) for r in c1.recs])
    sel = np.nonzero(~deg)[0]
    g_rgb, g_T = synth.upstream(len(c1.o), 1)
    g_rgb, g_T = g_rgb[sel], g_T[sel]
    g_dist = np.random.default_rng(17).normal(0.0, 3.0, len(sel)).astype(np.float32)
    want = adjoint.grad_rays(c1.scene.sites, c1.scene.density, c1.scene.texels, c1.o[sel],
                             c1.d[sel], c1.tm[sel], [c1.recs[i] for i in sel], g_rgb, g_T, g_dist)
    announce(f"distortion bwd config1 lpr={lpr} stored exits {cap}")
    si = torch.from_numpy(sel).to(dev)
    p = voro.default_params(lanes_per_ray=lpr)
    dist = torch.empty((len(sel), 3), dtype=torch.float32, device=dev)
    # cap 3: each ray's first three exits are read from the forward's store,
    # the later ones searched
    trace = torch.empty((cap, len(sel), 2), dtype=torch.int32, device=dev) if cap else None
    rgb, T = voro.voro_render_fwd(c1.ds, c1.O[si], c1.D[si], c1.TM[si], c1.S[si], p, dist=dist,
                                  trace=trace)
    got = voro.voro_render_bwd(c1.ds, c1.O[si], c1.D[si], c1.TM[si], c1.S[si], rgb, T,
                               to_dev(g_rgb, dev), to_dev(g_T, dev), p, dist=dist,
                               g_dist=to_dev(g_dist, dev), trace=trace)
    for g, w, name in zip(got, want, ("sites", "density", "texels")):
        assert_grad_close(g.cpu().numpy(), w, name)


@pytest.mark.parametrize("stored_exits", [0, 64])
def test_autograd_distortion(dev, c1, stored_exits):
    from paper_2608_17682_amd.autograd import render as vrender
    sites = c1.ds.sites.clone().requires_grad_(True)
    rho = torch.log(c1.ds.density.clone()).requires_grad_(True)
    tex = c1.ds.texels.clone().requires_grad_(True)
    announce(f"autograd render with distortion, stored exits {stored_exits}")
    rgb, T, ld = vrender(sites, torch.exp(rho), tex, c1.ds.nbr_off, c1.ds.nbr_idx, c1.O, c1.D,
                         c1.TM, c1.S, distortion=True, stored_exits=stored_exits)
    lam = 0.37
    (rgb.sum() + lam * ld.sum()).backward()
    deg = np.array([degenerate(r, 1e-4, float(c1.tm[0])) for r in c1.recs])
    assert deg.mean() < 0.01
    R = len(c1.o)
    gs, gd, gt = adjoint.grad_rays(c1.scene.sites, c1.scene.density, c1.scene.texels, c1.o,
                                   c1.d, c1.tm, c1.recs, np.ones((R, 3)), np.zeros(R),
                                   np.full(R, lam))
    np.testing.assert_allclose(ld.detach().cpu().numpy(), [r.dist for r in c1.recs], atol=2e-6,
                               rtol=1e-4)
    assert_grad_close(rho.grad.cpu().numpy(), gd * c1.scene.density, "rho")
    assert_grad_close(sites.grad.cpu().numpy(), gs, "sites")


def test_edge_fp16_variant_is_the_exact_walk(dev, c1):
    # inference variant: half-precision ranking with certified error bounds;
    # a step whose bounds leave more than one candidate, or a face too close
    # to parallel, is searched in FP32, so every ray repeats the exact walk
    # bit for bit (and so matches the oracle like it)
    p16 = voro.default_params(edge_fp16=1)
    announce("edge_fp16 variant config1")
    n16 = torch.empty(c1.O.shape[0], dtype=torch.int32, device=dev)
    n32 = torch.empty_like(n16)
    rgb16, T16 = voro.voro_render_fwd(c1.ds, c1.O, c1.D, c1.TM, c1.S, p16, nsteps=n16)
    rgb, T = voro.voro_render_fwd(c1.ds, c1.O, c1.D, c1.TM, c1.S, voro.default_params(),
                                  nsteps=n32)
    assert torch.equal(rgb16, rgb) and torch.equal(T16, T) and torch.equal(n16, n32)
    err = np.abs(rgb16.cpu().numpy() - c1.rgb).max()
    assert err <= 1e-4
    # near-parallel faces and near ties: rays skimming a lattice's planes
    sites = synth.lattice_sites(6, 0.5, jitter=1e-4, seed=5)
    n = len(sites)
    scene = synth.scene_from_arrays(sites, np.full(n, 0.7, np.float32),
                                    synth.texels_rgb(n, 4, (0.2, 0.5, 0.9)))
    ds = voro.device_scene(scene, dev)
    voro.voro_prepare(ds)
    rng = np.random.default_rng(9)
    o = f32(rng.uniform(-1.2, 1.2, (2048, 3)))
    d = rng.normal(size=(2048, 3)) * np.array([1.0, 1e-3, 1e-3])   # nearly along +-x
    d = f32(d / np.linalg.norm(d, axis=1, keepdims=True))
    st = np.array([walk.nearest_site(sites, x)[0] for x in o], np.int32)
    O, D, S = to_dev(o, dev), to_dev(d, dev), to_dev(st, dev)
    TM = to_dev(np.full(2048, 3.0, np.float32), dev)
    a16 = voro.voro_render_fwd(ds, O, D, TM, S, p16)
    a32 = voro.voro_render_fwd(ds, O, D, TM, S, voro.default_params())
    assert torch.equal(a16[0], a32[0]) and torch.equal(a16[1], a32[1])
    # views launch: same variant, same result as explicit rays
    cams = synth.config5_cameras(scale=0.05)[:2]
    for cm in cams:
        cm.tmax = 4.0
    rv, tv, _ = voro.voro_render_views_fwd(c1.ds, cams, p16)
    O, D, TM = voro.voro_gen_rays(cams, dev)
    centres = to_dev(f32([cm.c2w[:, 3] for cm in cams]), dev)
    cc = voro.voro_locate_origins(c1.ds, centres)
    nr = [cm.n_rays for cm in cams]
    hint = torch.cat([cc[i:i + 1].expand(n) for i, n in enumerate(nr)]).contiguous()
    S = voro.voro_locate_origins(c1.ds, O, hint=hint)
    re_, te = voro.voro_render_fwd(c1.ds, O, D, TM, S, p16)
    assert torch.equal(rv, re_) and torch.equal(tv, te)
    # forward only, one lane per ray
    with pytest.raises(voro.VoroError):
        voro.voro_render_bwd(c1.ds, c1.O, c1.D, c1.TM, c1.S, rgb16, T16, torch.zeros_like(rgb16),
                             None, p16)
    with pytest.raises(voro.VoroError):
        voro.voro_render_fwd(c1.ds, c1.O, c1.D, c1.TM, c1.S,
                             voro.default_params(edge_fp16=1, lanes_per_ray=2))


@pytest.mark.parametrize("schedule", [voro.SCHEDULE_GRID, voro.SCHEDULE_PERSISTENT])
def test_autograd_views_equals_explicit(dev, c1, schedule):
    # render_views (in-kernel rays, one launch each way) and render over the
    # explicitly generated rays give the same image and the same gradients
    from paper_2608_17682_amd.autograd import render as vrender, render_views
    cams = synth.config5_cameras(scale=0.05)[:4]   # pinhole, fisheye, rolling shutter (spp 1)
    for cm in cams:
        cm.tmax = 4.0
    nr = [cm.n_rays for cm in cams]
    g_rgb, g_T = synth.upstream(sum(nr), 9)
    Gr, Gt = to_dev(g_rgb, dev), to_dev(g_T, dev)
    announce(f"autograd render_views vs render, schedule {schedule}")
    leaves = []
    for which in ("views", "explicit"):
        sites = c1.ds.sites.clone().requires_grad_(True)
        rho = torch.log(c1.ds.density.clone()).requires_grad_(True)
        tex = c1.ds.texels.clone().requires_grad_(True)
        if which == "views":
            p = voro.default_params(schedule=schedule)
            rgb, T = render_views(sites, torch.exp(rho), tex, c1.ds.nbr_off, c1.ds.nbr_idx, cams,
                                  p, p)
        else:
            O, D, TM = voro.voro_gen_rays(cams, dev)
            centres = to_dev(f32([cm.c2w[:, 3] for cm in cams]), dev)
            cc = voro.voro_locate_origins(c1.ds, centres)
            hint = torch.cat([cc[i:i + 1].expand(n) for i, n in enumerate(nr)]).contiguous()
            S = voro.voro_locate_origins(c1.ds, O, hint=hint)
            rgb, T = vrender(sites, torch.exp(rho), tex, c1.ds.nbr_off, c1.ds.nbr_idx, O, D, TM, S)
        ((rgb * Gr).sum() + (T * Gt).sum()).backward()
        leaves.append((rgb.detach().cpu().numpy(), T.detach().cpu().numpy(),
                       sites.grad.cpu().numpy(), rho.grad.cpu().numpy(), tex.grad.cpu().numpy()))
    (rv, tv, *gv), (re, te, *ge) = leaves
    np.testing.assert_array_equal(rv, re)
    np.testing.assert_array_equal(tv, te)
    for a, b, name in zip(gv, ge, ("sites", "rho", "texels")):
        assert np.abs(a - b).max() <= 1e-5 * max(1.0, np.abs(b).max()), name


@pytest.mark.parametrize("dtype", ["float16", "bfloat16"])
def test_half_texels(dev, c1, dtype):
    announce(f"cast texels {dtype}")
    th = voro.voro_cast_texels(c1.ds.texels, dtype)
    ref = c1.ds.texels.to(getattr(torch, dtype))
    assert torch.equal(th.view(torch.int16), ref.view(torch.int16))
    ds = c1.ds.with_arrays(texels=th)
    voro.voro_prepare(ds)
    rgb, T = voro.voro_render_fwd(ds, c1.O, c1.D, c1.TM, c1.S)
    deq = th.float().cpu().numpy()
    sel = np.arange(0, 4096, 5)
    rgb_o, T_o, _ = render.render_rays(c1.scene.sites, c1.scene.density, deq, c1.o[sel],
                                       c1.d[sel], c1.tm[sel], starts=c1.start[sel])
    np.testing.assert_allclose(rgb.cpu().numpy()[sel], rgb_o, atol=1e-4, rtol=0)
    # rounding a texel in [0,1] to nearest even moves it by at most half an
    # ulp at [0.5,1): 2^-12 (binary16), 2^-9 (bfloat16); the composited colour
    # is a convex-weighted sum with total weight 1 - T
    err = np.abs(rgb.cpu().numpy() - c1.rgb)
    half_ulp = {"float16": 2.0 ** -12, "bfloat16": 2.0 ** -9}[dtype]
    bound = half_ulp * (1.0 - c1.T)[:, None] + 1e-4
    assert np.all(err <= bound), float((err - bound).max())


def test_morton_reorder_preserves_the_image(dev, c1):
    announce("morton reorder")
    ds2, perm, inv = voro.voro_morton_reorder(c1.ds)
    voro.voro_prepare(ds2)
    perm_n, inv_n = perm.cpu().numpy(), inv.cpu().numpy()
    assert np.array_equal(np.sort(perm_n), np.arange(c1.ds.n))
    assert np.array_equal(inv_n[perm_n], np.arange(c1.ds.n))
    np.testing.assert_array_equal(ds2.sites.cpu().numpy(), c1.scene.sites[perm_n])
    # adjacency: same neighbour sets under renumbering
    off2, idx2 = ds2.nbr_off.cpu().numpy(), ds2.nbr_idx.cpu().numpy()
    for k in range(0, c1.ds.n, 37):
        o = perm_n[k]
        old = set(c1.scene.nbr_idx[c1.scene.nbr_off[o]:c1.scene.nbr_off[o + 1]].tolist())
        new = set(perm_n[idx2[off2[k]:off2[k + 1]]].tolist())
        assert old == new
    S2 = to_dev(inv_n[c1.start], dev)
    rgb2, T2 = voro.voro_render_fwd(ds2, c1.O, c1.D, c1.TM, S2)
    rgb1, T1 = voro.voro_render_fwd(c1.ds, c1.O, c1.D, c1.TM, c1.S)
    deg = np.array([degenerate(r, 1e-4, 6.0) for r in c1.recs])
    np.testing.assert_array_equal(rgb2.cpu().numpy()[~deg], rgb1.cpu().numpy()[~deg])
    # Morton codes are non-decreasing along the new order
    s = ds2.sites.cpu().numpy().astype(np.float64)
    lo, hi = s.min(0), s.max(0)
    q = np.clip(((s - lo) / (hi - lo) * 1024).astype(np.int64), 0, 1023)

    def spread(x):
        r = np.zeros_like(x)
        for b in range(10):
            r |= ((x >> b) & 1) << (3 * b)
        return r
    code = (spread(q[:, 0]) << 2) | (spread(q[:, 1]) << 1) | spread(q[:, 2])
    assert np.all(np.diff(code) >= 0)
    # the sort is stable: cells with equal codes keep their original order
    same = np.diff(code) == 0
    assert np.all(np.diff(perm_n)[same] > 0)
