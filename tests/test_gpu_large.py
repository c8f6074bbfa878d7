"""GPU parity at the full scene sizes against the FP64 oracle's stored results.

* 2M sites on 20 ellipsoid surfaces, one 1280x840 interior view, FP32
  texels: 256 sampled rays (tests/golden/config3_rays.npz).
* 4M sites in the shell structure, binary16 texels, 8 mixed views in one
  launch (2 pinhole, 2 equidistant fisheye, 2 rolling shutter, 2 thin lens
  with 4 samples per pixel): 256 sampled pixels per view, 64 for the thin
  lens (tests/golden/config5_views.npz).

Both files are written by tests/golden/make_goldens.py from oracle/ alone
(brute force over all sites, FP64); each records a fingerprint of the scene
arrays, checked here against the scene these tests build.  Images come from
the launch configurations bench.py times (Morton-ordered cells, tuned launch
shapes); sequences from the oracle's own FP32 rays through the explicit-ray
entry point.  Tolerances: colour and transmittance 1e-4 on every ray but the
stop-degenerate ones, cell counts and sequences bit-exact on the
non-degenerate ones, gradients within 1e-4 of the largest component of
each kind (FP32 atomics in a different order), exact zeros elsewhere.
"""
import os

import numpy as np
import pytest
import torch

from paper_2608_17682_amd import autotune, synth, voro
from paper_2608_17682_amd.autograd import render_views
from helpers import scene_fingerprint, seq_hash

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    voro.lib()
    return torch.device("cuda:0")


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def load_golden(name):
    z = np.load(os.path.join(GOLDEN, name), allow_pickle=False)
    return {k: z[k] for k in z.files}


def morton_scene(scene, dev, tex_dtype=None):
    ds0 = voro.device_scene(scene, dev, tex_dtype=tex_dtype)
    ds, perm, inv = voro.voro_morton_reorder(ds0)
    del ds0
    voro.voro_prepare(ds)
    return ds, perm.cpu().numpy(), inv.cpu().numpy()


def dense_texel_grads(g):
    """The golden's sparse texel gradients as [C,R,R,3] over its touched cells."""
    res = int(g["grad_tex_res"])
    out = np.zeros((len(g["grad_cells"]) * res * res, 3))
    out[g["grad_tex_index"]] = g["grad_tex_rgb"]
    return out.reshape(-1, res, res, 3)


def assert_grads_match(g, gs, gd, gt, inv, what):
    """GPU gradients (Morton order, dense) against the oracle's touched cells."""
    ids = g["grad_cells"]
    k = inv[ids]
    want = {"sites": g["grad_sites"], "density": g["grad_density"],
            "texels": dense_texel_grads(g)}
    got = {"sites": gs[k], "density": gd[k], "texels": gt[k][..., :3]}
    for name in want:
        scale = max(1e-12, float(np.abs(want[name]).max()))
        err = float(np.abs(got[name] - want[name]).max())
        announce(f"{what} {name}: max err {err:.2e} of max |grad| {scale:.2e}")
        assert err <= 1e-4 * scale + 1e-6, (what, name, err, scale)
    mask = np.ones(len(gd), bool)
    mask[k] = False
    assert np.all(gd[mask] == 0) and np.all(gs[mask] == 0) and np.all(gt[mask] == 0), what
    assert np.all(gt[..., 3] == 0)


def check_sequences(ds, perm, inv, g, dev, params, what):
    """Explicit-ray walk of the oracle's FP32 rays: K and sequences bit-exact
    on the non-degenerate rays, colours within 1e-4 on the non-stop-degenerate."""
    R = len(g["o"])
    kmax = int(g["K"].max()) + 16
    O, D, TM = to_dev(g["o"], dev), to_dev(g["d"], dev), to_dev(g["tmax"], dev)
    S = to_dev(inv[g["start"]].astype(np.int32), dev)
    p = voro.voro_params.from_buffer_copy(params)
    p.max_record = kmax
    nsteps = torch.empty(R, dtype=torch.int32, device=dev)
    cells = torch.empty((R, kmax), dtype=torch.int32, device=dev)
    rgb, T = voro.voro_render_fwd(ds, O, D, TM, S, p, nsteps=nsteps, cells=cells)
    K, cells = nsteps.cpu().numpy(), cells.cpu().numpy()
    ok = ~g["degenerate"]
    assert ok.mean() > 0.9, ok.mean()
    assert np.array_equal(K[ok], g["K"][ok])
    mism = [r for r in np.nonzero(ok)[0] if seq_hash(perm[cells[r, :K[r]]]) != int(g["seq_hash"][r])]
    assert not mism, f"{what}: {len(mism)} sequences differ, first rays {mism[:5]}"
    sd = ~g["stop_degenerate"]
    assert np.abs(rgb.cpu().numpy() - g["rgb"])[sd].max() <= 1e-4
    assert np.abs(T.cpu().numpy() - g["T"])[sd].max() <= 1e-4
    announce(f"{what}: {ok.sum()} of {R} sequences equal (mean K {K.mean():.1f}, max {K.max()})")
    return rgb, T


# ------------------------------------------------------------------ 2M sites

class Case:
    pass


@pytest.fixture(scope="module")
def c3(dev):
    c = Case()
    c.g = load_golden("config3_rays.npz")
    announce("config3: 2M-site scene (built by a child process on a cache miss)")
    c.scene = synth.scene_cached("config3")
    assert scene_fingerprint(c.scene) == str(c.g["fingerprint"])
    c.cam = synth.config3_camera(c.scene)
    assert np.array_equal(c.cam.c2w, c.g["cam_c2w"])
    c.ds, c.perm, c.inv = morton_scene(c.scene, dev)
    c.pf = autotune.params_for(c.ds, [c.cam], "fwd")
    c.pb = autotune.params_for(c.ds, [c.cam], "bwd")
    return c


def test_config3_sequences_and_colours(dev, c3):
    announce("config3: explicit oracle rays, 256 sampled")
    check_sequences(c3.ds, c3.perm, c3.inv, c3.g, dev, c3.pf, "config3")


@pytest.mark.parametrize("cap", [0, 256])
def test_config3_adjoint_sampled_rays(dev, c3, cap):
    announce(f"config3: adjoint of the non-degenerate sampled rays (explicit rays, stored exits "
             f"{cap})")
    g = c3.g
    sel = ~g["degenerate"]
    O, D, TM = (to_dev(g[k][sel], dev) for k in ("o", "d", "tmax"))
    S = to_dev(c3.inv[g["start"][sel]].astype(np.int32), dev)
    trace = torch.empty((cap, O.shape[0], 2), dtype=torch.int32, device=dev) if cap else None
    rgb, T = voro.voro_render_fwd(c3.ds, O, D, TM, S, c3.pf, trace=trace)
    gs, gd, gt = voro.voro_render_bwd(c3.ds, O, D, TM, S, rgb, T, to_dev(g["g_rgb"][sel], dev),
                                      None, c3.pb, trace=trace)
    assert_grads_match(g, gs.cpu().numpy(), gd.cpu().numpy(), gt.cpu().numpy(), c3.inv,
                       "config3 explicit")


@pytest.mark.parametrize("stored_exits", [0, 256])
def test_config3_benchmark_autograd_step_matches_oracle(dev, c3, stored_exits):
    announce(f"config3: the benchmarked autograd render_views step (stored exits: "
             f"{stored_exits}), sampled pixels")
    g = c3.g
    ok = ~g["degenerate"]
    gimg = np.zeros((c3.cam.n_pixels, 3), np.float32)
    gimg[g["pixels"][ok]] = g["g_rgb"][ok]
    sites = c3.ds.sites.clone().requires_grad_(True)
    dens = c3.ds.density.clone().requires_grad_(True)
    tex = c3.ds.texels.clone().requires_grad_(True)
    rgb, T = render_views(sites, dens, tex, c3.ds.nbr_off, c3.ds.nbr_idx, [c3.cam], c3.pf, c3.pb,
                          stored_exits=stored_exits)
    sd = ~g["stop_degenerate"]
    px = g["pixels"]
    assert np.abs(rgb.detach().cpu().numpy()[px] - g["rgb"])[sd].max() <= 1e-4
    assert np.abs(T.detach().cpu().numpy()[px] - g["T"])[sd].max() <= 1e-4
    (rgb * to_dev(gimg, dev)).sum().backward()
    assert_grads_match(g, sites.grad.cpu().numpy(), dens.grad.cpu().numpy(),
                       tex.grad.cpu().numpy(), c3.inv, "config3 render_views")


def test_config3_full_frame_views_equals_explicit(dev, c3):
    announce("config3: full 1280x840 frame, tuned views launch vs explicit rays")
    rgb_v, T_v, _ = voro.voro_render_views_fwd(c3.ds, [c3.cam], c3.pf)
    O, D, TM = voro.voro_gen_rays([c3.cam], dev)
    S = voro.voro_locate_origins(c3.ds, O[:1]).expand(O.shape[0]).contiguous()
    rgb_e, T_e = voro.voro_render_fwd(c3.ds, O, D, TM, S, voro.default_params(img_w=1280))
    assert torch.equal(rgb_v, rgb_e) and torch.equal(T_v, T_e)


# ------------------------------------------------------------------ 4M sites

@pytest.fixture(scope="module")
def c5(dev):
    c = Case()
    c.g = load_golden("config5_views.npz")
    announce("config5: 4M-site scene (built by a child process on a cache miss)")
    c.scene = synth.scene_cached("config5")
    assert scene_fingerprint(c.scene) == str(c.g["fingerprint"])
    c.cams = synth.config5_cameras(1.0)
    c.ds, c.perm, c.inv = morton_scene(c.scene, dev, tex_dtype="float16")
    c.pf = autotune.params_for(c.ds, c.cams, "fwd")
    c.pb = autotune.params_for(c.ds, c.cams, "bwd")
    c.off = np.cumsum([0] + [cam.n_pixels for cam in c.cams])
    return c


def test_config5_sequences_and_colours(dev, c5):
    announce("config5: explicit oracle rays, 256 per view")
    check_sequences(c5.ds, c5.perm, c5.inv, c5.g, dev, c5.pf, "config5")


def test_config5_benchmark_launch_forward(dev, c5):
    announce("config5: 8 views, the benchmarked forward launch")
    g = c5.g
    rgb, T, _ = voro.voro_render_views_fwd(c5.ds, c5.cams, c5.pf)
    rgb, T = rgb.cpu().numpy(), T.cpu().numpy()
    checked = np.zeros(8, int)
    for v, p, r0, spp in zip(g["px_view"], g["px_pixel"], g["px_ray0"], g["px_spp"]):
        if g["stop_degenerate"][r0:r0 + spp].any():
            continue
        q = c5.off[v] + p
        assert np.abs(rgb[q] - g["rgb"][r0:r0 + spp].mean(0)).max() <= 1e-4, (v, p)
        assert abs(T[q] - g["T"][r0:r0 + spp].mean()) <= 1e-4, (v, p)
        checked[v] += 1
    announce(f"config5: pixels checked per view {checked.tolist()}")
    assert np.all(checked >= 0.9 * np.array([256, 256, 256, 256, 256, 256, 64, 64]))
    # fisheye pixels outside the image circle are empty
    assert T[c5.off[2]] == 1.0 and np.all(rgb[c5.off[2]] == 0)


@pytest.mark.parametrize("cap", [0, 256])
def test_config5_benchmark_launch_adjoint(dev, c5, cap):
    announce(f"config5: the benchmarked adjoint launch (stored exits: {cap} steps), upstream "
             "on the gradient pixels only")
    g = c5.g
    npx = int(c5.off[-1])
    g_all = synth.upstream(npx, 5, with_gT=False)[0]
    gimg = np.zeros((npx, 3), np.float32)
    for v, p, use in zip(g["px_view"], g["px_pixel"], g["px_grad"]):
        if use:
            gimg[c5.off[v] + p] = g_all[c5.off[v] + p]
    assert g["px_grad"].sum() >= 0.85 * (6 * 32 + 2 * 8)
    nr = sum(cam.n_rays for cam in c5.cams)
    trace = torch.empty((cap, nr, 2), dtype=torch.int32, device=dev) if cap else None
    rgb, T, ray = voro.voro_render_views_fwd(c5.ds, c5.cams, c5.pf, trace=trace)
    gs, gd, gt = voro.voro_render_views_bwd(c5.ds, c5.cams, rgb, T, ray, to_dev(gimg, dev), None,
                                            c5.pb, trace=trace)
    del trace
    assert_grads_match(g, gs.cpu().numpy(), gd.cpu().numpy(), gt.cpu().numpy(), c5.inv,
                       "config5 views")


def test_config5_persistent_views_adjoint_equals_explicit(dev, c5):
    announce("config5: views adjoint vs explicit-ray adjoint, all 7.3M rays")
    p = c5.pb
    npx = int(c5.off[-1])
    g_rgb = synth.upstream(npx, 5, with_gT=False)[0]
    st_v = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    rgb, T, ray_rgbT = voro.voro_render_views_fwd(c5.ds, c5.cams, c5.pf, stats=st_v)
    gv = voro.voro_render_views_bwd(c5.ds, c5.cams, rgb, T, ray_rgbT, to_dev(g_rgb, dev), None, p)
    O, D, TM = voro.voro_gen_rays(c5.cams, dev)
    centres = to_dev(np.array([cam.c2w[:, 3] for cam in c5.cams], np.float32), dev)
    cc = voro.voro_locate_origins(c5.ds, centres)
    nr = [cam.n_rays for cam in c5.cams]
    hint = torch.cat([cc[i:i + 1].expand(k) for i, k in enumerate(nr)]).contiguous()
    S = voro.voro_locate_origins(c5.ds, O, hint=hint)
    st_e = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    rgb_e, T_e = voro.voro_render_fwd(c5.ds, O, D, TM, S, voro.default_params(), stats=st_e)
    # the multi-view launch's per-ray results are the explicit path's, bit for
    # bit, and so are the walk statistics its workgroups gather
    assert torch.equal(rgb_e, ray_rgbT[:, :3].contiguous()) and torch.equal(T_e, ray_rgbT[:, 3])
    keep = [voro.STAT_NAMES.index(k) for k in ("rays", "steps", "degree_sum", "max_steps", "nan",
                                                "bad_start", "fp64_redecide", "skipped")]
    assert st_v[keep].tolist() == st_e[keep].tolist()
    gr = []
    off = 0
    for cam in c5.cams:
        gr.append(np.repeat(g_rgb[off:off + cam.n_pixels], cam.spp, 0) / cam.spp)
        off += cam.n_pixels
    ge = voro.voro_render_bwd(c5.ds, O, D, TM, S, rgb_e, T_e, to_dev(np.concatenate(gr), dev),
                              None, voro.default_params())
    for a, b, name in zip(gv, ge, ("sites", "density", "texels")):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.isfinite(a).all()
        assert np.abs(a - b).max() <= 1e-4 * max(1.0, np.abs(b).max()), name
