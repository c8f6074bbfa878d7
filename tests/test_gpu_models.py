"""GPU parity of the full appearance model and the SH comparison model on the
100k-site shell scene, through the multi-view launch.

Scene: the shell scene of config 2 (100k sites), with seeded surface + view
logit maps for the full model (Sec. 5.1-5.2) and seeded degree-3 SH
coefficients (Sec. 3.3), Morton-ordered.  Expected values: the FP64 oracle's
(tests/golden/config2_models.npz, written by tests/golden/make_goldens.py from
oracle/ only) on the 64x64 centre crop of pose 0.

* Forward, both models, grid and persistent schedules: colour and
  transmittance within 1e-4 on every crop ray but the stop-degenerate ones.
* Full-model adjoint over the whole 800x800 frame with the upstream gradient
  on the crop's centre 32x32 block only (its non-degenerate rays): 1015 rays
  whose records land on 327 cells, so the wave merge and the workgroup table
  see heavy contention.  Site, density and both maps' texel gradients within
  1e-4 of the largest of each kind (plus 1e-6), exact zeros elsewhere.
"""
import os

import numpy as np
import pytest
import torch

from paper_2608_17682_amd import synth, voro
from helpers import scene_fingerprint

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config2_models.npz")
SCHEDULES = [voro.SCHEDULE_GRID, voro.SCHEDULE_PERSISTENT]


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


class Case:
    pass


@pytest.fixture(scope="module")
def cm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    voro.lib()
    dev = torch.device("cuda:0")
    c = Case()
    z = np.load(GOLDEN, allow_pickle=False)
    c.g = {k: z[k] for k in z.files}
    announce("models: 100k-site shell scene, full-model maps and SH coefficients")
    scene, cams = synth.config2()
    assert scene_fingerprint(scene) == str(c.g["fingerprint"]), "scene differs from the golden's"
    c.cam = cams[0]
    c.dev = dev
    c.scenes = {}
    for name, tex in (("full", synth.full_texels(scene.n, scene.tex_res, seed=2)),
                      ("sh", synth.sh_coeffs(scene.n, seed=2))):
        ds0 = voro.DeviceScene(to_dev(scene.sites, dev), to_dev(scene.density, dev),
                               to_dev(scene.nbr_off, dev), to_dev(scene.nbr_idx, dev),
                               to_dev(tex, dev))
        ds, perm, inv = voro.voro_morton_reorder(ds0)
        voro.voro_prepare(ds)
        c.scenes[name] = (ds, inv.cpu().numpy())
    return c


def crop(c, img):
    return img.cpu().numpy()[c.g["pixels"]]


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("model", ["full", "sh"])
def test_models_forward_match_oracle(cm, model, schedule):
    announce(f"models: {model} forward, schedule {schedule}")
    ds, _ = cm.scenes[model]
    app = 1 if model == "full" else 2
    p = voro.default_params(appearance=app, schedule=schedule)
    rgb, T, _ = voro.voro_render_views_fwd(ds, [cm.cam], p)
    g = cm.g
    ok = ~g["stop_degenerate"]
    want = g["rgb"] if model == "full" else g["rgb_sh"]
    e_rgb = np.abs(crop(cm, rgb) - want)[ok]
    e_T = np.abs(crop(cm, T) - g["T"])[ok]
    announce(f"models {model}: max |rgb err| {e_rgb.max():.2e}, max |T err| {e_T.max():.2e} "
             f"over {ok.sum()} rays")
    assert ok.mean() > 0.99
    assert e_rgb.max() <= 1e-4 and e_T.max() <= 1e-4


def dense_texel_grads(g):
    """The golden's sparse texel gradients as [C, maps, R, R, 3] over its touched cells."""
    res, maps = int(g["grad_tex_res"]), int(g["grad_tex_maps"])
    out = np.zeros((len(g["grad_cells"]) * maps * res * res, 3))
    out[g["grad_tex_index"]] = g["grad_tex_rgb"]
    return out.reshape(-1, maps, res, res, 3)


@pytest.mark.parametrize("cap", [0, 256])
@pytest.mark.parametrize("schedule", SCHEDULES)
def test_full_model_adjoint_under_contention(cm, schedule, cap):
    announce(f"models: full-model adjoint, 32x32 block upstream, schedule {schedule}, "
             f"stored exits {cap}")
    ds, inv = cm.scenes["full"]
    g = cm.g
    p = voro.default_params(appearance=1, schedule=schedule)
    trace = (torch.empty((cap, cm.cam.n_rays, 2), dtype=torch.int32, device=cm.dev)
             if cap else None)
    rgb, T, ray = voro.voro_render_views_fwd(ds, [cm.cam], p, trace=trace)
    npx = cm.cam.n_pixels
    gimg = np.zeros((npx, 3), np.float32)
    use = g["grad_rays"]
    gimg[g["pixels"][use]] = g["g_rgb"][use]
    gs, gd, gt = voro.voro_render_views_bwd(ds, [cm.cam], rgb, T, ray, to_dev(gimg, cm.dev),
                                            None, p, trace=trace)
    gs, gd, gt = gs.cpu().numpy(), gd.cpu().numpy(), gt.cpu().numpy()
    assert gt.shape == (ds.n, 2, ds.tex_res, ds.tex_res, 4)
    k = inv[g["grad_cells"]]
    want = {"sites": g["grad_sites"], "density": g["grad_density"],
            "texels": dense_texel_grads(g)}
    got = {"sites": gs[k], "density": gd[k], "texels": gt[k][..., :3]}
    for name in want:
        scale = max(1e-12, float(np.abs(want[name]).max()))
        err = float(np.abs(got[name] - want[name]).max())
        announce(f"models full adjoint {name}: max err {err:.2e} of max |grad| {scale:.2e}")
        assert err <= 1e-4 * scale + 1e-6, (name, err, scale)
    # both maps carry gradient, and nothing outside the touched cells moves
    assert np.abs(want["texels"][:, 0]).max() > 0 and np.abs(want["texels"][:, 1]).max() > 0
    mask = np.ones(ds.n, bool)
    mask[k] = False
    assert np.all(gs[mask] == 0) and np.all(gd[mask] == 0) and np.all(gt[mask] == 0)
    assert np.all(gt[..., 3] == 0)
