"""GPU parity at the benchmarked 100k-site workload and its half-precision form.

Scene: 70% of 100k sites jittered on the unit sphere (density 50), 30%
uniform in [-2,2]^3 (density 0.01), 8x8 texels; pose 0 of the 800x800
pinhole orbit.  Rays: two 64x64 crops (centre and seeded), 8192 rays.  The
expected values are the FP64 oracle's (tests/golden/config2_crops.npz,
written by tests/golden/make_goldens.py from oracle/ only).

* The image comes from the launch the benchmark times: Morton-ordered cells,
  in-kernel ray generation, the tuned launch shape.  Colour and
  transmittance within 1e-4 of the oracle on every ray except those whose
  transmittance lands next to t_stop (Sec. 3.2 stop rule; they may stop one
  segment earlier or later).
* Cell counts and visited-cell sequences are bit-exact on every ray the
  oracle does not mark degenerate, walked from the oracle's FP32 rays.
* Texels stored in binary16 / bfloat16 (Sec. 5.6): within 1e-4 of the oracle
  fed the rounded texels, and within the rounding bound half-ulp x (1 - T)
  (2^-12 for binary16, 2^-9 for bfloat16, texels in [0,1]) plus 1e-4 of the
  oracle on the original FP32 texels.
"""
import os

import numpy as np
import pytest
import torch

from paper_2608_17682_amd import autotune, synth, voro
from helpers import scene_fingerprint, seq_hash

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config2_crops.npz")
HALF_ULP = {"float16": 2.0 ** -12, "bfloat16": 2.0 ** -9}


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


class Case:
    pass


@pytest.fixture(scope="module")
def c2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    voro.lib()
    dev = torch.device("cuda:0")
    c = Case()
    z = np.load(GOLDEN, allow_pickle=False)
    c.g = {k: z[k] for k in z.files}
    announce("config2: 100k-site shell scene (Qhull adjacency)")
    c.scene, cams = synth.config2()
    assert scene_fingerprint(c.scene) == str(c.g["fingerprint"]), "scene differs from the golden's"
    c.cam = cams[0]
    ds0 = voro.device_scene(c.scene, dev)
    c.ds, perm, inv = voro.voro_morton_reorder(ds0)
    voro.voro_prepare(c.ds)
    c.perm, c.inv = perm.cpu().numpy(), inv.cpu().numpy()
    c.params = autotune.params_for(c.ds, [c.cam], "fwd")
    c.dev = dev
    return c


def views_image(c, ds):
    rgb, T, _ = voro.voro_render_views_fwd(ds, [c.cam], c.params)
    px = c.g["pixels"]
    return rgb.cpu().numpy()[px], T.cpu().numpy()[px]


def test_config2_benchmark_launch_matches_oracle(c2):
    announce("config2: bench launch (views, Morton, tuned shape), f32 texels, 8192 crop rays")
    rgb, T = views_image(c2, c2.ds)
    ok = ~c2.g["stop_degenerate"]
    assert ok.mean() > 0.99
    err_rgb = np.abs(rgb - c2.g["rgb_float32"])[ok]
    err_T = np.abs(T - c2.g["T"])[ok]
    announce(f"config2 f32: max |rgb err| {err_rgb.max():.2e}, max |T err| {err_T.max():.2e}")
    assert err_rgb.max() <= 1e-4 and err_T.max() <= 1e-4
    # the stop-degenerate rays differ by at most one segment after T ~ t_stop
    bad = ~ok
    if bad.any():
        assert np.abs(rgb - c2.g["rgb_float32"])[bad].max() <= 2e-4


def test_config2_sequences_bit_exact(c2):
    announce("config2: explicit oracle rays, cell sequences (max_record 256)")
    g = c2.g
    R = len(g["o"])
    O, D, TM = (torch.from_numpy(np.ascontiguousarray(g[k])).to(c2.dev) for k in ("o", "d", "tmax"))
    S = torch.from_numpy(c2.inv[g["start"]].astype(np.int32)).to(c2.dev)
    p = voro.voro_params.from_buffer_copy(c2.params)
    p.max_record = 256
    nsteps = torch.empty(R, dtype=torch.int32, device=c2.dev)
    cells = torch.empty((R, 256), dtype=torch.int32, device=c2.dev)
    rgb, T = voro.voro_render_fwd(c2.ds, O, D, TM, S, p, nsteps=nsteps, cells=cells)
    K, cells = nsteps.cpu().numpy(), cells.cpu().numpy()
    assert K.max() <= 256
    ok = ~g["degenerate"]
    assert ok.mean() > 0.97
    assert np.array_equal(K[ok], g["K"][ok])
    mism = [r for r in np.nonzero(ok)[0]
            if seq_hash(c2.perm[cells[r, :K[r]]]) != int(g["seq_hash"][r])]
    assert not mism, f"{len(mism)} sequences differ, first rays {mism[:5]}"
    sd = ~g["stop_degenerate"]
    assert np.abs(rgb.cpu().numpy() - g["rgb_float32"])[sd].max() <= 1e-4
    assert np.abs(T.cpu().numpy() - g["T"])[sd].max() <= 1e-4
    announce(f"config2: {ok.sum()} of {R} sequences compared, all equal; mean K {K.mean():.1f}")


@pytest.mark.parametrize("dtype", ["float16", "bfloat16"])
def test_config4_half_texels_match_oracle(c2, dtype):
    announce(f"config4: {dtype} texels through the bench launch")
    dsh = c2.ds.with_arrays(texels=voro.voro_cast_texels(c2.ds.texels, dtype))
    voro.voro_prepare(dsh)
    rgb, T = views_image(c2, dsh)
    g = c2.g
    ok = ~g["stop_degenerate"]
    # against the oracle fed the rounded texels: the FP32 parity bar again
    e_deq = np.abs(rgb - g[f"rgb_{dtype}"])[ok]
    assert e_deq.max() <= 1e-4, e_deq.max()
    # against the original texels: the rounding bound
    e_orig = np.abs(rgb - g["rgb_float32"])[ok]
    bound = HALF_ULP[dtype] * (1.0 - g["T"][ok])[:, None] + 1e-4
    assert np.all(e_orig <= bound), float((e_orig - bound).max())
    announce(f"config4 {dtype}: vs rounded texels max {e_deq.max():.2e}; vs f32 texels max "
             f"{e_orig.max():.2e} mean {e_orig.mean():.2e} (bound {HALF_ULP[dtype]:.2e} (1-T))")
    voro.voro_prepare(c2.ds)
