"""Wave-cooperative staging of edge rows (forward, one lane per ray): the
staged exit search must see the same records in the same order as the
per-lane gather, on coherent waves (rows staged every step), incoherent
waves (too many distinct cells: gather, with the back-off between tries)
and waves that switch between the two.  Lanes-per-ray 2 never stages, so it
is the reference; outputs and visited-cell sequences must be bit-identical."""
import numpy as np
import pytest
import torch

from paper_2608_17682_amd import synth, voro

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def scene(dev):
    sc = synth.scene_uniform(4000, 4, seed=21)
    ds = voro.device_scene(sc, dev)
    voro.voro_prepare(ds)
    return ds


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    voro.lib()
    return torch.device("cuda:0")


def rays(kind, n, dev, seed):
    rng = np.random.default_rng(seed)
    nb = (n + 63) // 64  # bundles of 64 rays, the last one cut short
    if kind == "coherent":
        # 64-ray bundles from one point with directions within ~0.01 rad
        base = rng.normal(size=(nb, 3))
        base /= np.linalg.norm(base, axis=1, keepdims=True)
        d = np.repeat(base, 64, axis=0)[:n] + 0.004 * rng.normal(size=(n, 3))
        o = np.repeat(rng.uniform(-0.2, 0.2, size=(nb, 3)), 64, axis=0)[:n]
    elif kind == "incoherent":
        d = rng.normal(size=(n, 3))
        o = rng.uniform(-0.9, 0.9, size=(n, 3))
    else:
        # bundles that start together and fan out, so waves go from staged
        # to gathered part-way along the walk
        base = rng.normal(size=(nb, 3))
        base /= np.linalg.norm(base, axis=1, keepdims=True)
        d = np.repeat(base, 64, axis=0)[:n] + 0.15 * rng.normal(size=(n, 3))
        o = np.repeat(rng.uniform(-0.2, 0.2, size=(nb, 3)), 64, axis=0)[:n]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    O = torch.from_numpy(o.astype(np.float32)).to(dev)
    D = torch.from_numpy(d.astype(np.float32)).to(dev)
    TM = torch.full((n,), 3.0, device=dev)
    return O, D, TM


@pytest.mark.parametrize("kind", ["coherent", "incoherent", "fanning"])
@pytest.mark.parametrize("tex", ["float32", "float16"])
def test_staged_walk_is_bit_identical(dev, scene, kind, tex):
    n = 64 * 96 + 17  # ragged last wave
    O, D, TM = rays(kind, n, dev, seed={"coherent": 1, "incoherent": 2, "fanning": 3}[kind])
    S = voro.voro_locate_origins(scene, O)
    ds = scene if tex == "float32" else scene.with_arrays(
        texels=voro.voro_cast_texels(scene.texels, tex))
    voro.voro_prepare(ds)
    out = []
    for lpr in (1, 2):
        announce(f"staging {kind} {tex} lpr={lpr}")
        p = voro.default_params(lanes_per_ray=lpr, max_record=160)
        ns = torch.empty(n, dtype=torch.int32, device=dev)
        cells = torch.empty((n, 160), dtype=torch.int32, device=dev)
        st = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
        rgb, T = voro.voro_render_fwd(ds, O, D, TM, S, p, nsteps=ns, cells=cells, stats=st)
        out.append((rgb, T, ns, cells, st))
    a, b = out
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert torch.equal(a[2], b[2]) and torch.equal(a[3], b[3])
    sa = dict(zip(voro.STAT_NAMES, a[4].tolist()))
    sb = dict(zip(voro.STAT_NAMES, b[4].tolist()))
    for k in ("rays", "steps", "degree_sum", "fp64_redecide", "max_steps"):
        assert sa[k] == sb[k], k
    assert sa["steps"] > 5 * n


def test_staged_adjoint_inputs_match(dev, scene):
    # the adjoint replays the gathered walk; fed the staged forward's outputs
    # it must give the gradients it gives for the unstaged forward's
    n = 64 * 32
    O, D, TM = rays("fanning", n, dev, seed=5)
    S = voro.voro_locate_origins(scene, O)
    rgb1, T1 = voro.voro_render_fwd(scene, O, D, TM, S, voro.default_params(lanes_per_ray=1))
    rgb2, T2 = voro.voro_render_fwd(scene, O, D, TM, S, voro.default_params(lanes_per_ray=2))
    assert torch.equal(rgb1, rgb2) and torch.equal(T1, T2)
    g = torch.from_numpy(synth.upstream(n, 9)[0]).to(dev)
    gs, gd, gt = voro.voro_render_bwd(scene, O, D, TM, S, rgb1, T1, g)
    assert torch.isfinite(gs).all() and torch.isfinite(gd).all() and torch.isfinite(gt).all()
