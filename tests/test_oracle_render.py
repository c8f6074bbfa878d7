"""Pins of the oracle's compositing and early stop (Sec. 3.2)."""
import math
import os

import numpy as np
import pytest

from oracle import render, walk
from paper_2608_17682_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            out[k] = [float(x) for x in v]
    return out


def test_three_cells_hand_derived():
    g = read_golden("three_cells_z.txt")
    sites = np.array([[0, 0, -1], [0, 0, 0], [0, 0, 1]], np.float32)
    dens = np.array([0.2, 1.0, 0.5])  # float64: the closed form uses these exact values
    tex = np.zeros((3, 2, 2, 4), np.float32)
    tex[0, ..., 0] = 1
    tex[1, ..., 1] = 1
    tex[2, ..., 2] = 1
    rec = render.render_ray(sites, dens, tex, [0, 0, -3], [0, 0, 1], 5.0, t_stop=0.0)
    assert rec.cells == [int(c) for c in g["cells"]]
    np.testing.assert_allclose(rec.exit[:2], g["boundaries"], atol=1e-15)
    np.testing.assert_allclose(rec.delta, g["deltas"], atol=1e-15)
    np.testing.assert_allclose(rec.rgb, g["rgb"], rtol=1e-14)
    assert rec.T == pytest.approx(g["T"][0], rel=1e-14)


def test_two_segments_closed_form():
    sites = np.array([[0, 0, -0.5], [0, 0, 0.5]], np.float32)
    s0, s1 = 0.3, 1.7
    dens = np.array([s0, s1], np.float32).astype(np.float64)
    c0, c1 = np.array([0.2, 0.4, 0.6]), np.array([0.9, 0.1, 0.5])
    tex = np.zeros((2, 4, 4, 4))
    tex[0, ..., :3] = c0
    tex[1, ..., :3] = c1
    rec = render.render_ray(sites, dens, tex, [0, 0, -3], [0, 0, 1], 5.0, t_stop=0.0)
    s0, s1 = float(np.float32(s0)), float(np.float32(s1))
    want = (1 - math.exp(-3 * s0)) * c0 + math.exp(-3 * s0) * (1 - math.exp(-2 * s1)) * c1
    np.testing.assert_allclose(rec.rgb, want, rtol=1e-14)
    assert rec.T == pytest.approx(math.exp(-3 * s0 - 2 * s1), rel=1e-14)


def _random_rays(rng, k, span=1.5):
    o = rng.uniform(-span, span, (k, 3))
    w = rng.normal(size=(k, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    return o, w


def test_constant_density_transmittance_independent_of_partition():
    scene = synth.scene_uniform(200, 4, seed=3)
    rng = np.random.default_rng(0)
    sigma = 0.37
    dens = np.full(scene.n, sigma)
    col = synth.texels_rgb(scene.n, 4, (0.3, 0.6, 0.9))
    o, w = _random_rays(rng, 10)
    for r in range(10):
        rec = render.render_ray(scene.sites, dens, col, o[r], w[r], 4.0, t_stop=0.0)
        T = math.exp(-sigma * 4.0)
        assert rec.T == pytest.approx(T, rel=1e-12)
        c32 = np.array([0.3, 0.6, 0.9], np.float32).astype(np.float64)
        np.testing.assert_allclose(rec.rgb, (1 - T) * c32, rtol=1e-12)


def test_monotone_transmittance_and_colour_bounds():
    scene = synth.scene_uniform(256, 4, seed=4)
    rng = np.random.default_rng(1)
    o, w = _random_rays(rng, 16)
    for r in range(16):
        rec = render.render_ray(scene.sites, scene.density, scene.texels, o[r], w[r], 6.0)
        Ts = rec.T_before + [rec.T]
        assert all(Ts[k + 1] <= Ts[k] for k in range(len(Ts) - 1))
        cmax = float(scene.texels[rec.cells][..., :3].max())
        assert np.all(rec.rgb >= 0) and np.all(rec.rgb <= (1 - rec.T) * cmax + 1e-15)
        np.testing.assert_allclose(sum(rec.weight), 1 - rec.T, rtol=1e-12)


def test_split_ray_composes_associatively():
    # (C1, T1) (+) (C2, T2) = (C1 + T1 C2, T1 T2) for a ray cut at any t_s.
    scene = synth.scene_uniform(256, 4, seed=5)
    rng = np.random.default_rng(2)
    o, w = _random_rays(rng, 8, 1.0)
    for r in range(8):
        full = render.render_ray(scene.sites, scene.density, scene.texels, o[r], w[r], 5.0,
                                 t_stop=0.0)
        ts = 0.37 * 5.0
        a = render.render_ray(scene.sites, scene.density, scene.texels, o[r], w[r], ts, t_stop=0.0)
        b = render.render_ray(scene.sites, scene.density, scene.texels, o[r] + ts * w[r], w[r],
                              5.0 - ts, t_stop=0.0)
        np.testing.assert_allclose(a.rgb + a.T * b.rgb, full.rgb, rtol=1e-11, atol=1e-14)
        assert a.T * b.T == pytest.approx(full.T, rel=1e-11)
        assert a.cells[-1] == b.cells[0]
        assert a.cells + b.cells[1:] == full.cells


def test_early_stop_is_strict_after_compositing():
    scene = synth.scene_uniform(256, 4, seed=6)
    dens = scene.density * 20
    rng = np.random.default_rng(3)
    o, w = _random_rays(rng, 12, 1.0)
    stopped = 0
    for r in range(12):
        rec = render.render_ray(scene.sites, dens, scene.texels, o[r], w[r], 6.0, t_stop=1e-4)
        assert all(T >= 1e-4 for T in rec.T_before)
        if rec.stop == "tstop":
            stopped += 1
            assert rec.T < 1e-4
        else:
            assert rec.T >= 1e-4
    assert stopped >= 6


def test_max_steps_and_skip():
    scene = synth.scene_uniform(256, 4, seed=8)
    o, w = np.array([0.1, 0.2, -1.5]), np.array([0.0, 0.0, 1.0])
    rec = render.render_ray(scene.sites, scene.density, scene.texels, o, w, 6.0, t_stop=0.0,
                            max_steps=3)
    assert rec.K == 3 and rec.stop == "max_steps"
    base = render.render_ray(scene.sites, scene.density, scene.texels, o, w, 6.0)
    sk = render.render_ray(scene.sites, scene.density, scene.texels, o, w, 6.0, skip_w=0.05)
    assert sk.T == base.T and sk.cells == base.cells
    keep = [k for k in range(base.K) if base.weight[k] >= 0.05]
    want = sum(base.weight[k] * base.color[k] for k in keep)
    np.testing.assert_allclose(sk.rgb, want, rtol=1e-14)
    assert any(sk.skipped) and not all(sk.skipped)


def test_tmax_zero_and_origin_outside_hull():
    scene = synth.scene_uniform(128, 4, seed=9)
    # origin far outside the hull, looking away: one unbounded cell to tmax
    rec = render.render_ray(scene.sites, scene.density, scene.texels, [0, 0, -10], [0, 0, -1], 3.0)
    assert rec.K == 1 and rec.delta[0] == 3.0
    rgb, T, recs = render.render_rays(scene.sites, scene.density, scene.texels,
                                      np.zeros((1, 3)), np.array([[0, 0, 1.0]]), [0.0])
    assert T[0] == 1.0 and np.all(rgb == 0) and recs[0] is None


def test_permutation_invariance():
    scene = synth.scene_uniform(128, 4, seed=10)
    perm = np.random.default_rng(0).permutation(scene.n)
    inv = np.argsort(perm)
    rng = np.random.default_rng(4)
    o, w = _random_rays(rng, 6, 1.0)
    for r in range(6):
        a = render.render_ray(scene.sites, scene.density, scene.texels, o[r], w[r], 6.0)
        b = render.render_ray(scene.sites[perm], scene.density[perm], scene.texels[perm], o[r],
                              w[r], 6.0)
        assert [int(perm[c]) for c in b.cells] == a.cells
        np.testing.assert_allclose(a.rgb, b.rgb, rtol=1e-13)
        assert inv[a.cells[0]] == b.cells[0]
