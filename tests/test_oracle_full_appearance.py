"""Pins of the oracle's full appearance model (Sec. 5.1 surface map indexed
by the site-to-hit-point direction, Sec. 5.2 view map and logit-space sum
under a sigmoid) and of its adjoint: closed forms, a hand-derived two-cell
ray, derivatives of the octahedral map and bilinear lookup against
differences of the map itself, central finite differences of the forward,
and scale invariance (Sec. 5.4)."""
import math

import numpy as np
import pytest

from oracle import adjoint, appearance, render
from paper_2608_17682_amd import synth


def logistic(x):
    return 1.0 / (1.0 + math.exp(-x))


def test_sigmoid_special_values():
    assert float(appearance.sigmoid(0.0)) == 0.5
    xs = np.array([-800.0, -30.0, -1.5, 0.3, 2.0, 40.0, 800.0])
    s = appearance.sigmoid(xs)
    assert np.all(np.isfinite(s)) and s[0] == 0.0 and s[-1] == 1.0
    np.testing.assert_allclose(s + appearance.sigmoid(-xs), 1.0, rtol=0, atol=1e-15)
    for x in (-1.5, 0.3, 2.0):
        assert float(appearance.sigmoid(x)) == pytest.approx(logistic(x), rel=1e-15)


def _two_cells(R=3):
    sites = np.array([[0.0, 0.0, -0.5], [0.0, 0.0, 0.5]])
    dens = np.array([0.7, 1.9])
    rng = np.random.default_rng(5)
    tex = rng.normal(0.0, 1.0, (2, 2, R, R, 4))
    return sites, dens, tex


def test_two_cells_hand_derived():
    # o = (0,0,-3), w = +z, tmax 6: the start cell 0 is left at its bisector
    # z = 0 (t = 3), which is also where cell 1 is entered.  Cell 0's hit point
    # is its exit point (0,0,0): d = +z -> (u,v) = (0,0) -> texel (1,1) of a
    # 3x3 map with weight 1.  Cell 1's hit point is its entry point (0,0,0):
    # d = -z -> (1,1) -> texel (2,2).  The view direction -w = -z -> texel (2,2)
    # of both view maps.
    sites, dens, tex = _two_cells()
    rec = render.render_ray(sites, dens, tex, [0.0, 0.0, -3.0], [0.0, 0.0, 1.0], 6.0,
                            appearance=1)
    assert rec.cells == [0, 1]
    assert rec.t_hit == [3.0, 3.0]
    c0 = [logistic(tex[0, 0, 1, 1, ch] + tex[0, 1, 2, 2, ch]) for ch in range(3)]
    c1 = [logistic(tex[1, 0, 2, 2, ch] + tex[1, 1, 2, 2, ch]) for ch in range(3)]
    a0 = 1.0 - math.exp(-3.0 * 0.7)
    a1 = 1.0 - math.exp(-3.0 * 1.9)
    want = [a0 * c0[ch] + (1.0 - a0) * a1 * c1[ch] for ch in range(3)]
    np.testing.assert_allclose(rec.rgb, want, rtol=1e-14, atol=0)
    assert rec.T == pytest.approx(math.exp(-3.0 * (0.7 + 1.9)), rel=1e-14)


@pytest.mark.parametrize("which", ["surface", "view"])
def test_constant_logits_give_constant_colour(which):
    # one map constant per channel, the other zero: every cell shows
    # sigmoid(l), so C = (1 - T) sigmoid(l) whatever the partition
    scene = synth.scene_uniform(60, 4, seed=2)
    l = np.array([0.4, -1.2, 2.5])
    tex = np.zeros((60, 2, 4, 4, 4))
    tex[:, 0 if which == "surface" else 1, :, :, :3] = l
    rng = np.random.default_rng(4)
    for _ in range(6):
        o = rng.uniform(-0.7, 0.7, 3)
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        rec = render.render_ray(scene.sites, scene.density, tex, o, w, 3.0, appearance=1)
        sig = np.array([logistic(x) for x in l])
        np.testing.assert_allclose(rec.rgb, (1.0 - rec.T) * sig, rtol=1e-12, atol=1e-15)


def test_surface_map_varies_across_one_cell():
    # a single site: the ray stays in its cell; the hit point is the clipped
    # exit o + tmax w, and a surface map linear in (u, v) (reproduced exactly
    # by bilinear interpolation) returns a + b u + c v at d = (x - p)/|x - p|
    R = 5
    p = np.array([[0.1, -0.2, 0.3]])
    tex = np.zeros((1, 2, R, R, 4))
    cols = np.linspace(-1.0, 1.0, R)
    for r in range(R):
        for c in range(R):
            tex[0, 0, r, c, :3] = 0.3 + 0.8 * cols[c] - 0.5 * cols[r]
    rng = np.random.default_rng(9)
    for _ in range(8):
        o = rng.uniform(-1, 1, 3)
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        tmax = rng.uniform(0.5, 3.0)
        rec = render.render_ray(p, np.array([1.3]), tex, o, w, tmax, appearance=1)
        x = o + tmax * w
        d = (x - p[0]) / np.linalg.norm(x - p[0])
        u, v = appearance.octahedral(d)
        want = logistic(0.3 + 0.8 * u - 0.5 * v)
        np.testing.assert_allclose(rec.rgb, (1.0 - rec.T) * want, rtol=1e-12)


def test_octahedral_jacobian_matches_differences_of_the_map():
    rng = np.random.default_rng(1)
    h = 1e-7
    for _ in range(200):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        if min(abs(d[0]), abs(d[1]), abs(d[2])) < 1e-3:
            continue
        ju, jv = appearance.octahedral_jacobian(d)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            up, vp = appearance.octahedral(d + e)
            um, vm = appearance.octahedral(d - e)
            assert ju[a] == pytest.approx((up - um) / (2 * h), abs=1e-6)
            assert jv[a] == pytest.approx((vp - vm) / (2 * h), abs=1e-6)


def test_lookup_gradient_matches_differences_of_the_lookup():
    rng = np.random.default_rng(2)
    tex = rng.normal(size=(6, 6, 4))
    h = 1e-7
    for _ in range(100):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        dcu, dcv = appearance.lookup_grad_uv(tex, d)
        ju, jv = appearance.octahedral_jacobian(d)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            num = (appearance.lookup(tex, d + e) - appearance.lookup(tex, d - e)) / (2 * h)
            np.testing.assert_allclose(dcu * ju[a] + dcv * jv[a], num, atol=2e-5)


def _problem(seed, n=64, k=6, dens_scale=1.0, R=4):
    scene = synth.scene_uniform(n, R, seed=seed)
    rng = np.random.default_rng(300 + seed)
    tex = rng.normal(0.0, 1.0, (n, 2, R, R, 4))
    o = rng.uniform(-0.8, 0.8, (k, 3))
    w = rng.normal(size=(k, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    g = rng.normal(size=(k, 3))
    gT = rng.normal(size=k)
    return (scene.sites.astype(np.float64), scene.density.astype(np.float64) * dens_scale, tex,
            o, w, g, gT)


def _loss(sites, dens, tex, o, w, tmax, g, gT, starts):
    total = 0.0
    for r in range(len(o)):
        rec = render.render_ray(sites, dens, tex, o[r], w[r], tmax, start=starts[r],
                                appearance=1)
        total += float(g[r] @ rec.rgb) + gT[r] * rec.T
    return total


@pytest.mark.parametrize("seed,dens_scale", [(0, 1.0), (1, 12.0)])
def test_full_model_gradients_match_central_differences(seed, dens_scale):
    sites, dens, tex, o, w, g, gT = _problem(seed, dens_scale=dens_scale)
    tmax = 3.0
    recs = [render.render_ray(sites, dens, tex, o[r], w[r], tmax, appearance=1)
            for r in range(len(o))]
    starts = [rec.cells[0] for rec in recs]
    gs, gd, gt = adjoint.grad_rays(sites, dens, tex, o, w, tmax, recs, g, gT)
    assert gt.shape == tex.shape
    touched = sorted({c for rec in recs for c in rec.cells})
    rng = np.random.default_rng(seed)

    def fd(arr, idx, h):
        a0 = arr[idx]
        arr[idx] = a0 + h
        lp = _loss(sites, dens, tex, o, w, tmax, g, gT, starts)
        arr[idx] = a0 - h
        lm = _loss(sites, dens, tex, o, w, tmax, g, gT, starts)
        arr[idx] = a0
        return (lp - lm) / (2 * h)

    checked = 0
    for c in rng.choice(touched, size=min(10, len(touched)), replace=False):
        for ax in range(3):
            assert gs[c, ax] == pytest.approx(fd(sites, (c, ax), 1e-6), rel=2e-5, abs=2e-7)
            checked += 1
        assert gd[c] == pytest.approx(fd(dens, c, 1e-6 * max(1.0, dens[c])), rel=2e-5, abs=2e-7)
        for m in range(2):
            for (rr, cc, ch) in np.argwhere(gt[c, m] != 0)[:4]:
                assert gt[c, m, rr, cc, ch] == pytest.approx(fd(tex, (c, m, rr, cc, ch), 1e-6),
                                                             rel=2e-5, abs=2e-7)
                checked += 1
    assert checked >= 40
    assert np.all(gt[..., 3] == 0)


def test_full_model_scale_invariance():
    # d = (x - p)/|x - p| and the view direction are unchanged by a uniform
    # scale, so the image, T and dL/drho are too; dL/dp scales by 1/s
    sites, dens, tex, o, w, g, gT = _problem(3, n=80, k=5)
    s = 2.5
    out = []
    for scale in (1.0, s):
        recs = [render.render_ray(sites * scale, dens / scale, tex, o[r] * scale, w[r],
                                  3.0 * scale, appearance=1) for r in range(len(o))]
        grads = adjoint.grad_rays(sites * scale, dens / scale, tex, o * scale, w, 3.0 * scale,
                                  recs, g, gT)
        out.append((recs, grads))
    (ra, (gsa, gda, gta)), (rb, (gsb, gdb, gtb)) = out
    for a, b in zip(ra, rb):
        assert a.cells == b.cells
        np.testing.assert_allclose(a.rgb, b.rgb, rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(gda * dens, gdb * (dens / s), rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(gsa / s, gsb, rtol=1e-8, atol=1e-12)
    np.testing.assert_allclose(gta, gtb, rtol=1e-9, atol=1e-13)


def test_appearance_zero_is_unchanged_and_bad_layout_rejected():
    sites, dens, tex = _two_cells()
    with pytest.raises(ValueError):
        render.render_ray(sites, dens, tex[:, 0], [0, 0, -3.0], [0, 0, 1.0], 6.0, appearance=1)
    rec = render.render_ray(sites, dens, tex[:, 0], [0, 0, -3.0], [0, 0, 1.0], 6.0)
    assert rec.appearance == 0 and rec.t_hit == []
