"""Pins of the oracle's distortion loss (Sec. 5.3, eq. distortion-loss) and of
its adjoint: the depth map's special values, one- and two-interval closed
forms, the discretisation independence of a uniform weight spread, the
prefix-sum evaluation for ordered intervals, partial derivatives against
differences of the loss, and the chained ray gradient against central
differences of the forward."""
import math

import numpy as np
import pytest

from oracle import adjoint, distortion, render
from paper_2608_17682_amd import synth


def test_depth_map_special_values():
    assert float(distortion.s_of_t(0.0)) == 0.0
    assert float(distortion.s_of_t(1.0)) == 0.5
    assert float(distortion.s_of_t(3.0)) == pytest.approx(1.0 - 1.0 / 4.0, rel=1e-15)
    assert float(distortion.s_of_t(1e12)) == pytest.approx(1.0, rel=1e-11)


def test_single_and_two_interval_closed_forms():
    s = lambda t: 1.0 - 1.0 / (1.0 + t)
    w, a, b = 0.7, 0.5, 2.0
    assert distortion.distortion([w], [a], [b]) == pytest.approx(w * w * (s(b) - s(a)) / 3.0,
                                                                 rel=1e-14)
    w1, w2 = 0.3, 0.6
    t = [0.2, 1.1, 4.0]
    sb1, sb2 = (s(t[0]) + s(t[1])) / 2, (s(t[1]) + s(t[2])) / 2
    want = 2 * w1 * w2 * abs(sb1 - sb2) + (w1 ** 2 * (s(t[1]) - s(t[0])) +
                                           w2 ** 2 * (s(t[2]) - s(t[1]))) / 3.0
    assert distortion.distortion([w1, w2], t[:2], t[1:]) == pytest.approx(want, rel=1e-14)


@pytest.mark.parametrize("K", [1, 2, 5, 40])
def test_uniform_spread_is_independent_of_the_discretisation(K):
    # weights W/K on K equal intervals of s in [sa, sb]: pairs give
    # W^2 (sb-sa)(K^2-1)/(3K^2), the interval term W^2 (sb-sa)/(3K^2); the sum
    # is W^2 (sb - sa)/3 whatever K
    W, sa, sb = 0.8, 0.2, 0.9
    s_edges = np.linspace(sa, sb, K + 1)
    t_edges = s_edges / (1.0 - s_edges)          # inverse of s(t) = t/(1+t)
    d = distortion.distortion(np.full(K, W / K), t_edges[:-1], t_edges[1:])
    assert d == pytest.approx(W * W * (sb - sa) / 3.0, rel=1e-12)


def test_prefix_sum_form_for_ordered_intervals():
    rng = np.random.default_rng(0)
    t = np.sort(rng.uniform(0, 6, 30))
    w = rng.uniform(0, 0.2, 29)
    s0, s1 = t[:-1] / (1 + t[:-1]), t[1:] / (1 + t[1:])
    sb = (s0 + s1) / 2
    W = A = total = 0.0
    for k in range(len(w)):
        total += 2 * w[k] * (sb[k] * W - A) + w[k] ** 2 * (s1[k] - s0[k]) / 3
        W += w[k]
        A += w[k] * sb[k]
    assert distortion.distortion(w, t[:-1], t[1:]) == pytest.approx(total, rel=1e-12)


def test_partials_match_differences_of_the_loss():
    rng = np.random.default_rng(1)
    t = np.sort(rng.uniform(0, 5, 9))
    t0, t1 = t[:-1].copy(), t[1:].copy()
    w = rng.uniform(0, 0.3, 8)
    gw, g0, g1 = distortion.distortion_partials(w, t0, t1)
    h = 1e-7
    for k in range(8):
        for arr, g in ((w, gw), (t0, g0), (t1, g1)):
            a = arr[k]
            arr[k] = a + h
            fp = distortion.distortion(w, t0, t1)
            arr[k] = a - h
            fm = distortion.distortion(w, t0, t1)
            arr[k] = a
            assert g[k] == pytest.approx((fp - fm) / (2 * h), rel=1e-6, abs=1e-9)


@pytest.mark.parametrize("seed,dens_scale", [(0, 1.0), (1, 8.0)])
def test_ray_gradient_with_distortion_matches_central_differences(seed, dens_scale):
    scene = synth.scene_uniform(64, 3, seed=seed)
    sites = scene.sites.astype(np.float64)
    dens = scene.density.astype(np.float64) * dens_scale
    tex = scene.texels.astype(np.float64)
    rng = np.random.default_rng(40 + seed)
    k = 5
    o = rng.uniform(-0.8, 0.8, (k, 3))
    w = rng.normal(size=(k, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    g = rng.normal(size=(k, 3))
    gT = rng.normal(size=k)
    gdist = rng.normal(size=k)
    tmax = 3.0
    recs = [render.render_ray(sites, dens, tex, o[r], w[r], tmax) for r in range(k)]
    starts = [rec.cells[0] for rec in recs]
    gs, gd, gt = adjoint.grad_rays(sites, dens, tex, o, w, tmax, recs, g, gT, gdist)

    def loss():
        tot = 0.0
        for r in range(k):
            rec = render.render_ray(sites, dens, tex, o[r], w[r], tmax, start=starts[r])
            tot += float(g[r] @ rec.rgb) + gT[r] * rec.T + gdist[r] * rec.dist
        return tot

    def fd(arr, idx, h):
        a0 = arr[idx]
        arr[idx] = a0 + h
        lp = loss()
        arr[idx] = a0 - h
        lm = loss()
        arr[idx] = a0
        return (lp - lm) / (2 * h)

    touched = sorted({c for rec in recs for c in rec.cells})
    for c in np.random.default_rng(seed).choice(touched, size=min(10, len(touched)), replace=False):
        for ax in range(3):
            assert gs[c, ax] == pytest.approx(fd(sites, (c, ax), 1e-6), rel=2e-5, abs=2e-7)
        assert gd[c] == pytest.approx(fd(dens, c, 1e-6 * max(1.0, dens[c])), rel=2e-5, abs=2e-7)
    assert any(rec.dist > 0 for rec in recs)
