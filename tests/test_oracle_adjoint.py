"""Pins of the oracle's analytic gradient: central finite differences of the
oracle forward (FP64), closed forms (Sec. 5.4 density gradient; bisector
crossing derivative), scale invariance (Sec. 5.4) and permutation."""
import math

import numpy as np
import pytest

from oracle import adjoint, render
from paper_2608_17682_amd import synth


def loss(sites, dens, tex, o, w, tmax, g, gT, starts, t_stop=1e-4):
    total = 0.0
    for r in range(len(o)):
        rec = render.render_ray(sites, dens, tex, o[r], w[r], tmax, t_stop=t_stop,
                                start=starts[r])
        total += float(g[r] @ rec.rgb) + gT[r] * rec.T
    return total


def small_problem(seed, n=64, k=6, dens_scale=1.0):
    scene = synth.scene_uniform(n, 3, seed=seed)
    rng = np.random.default_rng(100 + seed)
    o = rng.uniform(-0.8, 0.8, (k, 3))
    w = rng.normal(size=(k, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    g = rng.normal(size=(k, 3))
    gT = rng.normal(size=k)
    sites = scene.sites.astype(np.float64)
    dens = scene.density.astype(np.float64) * dens_scale
    tex = scene.texels.astype(np.float64)
    return sites, dens, tex, o, w, g, gT


@pytest.mark.parametrize("seed,dens_scale", [(0, 1.0), (1, 1.0), (2, 15.0)])
def test_gradients_match_central_differences(seed, dens_scale):
    sites, dens, tex, o, w, g, gT = small_problem(seed, dens_scale=dens_scale)
    tmax = 3.0
    recs = []
    starts = []
    for r in range(len(o)):
        rec = render.render_ray(sites, dens, tex, o[r], w[r], tmax)
        recs.append(rec)
        starts.append(rec.cells[0])
    gs, gd, gt = adjoint.grad_rays(sites, dens, tex, o, w, tmax, recs, g, gT)
    touched = sorted({c for rec in recs for c in rec.cells})
    # an early-stopped ray's last exit face also moves with the (unvisited) next site
    beyond = sorted({rec.nxt[-1] for rec in recs
                     if rec.stop == "tstop" and rec.exit[-1] < tmax} - set(touched))
    rng = np.random.default_rng(seed)

    def fd(arr, idx, h):
        a0 = arr[idx]
        arr[idx] = a0 + h
        lp = loss(sites, dens, tex, o, w, tmax, g, gT, starts)
        arr[idx] = a0 - h
        lm = loss(sites, dens, tex, o, w, tmax, g, gT, starts)
        arr[idx] = a0
        return (lp - lm) / (2 * h)

    checked = 0
    for c in rng.choice(touched, size=min(12, len(touched)), replace=False):
        for ax in range(3):
            num = fd(sites, (c, ax), 1e-6)
            assert gs[c, ax] == pytest.approx(num, rel=2e-5, abs=2e-7), (c, ax)
            checked += 1
        num = fd(dens, c, 1e-6 * max(1.0, dens[c]))
        assert gd[c] == pytest.approx(num, rel=2e-5, abs=2e-7)
        for rr in range(3):
            for cc in range(3):
                num = fd(tex, (c, rr, cc, 1), 1e-6)
                assert gt[c, rr, cc, 1] == pytest.approx(num, rel=2e-5, abs=2e-7)
    for c in beyond:
        assert gd[c] == 0 and np.all(gt[c] == 0)
        for ax in range(3):
            num = fd(sites, (c, ax), 1e-6)
            assert gs[c, ax] == pytest.approx(num, rel=2e-5, abs=2e-7), (c, ax)
    assert checked >= 30
    if dens_scale > 1:
        assert beyond, "expected early-stopped rays whose exit face moves an unvisited site"
    assert np.all(gt[..., 3] == 0)
    # untouched cells get nothing
    mask = np.ones(len(sites), bool)
    mask[touched] = False
    assert np.all(gd[mask] == 0)
    mask[beyond] = False
    assert np.all(gs[mask] == 0)


def test_single_segment_density_gradient_identity():
    # One cell: T = exp(-sigma delta), alpha = 1 - T.  For L = T (g = 0, g_T = 1),
    # dL/dalpha = -1, so dL/dsigma = dL/dalpha * delta * (1 - alpha) and, under
    # sigma = exp(rho), dL/drho = dL/dalpha (1 - alpha) ln(1/(1 - alpha)).
    sites = np.array([[0.0, 0.0, 0.0]])
    sigma, tmax = 0.8, 2.5
    dens = np.array([sigma])
    tex = np.zeros((1, 2, 2, 4))
    rec = render.render_ray(sites, dens, tex, [0, 0, -1], [0, 0, 1], tmax, t_stop=0.0)
    gs, gd, gt = adjoint.grad_rays(sites, dens, tex, np.array([[0, 0, -1.0]]),
                                   np.array([[0, 0, 1.0]]), tmax, [rec], np.zeros((1, 3)), [1.0])
    alpha = 1 - math.exp(-sigma * tmax)
    assert gd[0] == pytest.approx(-1.0 * tmax * (1 - alpha), rel=1e-14)
    assert gd[0] * sigma == pytest.approx(-(1 - alpha) * math.log(1 / (1 - alpha)), rel=1e-13)
    assert np.all(gs == 0)


def test_two_site_crossing_derivative():
    # p0 = (0,0,-1/2), p1 = (0,0,1/2 + e): the crossing is t* = 3 + e/2, so
    # dt*/dp1_z = 1/2 = (p1 - x)_z / (n.w) at x = (0,0,0); lateral moves of p1
    # leave t* unchanged to first order.
    sites = np.array([[0, 0, -0.5], [0, 0, 0.5]])
    da, db = adjoint.face_dt_dsites(sites, 0, 1, [0, 0, -3], [0, 0, 1], 3.0)
    np.testing.assert_allclose(db, [0, 0, 0.5], atol=1e-15)
    np.testing.assert_allclose(da, [0, 0, 0.5], atol=1e-15)
    # and through the renderer: L = T with densities (s0, s1) -> dL/dp1_z
    s0, s1, tmax = 0.4, 1.1, 5.0
    dens = np.array([s0, s1])
    tex = np.zeros((2, 2, 2, 4))
    o, w = np.array([[0, 0, -3.0]]), np.array([[0, 0, 1.0]])
    rec = render.render_ray(sites, dens, tex, o[0], w[0], tmax, t_stop=0.0)
    gs, _, _ = adjoint.grad_rays(sites, dens, tex, o, w, tmax, [rec], np.zeros((1, 3)), [1.0])
    # T = exp(-s0 t* - s1 (tmax - t*)) -> dT/dt* = (s1 - s0) T
    T = math.exp(-s0 * 3 - s1 * 2)
    assert gs[1, 2] == pytest.approx((s1 - s0) * T * 0.5, rel=1e-13)
    assert gs[0, 2] == pytest.approx((s1 - s0) * T * 0.5, rel=1e-13)
    assert abs(gs[1, 0]) < 1e-15 and abs(gs[1, 1]) < 1e-15


def test_scale_invariance():
    # Scaling sites, origins and tmax by s and sigma by 1/s leaves the image,
    # T and dL/drho = sigma dL/dsigma unchanged; dL/dp scales by 1/s (Sec. 5.4).
    sites, dens, tex, o, w, g, gT = small_problem(3, n=80, k=5)
    s = 2.5
    out = []
    for scale in (1.0, s):
        recs = [render.render_ray(sites * scale, dens / scale, tex, o[r] * scale, w[r], 3.0 * scale)
                for r in range(len(o))]
        grads = adjoint.grad_rays(sites * scale, dens / scale, tex, o * scale, w, 3.0 * scale,
                                  recs, g, gT)
        out.append((recs, grads))
    (ra, (gsa, gda, gta)), (rb, (gsb, gdb, gtb)) = out
    for a, b in zip(ra, rb):
        assert a.cells == b.cells
        np.testing.assert_allclose(a.rgb, b.rgb, rtol=1e-12, atol=1e-15)
        assert a.T == pytest.approx(b.T, rel=1e-12)
    np.testing.assert_allclose(gda * dens, gdb * (dens / s), rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(gsa / s, gsb, rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(gta, gtb, rtol=1e-10, atol=1e-14)


def test_gradients_permute_with_sites():
    sites, dens, tex, o, w, g, gT = small_problem(4, n=70, k=4)
    perm = np.random.default_rng(9).permutation(len(sites))
    ra = [render.render_ray(sites, dens, tex, o[r], w[r], 3.0) for r in range(len(o))]
    ga = adjoint.grad_rays(sites, dens, tex, o, w, 3.0, ra, g, gT)
    rb = [render.render_ray(sites[perm], dens[perm], tex[perm], o[r], w[r], 3.0)
          for r in range(len(o))]
    gb = adjoint.grad_rays(sites[perm], dens[perm], tex[perm], o, w, 3.0, rb, g, gT)
    for x, y in zip(ga, gb):
        np.testing.assert_allclose(x[perm], y, rtol=1e-12, atol=1e-15)
