"""Pins of the oracle's spherical-harmonic colour (Sec. 3.3): agreement with
scipy's complex spherical harmonics (an independent library definition),
orthonormality on the sphere by quadrature, textbook special values, and a
constant-colour closed form through the renderer."""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import render, sh
from paper_2608_17682_amd import synth


def complex_sh(l, m, polar, azim):
    if hasattr(sp, "sph_harm_y"):
        return sp.sph_harm_y(l, m, polar, azim)
    return sp.sph_harm(m, l, azim, polar)


def test_matches_scipy_complex_harmonics():
    # real Y_l^m = sqrt(2) (-1)^m Re Y_l^m (m > 0), sqrt(2) (-1)^m Im Y_l^|m| (m < 0)
    rng = np.random.default_rng(0)
    for _ in range(50):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        polar, azim = math.acos(d[2]), math.atan2(d[1], d[0])
        got = sh.real_sh(d)
        for l in range(4):
            for m in range(-l, l + 1):
                y = complex_sh(l, abs(m), polar, azim)
                if m == 0:
                    want = y.real
                elif m > 0:
                    want = math.sqrt(2) * (-1) ** m * y.real
                else:
                    want = math.sqrt(2) * (-1) ** m * y.imag
                assert got[l * l + l + m] == pytest.approx(want, abs=1e-12), (l, m)


def test_orthonormal_on_the_sphere():
    x, wx = np.polynomial.legendre.leggauss(12)     # exact for the degree-6 products
    n_phi = 16
    G = np.zeros((16, 16))
    for ct, w in zip(x, wx):
        st = math.sqrt(1 - ct * ct)
        for k in range(n_phi):
            ph = 2 * math.pi * k / n_phi
            y = sh.real_sh([st * math.cos(ph), st * math.sin(ph), ct])
            G += w * (2 * math.pi / n_phi) * np.outer(y, y)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_textbook_values():
    c0 = 0.5 / math.sqrt(math.pi)
    c1 = math.sqrt(3 / (4 * math.pi))
    assert sh.real_sh([0, 0, 1])[0] == pytest.approx(c0, rel=1e-15)
    assert sh.real_sh([0, 0, 1])[2] == pytest.approx(c1, rel=1e-14)      # Y_1^0 at +z
    assert sh.real_sh([1, 0, 0])[3] == pytest.approx(c1, rel=1e-14)      # Y_1^1 at +x
    assert sh.real_sh([0, 1, 0])[1] == pytest.approx(c1, rel=1e-14)      # Y_1^-1 at +y
    # Y_2^0 at +z: sqrt(5/(16 pi)) (3 - 1)
    assert sh.real_sh([0, 0, 1])[6] == pytest.approx(math.sqrt(5 / (16 * math.pi)) * 2, rel=1e-14)


def test_constant_colour_through_the_renderer():
    scene = synth.scene_uniform(50, 2, seed=6)
    k = np.zeros((50, 48))
    rgb0 = np.array([0.2, 0.5, 0.9])
    k[:, 0:3] = rgb0 / (0.5 / math.sqrt(math.pi))     # only the l = 0 term
    rng = np.random.default_rng(3)
    for _ in range(5):
        o = rng.uniform(-0.7, 0.7, 3)
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        rec = render.render_ray(scene.sites, scene.density, k, o, w, 3.0, appearance=2)
        np.testing.assert_allclose(rec.rgb, (1 - rec.T) * rgb0, rtol=1e-12, atol=1e-15)
