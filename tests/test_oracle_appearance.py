"""Pins of the octahedral map and bilinear lookup (Sec. 5.1)."""
import math

import numpy as np
import pytest

from oracle import appearance


def unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("d,uv", [
    ((1, 0, 0), (1, 0)), ((-1, 0, 0), (-1, 0)),
    ((0, 1, 0), (0, 1)), ((0, -1, 0), (0, -1)),
    ((0, 0, 1), (0, 0)), ((0, 0, -1), (1, 1)),   # sign(0) = +1 puts -z at the (+,+) corner
])
def test_axis_directions(d, uv):
    assert appearance.octahedral(d) == pytest.approx(uv, abs=0)


def test_hemisphere_branches_agree_on_equator():
    # On d_z = 0 the lower-hemisphere unfold reduces to the upper branch,
    # so the map is continuous across the equator.
    for ang in np.linspace(0, 2 * math.pi, 37):
        d = np.array([math.cos(ang), math.sin(ang), 0.0])
        u0, v0 = appearance.octahedral(d)
        u1, v1 = appearance.octahedral(d + np.array([0, 0, -1e-13]))
        assert abs(u0 - u1) < 1e-12 and abs(v0 - v1) < 1e-12


def test_octahedron_faces_land_in_expected_regions():
    rng = np.random.default_rng(0)
    for _ in range(200):
        d = unit(rng.normal(size=3))
        u, v = appearance.octahedral(d)
        assert -1 <= u <= 1 and -1 <= v <= 1
        inner = abs(u) + abs(v) <= 1 + 1e-12
        assert inner == (d[2] >= 0) or abs(abs(u) + abs(v) - 1) < 1e-12
        # the unfold keeps the quadrant of (d_x, d_y)
        assert (u >= 0) == (d[0] >= 0) or abs(u) < 1e-12
        assert (v >= 0) == (d[1] >= 0) or abs(v) < 1e-12


def test_map_is_injective_on_samples():
    rng = np.random.default_rng(1)
    ds = [unit(rng.normal(size=3)) for _ in range(300)]
    uvs = np.array([appearance.octahedral(d) for d in ds])
    for a in range(len(ds)):
        for b in range(a + 1, len(ds)):
            if np.linalg.norm(ds[a] - ds[b]) > 1e-6:
                assert np.linalg.norm(uvs[a] - uvs[b]) > 1e-9


def test_constant_texture_constant_colour():
    tex = np.zeros((8, 8, 4))
    tex[..., :3] = (0.2, 0.5, 0.9)
    rng = np.random.default_rng(2)
    for _ in range(50):
        np.testing.assert_allclose(appearance.lookup(tex, unit(rng.normal(size=3))),
                                   (0.2, 0.5, 0.9), atol=1e-15)


def test_texel_centres_return_the_texel():
    # Corner-aligned reading: on an R x R texture, u = -1 + 2c/(R-1) is column c.
    R = 5
    tex = np.random.default_rng(3).uniform(size=(R, R, 4))
    # upper hemisphere: q = (0.5, 0, 0.5) -> (u, v) = (0.5, 0) -> column 3, row 2
    np.testing.assert_allclose(appearance.lookup(tex, unit([0.5, 0.0, 0.5])), tex[2, 3, :3],
                               atol=1e-14)
    # q = (-0.5, 0.5, 0) -> (u, v) = (-0.5, 0.5) -> column 1, row 3
    np.testing.assert_allclose(appearance.lookup(tex, unit([-0.5, 0.5, 0.0])), tex[3, 1, :3],
                               atol=1e-14)
    # lower hemisphere: q = (0.25, 0.25, -0.5) -> (0.75, 0.75); on R = 9 that is texel (7, 7)
    tex9 = np.random.default_rng(4).uniform(size=(9, 9, 4))
    np.testing.assert_allclose(appearance.lookup(tex9, unit([0.25, 0.25, -0.5])), tex9[7, 7, :3],
                               atol=1e-14)
    # -z lands on the last row and column
    np.testing.assert_allclose(appearance.lookup(tex9, [0, 0, -1]), tex9[8, 8, :3], atol=0)


def test_texture_linear_in_rows_and_columns_is_reproduced():
    # Bilinear interpolation reproduces any texture affine in (column, row):
    # distinct slopes catch a transposed or flipped index.
    R = 8
    rows, cols = np.meshgrid(np.arange(R), np.arange(R), indexing="ij")
    tex = np.zeros((R, R, 4))
    tex[..., 0] = 0.1 + 0.03 * cols + 0.07 * rows
    tex[..., 1] = 0.9 - 0.05 * cols
    tex[..., 2] = 0.2 + 0.11 * rows
    rng = np.random.default_rng(5)
    for _ in range(100):
        d = unit(rng.normal(size=3))
        u, v = appearance.octahedral(d)
        col = (u + 1) / 2 * (R - 1)
        row = (v + 1) / 2 * (R - 1)
        want = [0.1 + 0.03 * col + 0.07 * row, 0.9 - 0.05 * col, 0.2 + 0.11 * row]
        np.testing.assert_allclose(appearance.lookup(tex, d), want, atol=1e-13)


def test_bilinear_weights_partition_of_unity_and_continuity():
    rng = np.random.default_rng(6)
    for _ in range(100):
        d = unit(rng.normal(size=3))
        taps = appearance.bilinear_weights(d, 6)
        assert abs(sum(t[2] for t in taps) - 1) < 1e-14
        assert all(t[2] >= -1e-15 for t in taps)
    # across a texel boundary the colour is continuous
    tex = np.random.default_rng(7).uniform(size=(4, 4, 4))
    # u crosses the column boundary at u = -1/3 (column 1 for R = 4)
    for eps in (1e-9, -1e-9):
        d = unit([-1 / 3 + eps, 0.1, 1 - 1 / 3 - 0.1])
        c = appearance.lookup(tex, d)
        d0 = unit([-1 / 3, 0.1, 1 - 1 / 3 - 0.1])
        np.testing.assert_allclose(c, appearance.lookup(tex, d0), atol=1e-7)
