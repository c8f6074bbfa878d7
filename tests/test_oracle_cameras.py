"""Pins of the oracle's ray generation (Sec. 6.5, App. D camera effects)."""
import math

import numpy as np
import pytest

from oracle import cameras
from paper_2608_17682_amd import synth


def pose():
    return synth.look_at((0.3, -0.2, -3.0), (0.1, 0.05, 0.0))


def project(c2w, W, H, fov, X):
    """Textbook pinhole projection K [R^T | -R^T c] X with f from the horizontal FOV."""
    R, c = c2w[:, :3], c2w[:, 3]
    f = (W / 2.0) / math.tan(fov / 2.0)
    Xc = (X - c) @ R
    return f * Xc[:, 0] / Xc[:, 2] + W / 2.0, f * Xc[:, 1] / Xc[:, 2] + H / 2.0


def test_pinhole_rays_project_back_to_pixel_centres():
    W, H, fov = 37, 23, math.radians(60)
    M = pose()
    o, d, tm, valid = cameras.camera_rays(0, W, H, M, fov, 6.0)
    assert valid.all() and np.all(tm == 6.0)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    x, y = project(M, W, H, fov, o + 2.0 * d)
    xs, ys = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    np.testing.assert_allclose(x, xs.reshape(-1), atol=1e-10)
    np.testing.assert_allclose(y, ys.reshape(-1), atol=1e-10)


def test_pinhole_horizontal_fov_and_axes():
    # a point at half the FOV to the right projects onto the image's right edge
    W, H, fov = 64, 48, math.radians(60)
    M = synth.look_at((0, 0, -3), (0, 0, 0))
    # 2 units ahead along the axis, turned right by fov/2
    X = (M[:, 3] + 2.0 * (math.tan(fov / 2) * M[:, 0] + M[:, 2]))[None]
    x, y = project(M, W, H, fov, X)
    assert x[0] == pytest.approx(W, abs=1e-9) and y[0] == pytest.approx(H / 2, abs=1e-9)
    # OpenCV axes: image +y is down, i.e. world -y for this upright pose
    assert np.allclose(M[:, 1], [0, -1, 0]) and np.allclose(M[:, 2], [0, 0, 1])
    o, d, _, _ = cameras.camera_rays(0, W, H, M, fov, 6.0)
    top = d[:W].mean(0)
    assert top[1] > 0.1      # the first image row looks up (+y world)


def test_fisheye_equidistant():
    W = H = 65
    M = pose()
    fov = math.pi
    o, d, tm, valid = cameras.camera_rays(1, W, H, M, fov, 8.0)
    axis = M[:, 2]
    centre = (H // 2) * W + W // 2
    np.testing.assert_allclose(d[centre], axis, atol=1e-15)
    xs, ys = np.meshgrid(np.arange(W) + 0.5 - W / 2, np.arange(H) + 0.5 - H / 2)
    r = np.hypot(xs, ys).reshape(-1)
    theta = np.arccos(np.clip(d @ axis, -1, 1))
    # angle from the axis grows linearly with pixel radius, reaching fov/2 at r = W/2
    np.testing.assert_allclose(theta[valid], (r[valid] / (W / 2)) * (fov / 2), atol=1e-12)
    assert np.all(valid == (r <= W / 2))
    assert np.all(tm[~valid] == 0) and np.all(tm[valid] == 8.0)
    assert abs(valid.sum() - math.pi * (W / 2) ** 2) < 2 * math.pi * W / 2


def test_rolling_shutter_rows():
    W, H, fov = 20, 9, math.radians(60)
    M = pose()
    delta = 0.1 * M[:, 0]
    o, d, _, _ = cameras.camera_rays(2, W, H, M, fov, 8.0, rs_delta=delta)
    o0, d0, _, _ = cameras.camera_rays(0, W, H, M, fov, 8.0)
    np.testing.assert_allclose(d, d0, atol=0)
    np.testing.assert_allclose(o[:W], np.broadcast_to(M[:, 3], (W, 3)), atol=1e-15)
    np.testing.assert_allclose(o[-W:], np.broadcast_to(M[:, 3] + delta, (W, 3)), atol=1e-15)
    rows = o.reshape(H, W, 3)[:, 0, :]
    steps = np.diff(rows, axis=0)
    np.testing.assert_allclose(steps, np.broadcast_to(delta / (H - 1), steps.shape), atol=1e-15)


def test_thin_lens():
    W, H, fov, spp = 16, 12, math.radians(60), 4
    M = pose()
    # aperture 0 reduces to the pinhole exactly
    o, d, _, _ = cameras.camera_rays(3, W, H, M, fov, 8.0, lens_radius=0.0, focus_dist=3.0,
                                     spp=spp)
    o0, d0, _, _ = cameras.camera_rays(0, W, H, M, fov, 8.0)
    np.testing.assert_allclose(d.reshape(-1, spp, 3), np.repeat(d0[:, None], spp, 1), atol=1e-15)
    np.testing.assert_allclose(o, np.broadcast_to(M[:, 3], o.shape), atol=1e-15)
    # every lens sample of a pixel meets the pixel's focal point on the plane z_cam = 3
    o, d, _, _ = cameras.camera_rays(3, W, H, M, fov, 8.0, lens_radius=0.05, focus_dist=3.0,
                                     spp=spp)
    R, c = M[:, :3], M[:, 3]
    oc = (o - c) @ R
    dc = d @ R
    t = (3.0 - oc[:, 2]) / dc[:, 2]
    hit = (oc + t[:, None] * dc).reshape(-1, spp, 3)
    np.testing.assert_allclose(hit, np.repeat(hit[:, :1], spp, 1), atol=1e-13)
    focal0 = (d0 @ R) * (3.0 / (d0 @ R)[:, 2:3])
    np.testing.assert_allclose(hit[:, 0], focal0, atol=1e-13)
    # lens points lie in the lens disk on the z_cam = 0 plane
    assert np.all(np.abs(oc[:, 2]) < 1e-15)
    assert np.all(np.hypot(oc[:, 0], oc[:, 1]) <= 0.05 + 1e-15)


def test_concentric_disk_map():
    # The concentric map sends the square ring max(|2a-1|, |2b-1|) = r onto the
    # circle of radius r, and keeps the quadrant.
    rng = np.random.default_rng(0)
    for _ in range(200):
        a, b = rng.uniform(size=2)
        x, y = cameras.concentric_disk(a, b)
        assert math.hypot(x, y) == pytest.approx(max(abs(2 * a - 1), abs(2 * b - 1)), abs=1e-14)
        assert (x >= 0) == (2 * a - 1 >= 0) or abs(x) < 1e-14
        assert (y >= 0) == (2 * b - 1 >= 0) or abs(y) < 1e-14
    assert cameras.concentric_disk(0.5, 0.5) == (0.0, 0.0)
    x, y = cameras.concentric_disk(1.0, 0.5)
    assert x == pytest.approx(1.0) and y == pytest.approx(0.0, abs=1e-15)


def test_motion_blur_samples_are_pinholes_at_moved_centres():
    # sample s of a pixel is the pinhole ray of the camera moved to
    # c + (s + 0.5)/spp * delta; delta = 0 repeats the pinhole ray spp times
    W, H, fov, spp = 9, 7, math.radians(60), 5
    M = pose()
    delta = np.array([0.2, -0.1, 0.05])
    o, d, tm, valid = cameras.camera_rays(4, W, H, M, fov, 6.0, rs_delta=delta, spp=spp)
    assert len(o) == W * H * spp and valid.all()
    for s in range(spp):
        Ms = M.copy()
        Ms[:, 3] = M[:, 3] + (s + 0.5) / spp * delta
        op, dp, _, _ = cameras.camera_rays(0, W, H, Ms, fov, 6.0)
        np.testing.assert_allclose(o[s::spp], op, atol=1e-15)
        np.testing.assert_allclose(d[s::spp], dp, atol=1e-15)
    o0, d0, _, _ = cameras.camera_rays(4, W, H, M, fov, 6.0, spp=3)
    op, dp, _, _ = cameras.camera_rays(0, W, H, M, fov, 6.0)
    np.testing.assert_array_equal(o0, np.repeat(op, 3, 0))
    np.testing.assert_array_equal(d0, np.repeat(dp, 3, 0))
    # the middle sample of an odd count sits at mid-exposure
    np.testing.assert_allclose(o[2], M[:, 3] + 0.5 * delta, atol=1e-15)
