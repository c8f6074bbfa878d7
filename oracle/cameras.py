"""Ray generation for the camera models of Sec. 6.5 / App. D, FP64.

The paper changes only ray generation for non-pinhole effects: a fisheye
emits the ray its lens model prescribes per pixel, rolling shutter uses a
row-dependent pose, depth of field emits a bundle of aperture rays per pixel
whose colours are averaged.  The concrete models (readings; the paper names
the effects but not their formulas):

* pinhole: f = (W/2) / tan(fov/2) (horizontal FOV), principal point at the
  image centre, pixel centres at (x + 0.5, y + 0.5); camera axes +x right,
  +y down, +z forward; c2w columns are those axes and the centre;
* equidistant fisheye: theta = r / f with f = (W/2) / (fov/2), r the
  pixel-centre distance from the image centre; pixels with theta > fov/2
  emit no ray;
* rolling shutter: row y is exposed with the centre c0 + s * delta,
  s = y / (H - 1), orientation fixed;
* thin lens: spp = g*g stratum-centre samples ((i+0.5)/g, (j+0.5)/g) mapped
  to the unit disk by the concentric map of Shirley and Chiu (1997), scaled
  by the lens radius; every sample of a pixel aims at the pixel's pinhole
  point on the plane z = focus_dist (camera frame).

Ray order: view by view, pixels row-major, then samples.
"""
from __future__ import annotations

import math

import numpy as np


def _pixel_grid(W, H):
    ys, xs = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    return xs.reshape(-1) + 0.5, ys.reshape(-1) + 0.5


def concentric_disk(a, b):
    """Shirley-Chiu concentric square-to-disk map of (a, b) in [0,1]^2."""
    x = 2.0 * a - 1.0
    y = 2.0 * b - 1.0
    if x == 0.0 and y == 0.0:
        return 0.0, 0.0
    if abs(x) > abs(y):
        r, phi = x, (math.pi / 4.0) * (y / x)
    else:
        r, phi = y, math.pi / 2.0 - (math.pi / 4.0) * (x / y)
    return r * math.cos(phi), r * math.sin(phi)


def camera_rays(model, width, height, c2w, fov, tmax, rs_delta=(0.0, 0.0, 0.0),
                lens_radius=0.0, focus_dist=1.0, spp=1):
    """All rays of one view: (origins[R,3], dirs[R,3] unit, tmax[R], valid[R])."""
    W, H = int(width), int(height)
    M = np.asarray(c2w, np.float64)
    Rm, c = M[:, :3], M[:, 3]
    px, py = _pixel_grid(W, H)
    n = W * H
    if model in (0, 2, 3, 4):
        f = (W / 2.0) / math.tan(fov / 2.0)
        dc = np.stack([(px - W / 2.0) / f, (py - H / 2.0) / f, np.ones(n)], 1)
    if model == 0:          # pinhole
        d = dc @ Rm.T
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        o = np.broadcast_to(c, (n, 3)).copy()
        valid = np.ones(n, bool)
    elif model == 1:        # equidistant fisheye
        f = (W / 2.0) / (fov / 2.0)
        dx, dy = px - W / 2.0, py - H / 2.0
        r = np.hypot(dx, dy)
        theta = r / f
        valid = theta <= fov / 2.0
        st = np.sin(theta)
        with np.errstate(invalid="ignore", divide="ignore"):
            ux = np.where(r > 0, dx / r, 0.0)
            uy = np.where(r > 0, dy / r, 0.0)
        dcf = np.stack([st * ux, st * uy, np.cos(theta)], 1)
        d = dcf @ Rm.T
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        o = np.broadcast_to(c, (n, 3)).copy()
    elif model == 2:        # rolling shutter
        s = (py - 0.5) / (H - 1) if H > 1 else np.zeros(n)
        o = c[None, :] + s[:, None] * np.asarray(rs_delta, np.float64)[None, :]
        d = dc @ Rm.T
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        valid = np.ones(n, bool)
    elif model == 3:        # thin lens
        g = int(round(math.sqrt(spp)))
        if g * g != spp:
            raise ValueError("spp must be a square number")
        os_, ds_ = [], []
        focal = dc * focus_dist
        for k in range(spp):
            lx, ly = concentric_disk((k % g + 0.5) / g, (k // g + 0.5) / g)
            L = np.array([lx * lens_radius, ly * lens_radius, 0.0])
            dd = (focal - L) @ Rm.T
            dd /= np.linalg.norm(dd, axis=1, keepdims=True)
            os_.append(np.broadcast_to(c + Rm @ L, (n, 3)))
            ds_.append(dd)
        # order: pixel-major, then sample
        o = np.stack(os_, 1).reshape(n * spp, 3)
        d = np.stack(ds_, 1).reshape(n * spp, 3)
        valid = np.ones(n * spp, bool)
        n = n * spp
    elif model == 4:        # motion blur
        d1 = dc @ Rm.T
        d1 /= np.linalg.norm(d1, axis=1, keepdims=True)
        delta = np.asarray(rs_delta, np.float64)
        os_ = [np.broadcast_to(c + ((k + 0.5) / spp) * delta, (n, 3)) for k in range(spp)]
        o = np.stack(os_, 1).reshape(n * spp, 3)
        d = np.repeat(d1, spp, axis=0)
        valid = np.ones(n * spp, bool)
        n = n * spp
    else:
        raise ValueError(f"unknown camera model {model}")
    tm = np.where(valid, float(tmax), 0.0)
    return o, d, tm, valid


def camera_rays_of(cam):
    """camera_rays for any object with the camera-description attributes."""
    return camera_rays(cam.model, cam.width, cam.height, cam.c2w, cam.fov, cam.tmax,
                       cam.rs_delta, cam.lens_radius, cam.focus_dist, cam.spp)
