// Ray generation per camera model (Sec. 6.5 / App. D: only ray generation
// changes between pinhole, fisheye, rolling shutter, depth of field and
// motion blur).
// One device function serves voro_gen_rays and the persistent multi-view
// kernels, so both produce bit-identical rays.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "voro.h"
#include "voro_device.hpp"

namespace voro {

struct CamTable {
  voro_camera cam[VORO_MAX_VIEWS];
  int ray_off[VORO_MAX_VIEWS + 1];   // first ray of each view
  int pix_off[VORO_MAX_VIEWS + 1];   // first pixel of each view
  int tile_off[VORO_MAX_VIEWS + 1];  // first work tile of each view (persistent launch)
  int g[VORO_MAX_VIEWS];             // thin lens: samples per pixel side (spp = g*g)
  int gx[VORO_MAX_VIEWS];            // a pixel's samples laid out as a gx x gy block
  int gy[VORO_MAX_VIEWS];            // of the view's sample grid (spp = gx*gy)
  float focal[VORO_MAX_VIEWS];       // focal length in pixels (camera_focal)
  int V;
};

// Shirley-Chiu concentric map of (a, b) in [0,1]^2 to the unit disk.
__device__ __forceinline__ void concentric(float a, float b, float& x, float& y) {
  const float sx = 2.0f * a - 1.0f;
  const float sy = 2.0f * b - 1.0f;
  if (sx == 0.0f && sy == 0.0f) {
    x = 0.0f;
    y = 0.0f;
    return;
  }
  const float q = 0.78539816339744831f;  // pi/4
  float r, phi;
  if (fabsf(sx) > fabsf(sy)) {
    r = sx;
    phi = q * (sy / sx);
  } else {
    r = sy;
    phi = 2.0f * q - q * (sx / sy);
  }
  float sn, cs;
  sincosf(phi, &sn, &cs);
  x = r * cs;
  y = r * sn;
}

// Focal length in pixels, once per view on the host: (W/2) / (fov/2) for
// the equidistant fisheye (theta = r / f), (W/2) / tan(fov/2) otherwise
// (evaluated in FP64 and rounded once).  Kept out of the kernels so that no
// per-ray tangent (and its constants) competes for registers with the walk.
static inline float camera_focal(const voro_camera& c) {
  const float W = (float)c.width;
  if (c.model == VORO_CAM_FISHEYE) return (0.5f * W) / (0.5f * c.fov);
  return (float)((0.5 * (double)W) / std::tan(0.5 * (double)c.fov));
}

// Ray of pixel (px, py), sample s of camera c with focal length f (pixels,
// camera_focal).  Returns false (tmax = 0) for fisheye pixels outside the
// image circle.
__device__ __forceinline__ bool gen_ray(const voro_camera& c, int g, float f, int px, int py,
                                        int s, float& ox, float& oy, float& oz, float& dx,
                                        float& dy, float& dz, float& tmax) {
  const float* M = c.c2w;
  const float W = (float)c.width;
  const float H = (float)c.height;
  const float u = ((float)px + 0.5f) - 0.5f * W;
  const float v = ((float)py + 0.5f) - 0.5f * H;
  ox = M[3];
  oy = M[7];
  oz = M[11];
  float cx, cy, cz;
  bool valid = true;
  if (c.model == VORO_CAM_FISHEYE) {
    const float r2 = u * u + v * v;  // exact on the half-integer pixel grid
    valid = r2 <= 0.25f * W * W;
    const float r = sqrtf(r2);
    const float th = r / f;
    float st, ct;
    sincosf(th, &st, &ct);
    if (r > 0.0f) {
      cx = st * (u / r);
      cy = st * (v / r);
    } else {
      cx = 0.0f;
      cy = 0.0f;
    }
    cz = ct;
  } else {
    const float x = u / f;
    const float y = v / f;
    if (c.model == VORO_CAM_THIN_LENS) {
      const float a = ((float)(s % g) + 0.5f) / (float)g;
      const float b = ((float)(s / g) + 0.5f) / (float)g;
      float lx, ly;
      concentric(a, b, lx, ly);
      lx *= c.lens_radius;
      ly *= c.lens_radius;
      cx = c.focus_dist * x - lx;
      cy = c.focus_dist * y - ly;
      cz = c.focus_dist;
      ox = ox + (M[0] * lx + M[1] * ly);
      oy = oy + (M[4] * lx + M[5] * ly);
      oz = oz + (M[8] * lx + M[9] * ly);
    } else {
      cx = x;
      cy = y;
      cz = 1.0f;
    }
    if (c.model == VORO_CAM_ROLLING_SHUTTER || c.model == VORO_CAM_MOTION_BLUR) {
      // rolling shutter: the row's exposure time; motion blur: the sample's
      const float sr = c.model == VORO_CAM_ROLLING_SHUTTER
                           ? (float)py / (H - 1.0f)
                           : ((float)s + 0.5f) / (float)c.spp;
      ox = fmaf(sr, c.rs_delta[0], ox);
      oy = fmaf(sr, c.rs_delta[1], oy);
      oz = fmaf(sr, c.rs_delta[2], oz);
    }
  }
  dx = fmaf(M[2], cz, fmaf(M[1], cy, M[0] * cx));
  dy = fmaf(M[6], cz, fmaf(M[5], cy, M[4] * cx));
  dz = fmaf(M[10], cz, fmaf(M[9], cy, M[8] * cx));
  const float inv = 1.0f / sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
  dx *= inv;
  dy *= inv;
  dz *= inv;
  tmax = valid ? c.tmax : 0.0f;
  return valid;
}

// the view holding global index i given the prefix offsets off[0..V]
__device__ __forceinline__ int find_view(const int* off, int V, int i) {
  int v = 0;
  while (v + 1 < V && i >= off[v + 1]) ++v;
  return v;
}

}  // namespace voro
