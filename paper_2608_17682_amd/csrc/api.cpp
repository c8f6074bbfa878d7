// Host-only part of the C ABI: version, errors, defaults, argument checks,
// workspace sizing.  None of these functions touches a device unless stated.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "host_common.hpp"
#include "voro.h"

namespace voro {

static thread_local char g_err[512] = {0};

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = 0; }

voro_status fail(voro_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

voro_status check_scene(const voro_scene* s) {
  if (!s) return fail(VORO_EINVAL, "scene is NULL");
  if (s->n_sites < 1) return fail(VORO_EINVAL, "n_sites must be >= 1 (got %d)", s->n_sites);
  if (s->tex_res < VORO_MIN_TEX_RES || s->tex_res > VORO_MAX_TEX_RES)
    return fail(VORO_EINVAL, "tex_res %d outside [%d, %d]", s->tex_res, VORO_MIN_TEX_RES,
                VORO_MAX_TEX_RES);
  if (s->tex_dtype != VORO_TEX_F32 && s->tex_dtype != VORO_TEX_F16 &&
      s->tex_dtype != VORO_TEX_BF16)
    return fail(VORO_EINVAL, "unknown tex_dtype %d", s->tex_dtype);
  if (s->tex_maps < 0 || s->tex_maps > 3)
    return fail(VORO_EINVAL, "tex_maps must be 0, 1, 2 or 3 (got %d)", s->tex_maps);
  if (s->n_edges < 0 || s->n_edges >= ((int64_t)1 << 31))
    return fail(VORO_EINVAL, "n_edges %lld out of range [0, 2^31)", (long long)s->n_edges);
  if (!s->sites || !s->density || !s->nbr_off || !s->texels)
    return fail(VORO_EINVAL, "scene has a NULL array");
  if (s->n_edges > 0 && !s->nbr_idx) return fail(VORO_EINVAL, "nbr_idx is NULL");
  if (!aligned(s->sites, 4) || !aligned(s->density, 4) || !aligned(s->nbr_off, 4) ||
      (s->nbr_idx && !aligned(s->nbr_idx, 4)))
    return fail(VORO_EINVAL, "scene arrays must be 4-byte aligned");
  const size_t ta = s->tex_dtype == VORO_TEX_F32 ? 16 : 8;
  if (!aligned(s->texels, ta))
    return fail(VORO_EINVAL, "texels must be %zu-byte aligned", ta);
  return VORO_OK;
}

voro_status check_ws(const voro_scene* s, const void* ws, size_t ws_bytes) {
  if (!ws) return fail(VORO_EWORKSPACE, "workspace is NULL");
  if (!aligned(ws, 256)) return fail(VORO_EINVAL, "workspace must be 256-byte aligned");
  const WsLayout L = ws_layout(s->n_sites, s->n_edges);
  if (ws_bytes < L.total)
    return fail(VORO_EWORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  return VORO_OK;
}

voro_status check_params(const voro_params* p, bool backward) {
  if (!p) return fail(VORO_EINVAL, "params is NULL");
  if (!(p->t_stop >= 0.0f) || !std::isfinite(p->t_stop))
    return fail(VORO_EINVAL, "t_stop must be finite and >= 0");
  if (!(p->skip_w >= 0.0f) || !std::isfinite(p->skip_w))
    return fail(VORO_EINVAL, "skip_w must be finite and >= 0");
  if (backward && p->skip_w != 0.0f)
    return fail(VORO_EINVAL, "the adjoint needs skip_w == 0 (skipped lookups have no gradient)");
  if (p->max_steps < 1) return fail(VORO_EINVAL, "max_steps must be >= 1");
  if (!(p->tie_window >= 0.0f) || !std::isfinite(p->tie_window))
    return fail(VORO_EINVAL, "tie_window must be finite and >= 0");
  if (p->appearance < 0 || p->appearance > 2)
    return fail(VORO_EUNSUPPORTED, "appearance %d not built (0 = ray-direction texture, "
                "1 = surface + view maps, 2 = degree-3 spherical harmonics)", p->appearance);
  if (backward && p->appearance == 2)
    return fail(VORO_EUNSUPPORTED, "the spherical-harmonic comparison model is forward only");
  const int l = p->lanes_per_ray;
  if (!(l == 0 || l == 1 || l == 2 || l == 4 || l == 8 || l == 16))
    return fail(VORO_EINVAL, "lanes_per_ray must be 0, 1, 2, 4, 8 or 16");
  if (p->tile_w < 0 || p->tile_h < 0) return fail(VORO_EINVAL, "tile sizes must be >= 0");
  if ((p->tile_w == 0) != (p->tile_h == 0))
    return fail(VORO_EINVAL, "tile_w and tile_h must both be 0 or both be set");
  if (p->tile_w > 0) {
    const int lpr = l == 0 ? 1 : l;
    if (p->tile_w * p->tile_h * lpr != 64)
      return fail(VORO_EINVAL, "tile_w * tile_h * lanes_per_ray must be 64");
  }
  if (p->img_w < 0) return fail(VORO_EINVAL, "img_w must be >= 0");
  if (p->max_record < 0) return fail(VORO_EINVAL, "max_record must be >= 0");
  if (!(p->block == 0 || p->block == 64 || p->block == 128 || p->block == 256))
    return fail(VORO_EINVAL, "block must be 0, 64, 128 or 256");
  if (p->schedule < VORO_SCHEDULE_DEFAULT || p->schedule > VORO_SCHEDULE_REFILL)
    return fail(VORO_EINVAL, "unknown schedule %d", p->schedule);
  if (p->edge_fp16 != 0 && p->edge_fp16 != 1)
    return fail(VORO_EINVAL, "edge_fp16 must be 0 or 1");
  if (p->edge_fp16 && backward)
    return fail(VORO_EUNSUPPORTED, "edge_fp16 is a forward-only inference variant");
  if (p->edge_fp16 && !(p->lanes_per_ray == 0 || p->lanes_per_ray == 1))
    return fail(VORO_EUNSUPPORTED, "edge_fp16 needs one lane per ray");
  for (int i = 0; i < 3; ++i)
    if (p->reserved[i] != 0) return fail(VORO_EINVAL, "params.reserved must be 0");
  return VORO_OK;
}

// The texel layout must match the appearance model, and gradient record
// keys (cell * maps + map) * R^2 + quad must fit an int.
voro_status check_appearance(const voro_scene* s, const voro_params* p) {
  if (s->tex_maps == 3 || p->appearance == 2) {
    if (s->tex_maps != 3 || p->appearance != 2)
      return fail(VORO_EINVAL, "spherical-harmonic coefficients (tex_maps = 3) go with "
                  "appearance 2 and only with it");
    if (!aligned(s->texels, 16))
      return fail(VORO_EINVAL, "spherical-harmonic coefficients must be 16-byte aligned");
    return VORO_OK;
  }
  const int maps = s->tex_maps == 2 ? 2 : 1;
  if (p->appearance == 1 && maps != 2)
    return fail(VORO_EINVAL, "appearance 1 needs two texture maps per cell (tex_maps = 2)");
  if (p->appearance == 0 && maps != 1)
    return fail(VORO_EINVAL, "appearance 0 needs one texture map per cell (tex_maps = 0 or 1)");
  if ((int64_t)s->n_sites * maps * s->tex_res * s->tex_res >= ((int64_t)1 << 31))
    return fail(VORO_EINVAL, "n_sites * tex_maps * tex_res^2 must be < 2^31");
  return VORO_OK;
}

Launch resolve_launch(const voro_params* p) {
  Launch L;
  L.lpr = p->lanes_per_ray == 0 ? 1 : p->lanes_per_ray;
  L.block = p->block == 0 ? 256 : p->block;
  if (p->tile_w > 0) {
    L.tile_w = p->tile_w;
    L.tile_h = p->tile_h;
  } else {
    // square-ish default tile of 64 / lpr rays
    const int rays = 64 / L.lpr;
    int w = 1;
    while (w * w < rays) w <<= 1;
    L.tile_w = w;
    L.tile_h = rays / w;
  }
  return L;
}

voro_status check_cameras(const voro_camera* cams, int32_t V, int64_t* n_rays,
                          int64_t* n_pixels) {
  if (!cams) return fail(VORO_EINVAL, "cameras is NULL");
  if (V < 1 || V > VORO_MAX_VIEWS)
    return fail(VORO_EINVAL, "V must be in [1, %d] (got %d)", VORO_MAX_VIEWS, V);
  int64_t nr = 0, np = 0;
  for (int v = 0; v < V; ++v) {
    const voro_camera& c = cams[v];
    if (c.model < VORO_CAM_PINHOLE || c.model > VORO_CAM_MOTION_BLUR)
      return fail(VORO_EINVAL, "camera %d: unknown model %d", v, c.model);
    if (c.width < 1 || c.height < 1 || c.width > 65536 || c.height > 65536)
      return fail(VORO_EINVAL, "camera %d: bad size %dx%d", v, c.width, c.height);
    if (c.model == VORO_CAM_ROLLING_SHUTTER && c.height < 2)
      return fail(VORO_EINVAL, "camera %d: rolling shutter needs height >= 2", v);
    if (c.model == VORO_CAM_THIN_LENS) {
      const int g = (int)std::lround(std::sqrt((double)c.spp));
      if (c.spp < 1 || c.spp > 64 || g * g != c.spp)
        return fail(VORO_EINVAL, "camera %d: spp must be a square number in [1, 64]", v);
      if (!(c.lens_radius >= 0.0f) || !(c.focus_dist > 0.0f))
        return fail(VORO_EINVAL, "camera %d: need lens_radius >= 0 and focus_dist > 0", v);
    } else if (c.model == VORO_CAM_MOTION_BLUR) {
      if (c.spp < 1 || c.spp > 64)
        return fail(VORO_EINVAL, "camera %d: spp must be in [1, 64] for motion blur", v);
    } else if (c.spp != 1) {
      return fail(VORO_EINVAL, "camera %d: spp must be 1 for this model", v);
    }
    const float maxfov = c.model == VORO_CAM_FISHEYE ? 6.2831853f : 3.1415926f;
    if (!(c.fov > 0.0f) || !(c.fov < maxfov))
      return fail(VORO_EINVAL, "camera %d: fov out of range", v);
    if (!(c.tmax > 0.0f) || !std::isfinite(c.tmax))
      return fail(VORO_EINVAL, "camera %d: tmax must be finite and > 0", v);
    for (int i = 0; i < 12; ++i)
      if (!std::isfinite(c.c2w[i])) return fail(VORO_EINVAL, "camera %d: c2w not finite", v);
    if (c.reserved != 0) return fail(VORO_EINVAL, "camera %d: reserved must be 0", v);
    np += (int64_t)c.width * c.height;
    nr += (int64_t)c.width * c.height * c.spp;
  }
  if (nr >= ((int64_t)1 << 31)) return fail(VORO_EINVAL, "too many rays (%lld)", (long long)nr);
  if (n_rays) *n_rays = nr;
  if (n_pixels) *n_pixels = np;
  return VORO_OK;
}

voro_status check_device() {
  static std::atomic<int> ok{0};
  if (ok.load(std::memory_order_relaxed)) return VORO_OK;
  int n = 0;
  const hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n < 1) {
    (void)hipGetLastError();
    return fail(VORO_ENODEV, "no HIP device (%s)", e == hipSuccess ? "count 0" : hipGetErrorString(e));
  }
  ok.store(1, std::memory_order_relaxed);
  return VORO_OK;
}

voro_status check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(VORO_EHIP, "%s: %s", what, hipGetErrorString(e));
  return VORO_OK;
}

}  // namespace voro

using namespace voro;

extern "C" {

const char* voro_version(void) { return "voro 0.1.0 gfx950"; }

const char* voro_last_error(void) { return g_err; }

voro_status voro_default_params(voro_params* p) {
  if (!p) return fail(VORO_EINVAL, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->t_stop = 1e-4f;
  p->skip_w = 0.0f;
  p->max_steps = 4096;
  p->tie_window = 1e-6f;
  p->appearance = 0;
  return VORO_OK;
}

voro_status voro_workspace_size(const voro_scene* scene, size_t* bytes) {
  voro_status st = check_scene(scene);
  if (st != VORO_OK) return st;
  if (!bytes) return fail(VORO_EINVAL, "bytes is NULL");
  *bytes = ws_layout(scene->n_sites, scene->n_edges).total;
  return VORO_OK;
}

voro_status voro_camera_counts(const voro_camera* cams, int32_t V, int64_t* n_rays,
                               int64_t* n_pixels) {
  return check_cameras(cams, V, n_rays, n_pixels);
}

}  // extern "C"
