// Host-side helpers shared by the C entry points: error reporting, argument
// validation, workspace layout and launch checks.  No device code.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>

#include "voro.h"

namespace voro {

// thread-local last-error text (defined in api.cpp)
void set_error(const char* fmt, ...);
void clear_error();

voro_status fail(voro_status st, const char* fmt, ...);

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace layout: cell records, edge records (FP32, then a half copy of the
// edge vectors), nearest-site partials, persistent-launch counters and
// per-view start cells, and the adjoint's per-cell accumulator of position
// and density gradients (one float4 per cell, zero between adjoint calls).
constexpr int kLocateBruteMax = 64;    // origins searched by brute force
constexpr int kLocateChunks = 256;     // max partial results per origin
struct WsLayout {
  size_t cells, edges, edges16, locate, counters, cellg, total;
};

inline WsLayout ws_layout(int32_t n, int64_t m) {
  WsLayout L;
  L.cells = 0;
  L.edges = align256((size_t)n * 32);
  L.edges16 = align256(L.edges + (size_t)m * 16);
  L.locate = align256(L.edges16 + (size_t)m * 8 + 16);
  L.counters = align256(L.locate + (size_t)kLocateBruteMax * kLocateChunks * 16);
  L.cellg = align256(L.counters + 4096);
  L.total = align256(L.cellg + (size_t)n * 16);
  return L;
}

// adds the workspace's per-cell accumulator into g_sites / g_density and
// clears it (stream-ordered after an adjoint kernel; defined in walk.hip)
voro_status launch_fold_cell_grads(const voro_scene* scene, void* ws, float* g_sites,
                                   float* g_density, hipStream_t st);

voro_status check_scene(const voro_scene* s);
voro_status check_ws(const voro_scene* s, const void* ws, size_t ws_bytes);
voro_status check_params(const voro_params* p, bool backward);
voro_status check_appearance(const voro_scene* s, const voro_params* p);
voro_status check_cameras(const voro_camera* cams, int32_t V, int64_t* n_rays, int64_t* n_pixels);
voro_status check_device();
voro_status check_launch(const char* what);

inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

// stored-exit arguments: a capacity of at least one step, 8-byte alignment
inline voro_status check_trace(const int32_t* trace, int32_t trace_cap) {
  if (!trace) return VORO_OK;
  if (trace_cap < 1) return fail(VORO_EINVAL, "trace_cap = %d: must be >= 1 with a trace", trace_cap);
  if (!aligned(trace, 8)) return fail(VORO_EINVAL, "trace must be 8-byte aligned");
  return VORO_OK;
}

// effective launch parameters after defaults
struct Launch {
  int lpr, tile_w, tile_h, block;
};
Launch resolve_launch(const voro_params* p);

}  // namespace voro
