// Scene packing, forward walk and its adjoint (explicit rays).
//
// Sec. 3.1: from the cell holding the origin, repeatedly cross the nearest
// forward bisector between the current site and its Delaunay neighbours.
// Sec. 3.2: per visited cell alpha = 1 - exp(-sigma delta), front-to-back
// compositing C = sum T_k alpha_k c_k, stop once T falls below t_stop.
// Sec. 5.1: c_k is the cell's octahedral texture sampled bilinearly at the
// ray direction.  Sec. 5.6: the low-weight texel lookup may be skipped.
#include <hip/hip_runtime.h>

#include "host_common.hpp"
#include "voro_device.hpp"
#include "walk_impl.hpp"

namespace voro {

// ------------------------------------------------------------------ prepare
// 16 lanes per cell: lane 0 writes the cell record, all 16 stride over the
// cell's row writing edge records (coalesced 256-byte runs).  Rows keep the
// adjacency's own offsets: compact, so the walk's working set is as small
// as the adjacency.
struct PrepArgs {
  const float* sites;
  const float* density;
  const int32_t* nbr_off;
  const int32_t* nbr_idx;
  int n;
  int m;
  float4* cells;
  float4* edges;
  uint2* edges16;
  float4* cellg;  // the adjoint's per-cell accumulator, cleared here
  unsigned long long* stats;
};

__global__ void __launch_bounds__(256) k_prepare(PrepArgs a) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long cell = gid >> 4;
  const int l16 = threadIdx.x & 15;
  if (cell >= a.n) return;
  const int i = (int)cell;
  const int off = a.nbr_off[i];
  const int end = a.nbr_off[i + 1];
  const bool bad_row = off < 0 || end < off || end > a.m;
  const int deg = bad_row ? 0 : end - off;
  const float px = a.sites[3 * (size_t)i];
  const float py = a.sites[3 * (size_t)i + 1];
  const float pz = a.sites[3 * (size_t)i + 2];
  if (l16 == 0) {
    a.cells[2 * (size_t)i] = make_float4(px, py, pz, a.density[i]);
    a.cells[2 * (size_t)i + 1] = make_float4(__int_as_float(bad_row ? 0 : off),
                                             __int_as_float(deg), 0.0f, 0.0f);
    a.cellg[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (bad_row && a.stats) atomicAdd(&a.stats[VORO_STAT_BAD_CSR], 1ull);
  }
  if (bad_row) return;
  for (int e = l16; e < deg; e += 16) {
    // null record: m = 0 gives m.w = 0, which no exit search accepts
    float4 E = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(i));
    {
      const int j = a.nbr_idx[off + e];
      if (j < 0 || j >= a.n || j == i) {
        if (a.stats) atomicAdd(&a.stats[VORO_STAT_BAD_CSR], 1ull);
      } else {
        const double nx = (double)a.sites[3 * (size_t)j] - (double)px;
        const double ny = (double)a.sites[3 * (size_t)j + 1] - (double)py;
        const double nz = (double)a.sites[3 * (size_t)j + 2] - (double)pz;
        const double nn = nx * nx + ny * ny + nz * nz;
        E.w = __int_as_float(j);
        if (nn > 0.0) {  // coincident sites share no face: keep the null vector
          const double inv = 1.0 / nn;
          E.x = (float)(nx * inv);
          E.y = (float)(ny * inv);
          E.z = (float)(nz * inv);
        }
      }
    }
    a.edges[off + e] = E;
    // half copy (round to nearest even; magnitudes clamped to the f16 range)
    const _Float16 hx = (_Float16)fminf(fmaxf(E.x, -65504.0f), 65504.0f);
    const _Float16 hy = (_Float16)fminf(fmaxf(E.y, -65504.0f), 65504.0f);
    const _Float16 hz = (_Float16)fminf(fmaxf(E.z, -65504.0f), 65504.0f);
    a.edges16[off + e] =
        make_uint2((unsigned)__builtin_bit_cast(uint16_t, hx) |
                       ((unsigned)__builtin_bit_cast(uint16_t, hy) << 16),
                   (unsigned)__builtin_bit_cast(uint16_t, hz));
  }
}

// Adds the per-cell accumulator into the caller's position and density
// gradients (+=) and clears it; cells the adjoint did not touch are skipped.
__global__ void __launch_bounds__(256) k_fold_cell_grads(float4* __restrict__ acc, int n,
                                                         float* __restrict__ g_sites,
                                                         float* __restrict__ g_density) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 v = acc[i];
  if (v.x == 0.0f && v.y == 0.0f && v.z == 0.0f && v.w == 0.0f) return;
  g_sites[3 * i] += v.x;
  g_sites[3 * i + 1] += v.y;
  g_sites[3 * i + 2] += v.z;
  g_density[i] += v.w;
  acc[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

voro_status launch_fold_cell_grads(const voro_scene* scene, void* ws, float* g_sites,
                                   float* g_density, hipStream_t st) {
  const WsLayout L = ws_layout(scene->n_sites, scene->n_edges);
  const int n = scene->n_sites;
  hipLaunchKernelGGL(k_fold_cell_grads, dim3((n + 255) / 256), dim3(256), 0, st,
                     reinterpret_cast<float4*>((char*)ws + L.cellg), n, g_sites, g_density);
  return check_launch("adjoint: fold position and density gradients");
}

float4* cell_grads(const voro_scene* s, void* ws) {
  return reinterpret_cast<float4*>((char*)ws + ws_layout(s->n_sites, s->n_edges).cellg);
}

// ------------------------------------------------------- explicit-ray launch
struct RayArgs {
  DevScene s;
  WalkParams w;
  RayMap map;
  const float* o;
  const float* d;
  const float* tmax;
  const int32_t* start;
  // forward outputs
  float* rgb;
  float* T;
  int32_t* nsteps;
  int32_t* cells_out;
  int max_record;
  float* dist_out;  // [R,3] distortion loss, sum w sbar, sum w (or null)
  // backward inputs / outputs
  const float* rgb_in;
  const float* T_in;
  const float* g_rgb;
  const float* g_T;
  const float* dist_in;  // [R,3] saved by the forward (with g_dist)
  const float* g_dist;   // [R] upstream gradient of the distortion loss (or null)
  Grads g;
  unsigned long long* stats;
  // stored exits, [trace_cap][n_rays] (null: the adjoint searches every step)
  int2* trace;
  int trace_cap;
};

// the stored exits of one ray (none for a lane without a ray)
__device__ __forceinline__ ExitTrace ray_exits(const RayArgs& a, int ray) {
  ExitTrace x;
  x.p = a.trace && ray >= 0 ? a.trace + ray : nullptr;
  x.stride = (unsigned)a.map.n_rays;
  x.cap = a.trace_cap;
  return x;
}

// One lane per ray walks with staged edge rows (dynamic LDS:
// kStageBytesPerWave per wave), also when gathered rows are ranked in half
// precision.  The one-lane-per-ray exact single-map walk is held to five
// waves per SIMD (96 VGPRs), as in the multi-view forward: the stored-exit
// arguments would otherwise take it to 98 and four waves.
template <int LPR, int APP, bool E16>
struct RenderFwdWaves {
  static constexpr int value = (LPR == 1 && APP == 0 && !E16) ? 5 : 1;
};

template <int LPR, int TEX, int APP, bool E16>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(RenderFwdWaves<LPR, APP, E16>::value, 8)))
    k_render_fwd(RayArgs a) {
  extern __shared__ float4 slabs[];
  const int nwaves = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int grp = lane / LPR;
  const int sub = lane % LPR;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int ray = map_ray<LPR>(a.map, lb, wave, nwaves, grp);
  Counters cnt;
  constexpr bool staged = LPR == 1;
  if (ray >= 0 || staged) {
    RayIn r{};
    if (ray >= 0) {
      r.ox = a.o[3 * (size_t)ray];
      r.oy = a.o[3 * (size_t)ray + 1];
      r.oz = a.o[3 * (size_t)ray + 2];
      r.dx = a.d[3 * (size_t)ray];
      r.dy = a.d[3 * (size_t)ray + 1];
      r.dz = a.d[3 * (size_t)ray + 2];
      r.tmax = a.tmax[ray];
      r.start = a.start[ray];
    }
    int32_t* rec = (ray >= 0 && a.cells_out && a.max_record > 0)
                       ? a.cells_out + (size_t)ray * a.max_record
                       : nullptr;
    const RayOut out =
        staged ? walk_forward_staged<TEX, APP, E16>(a.s, a.w, r, ray >= 0, lane,
                                               slabs + wave * (kStageBytesPerWave / 16), rec,
                                               a.max_record, cnt, a.dist_out != nullptr,
                                               ray_exits(a, ray))
               : walk_forward<LPR, TEX, APP, E16>(a.s, a.w, r, sub, rec, a.max_record, cnt,
                                             a.dist_out != nullptr, ray_exits(a, ray));
    if (ray >= 0 && sub == 0) {
      a.rgb[3 * (size_t)ray] = out.r;
      a.rgb[3 * (size_t)ray + 1] = out.g;
      a.rgb[3 * (size_t)ray + 2] = out.b;
      a.T[ray] = out.T;
      if (a.nsteps) a.nsteps[ray] = out.k;
      if (a.dist_out) {
        a.dist_out[3 * (size_t)ray] = out.dist;
        a.dist_out[3 * (size_t)ray + 1] = out.dist_a;
        a.dist_out[3 * (size_t)ray + 2] = out.dist_w;
      }
      if (rec)
        for (int k = out.k; k < a.max_record; ++k) rec[k] = -1;
    }
  }
  if (a.stats) flush_counters(cnt, sub == 0, lane, a.stats);
}

// The one-lane-per-ray single-map form runs at four waves per SIMD with the
// 528-entry table (as the persistent multi-view adjoint); the others keep
// the larger table at three.
template <int LPR, int APP>
struct RenderBwdShape {
  static constexpr bool quad = LPR == 1 && APP == 0;
  static constexpr int waves = quad ? 4 : 1;
  static constexpr int cap = quad ? kTableCapQuad : TableShape<APP>::cap;
};

template <int LPR, int TEX, int APP>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(RenderBwdShape<LPR, APP>::waves, 8)))
    k_render_bwd(RayArgs a) {
  const int nwaves = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int grp = lane / LPR;
  const int sub = lane % LPR;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int ray = map_ray<LPR>(a.map, lb, wave, nwaves, grp);
  Counters cnt;
  RayIn r = {};
  Upstream u = {};
  if (ray >= 0) {
    r.ox = a.o[3 * (size_t)ray];
    r.oy = a.o[3 * (size_t)ray + 1];
    r.oz = a.o[3 * (size_t)ray + 2];
    r.dx = a.d[3 * (size_t)ray];
    r.dy = a.d[3 * (size_t)ray + 1];
    r.dz = a.d[3 * (size_t)ray + 2];
    r.tmax = a.tmax[ray];
    r.start = a.start[ray];
    u.Cr = a.rgb_in[3 * (size_t)ray];
    u.Cg = a.rgb_in[3 * (size_t)ray + 1];
    u.Cb = a.rgb_in[3 * (size_t)ray + 2];
    u.Tf = a.T_in[ray];
    u.gr = a.g_rgb[3 * (size_t)ray];
    u.gg = a.g_rgb[3 * (size_t)ray + 1];
    u.gb = a.g_rgb[3 * (size_t)ray + 2];
    u.gT = a.g_T ? a.g_T[ray] : 0.0f;
    if (a.g_dist) {
      u.D = a.dist_in[3 * (size_t)ray];
      u.DA = a.dist_in[3 * (size_t)ray + 1];
      u.DW = a.dist_in[3 * (size_t)ray + 2];
      u.gD = a.g_dist[ray];
    }
  }
  constexpr int kCap = RenderBwdShape<LPR, APP>::cap;
  constexpr int kOb = TableShape<APP>::outbox;
  __shared__ int s_keys[kCap];
  __shared__ float s_vals[16 * kCap];
  __shared__ int s_okeys[4][kOb];
  __shared__ float s_ovals[4][kStageStride * kOb];
  GradTable<kCap> tab;
  tab.keys = s_keys;
  tab.vals = s_vals;
  const Outbox ob{s_okeys[wave], s_ovals[wave], kOb};
  table_clear(tab);
  __syncthreads();
  // all lanes take part: the gradient records are merged across the wave,
  // then across the workgroup in the LDS table
  walk_backward<LPR, TEX, APP, kCap>(a.s, a.w, r, u, ray >= 0, sub, lane, a.g, &tab, ob, cnt,
                               a.g_dist != nullptr, ray_exits(a, ray));
  __syncthreads();
  table_flush(tab, a.g, a.s.res * a.s.res, a.s.res);
  if (a.stats) flush_counters(cnt, sub == 0, lane, a.stats);
}

template <int LPR, int TEX, int APP>
static void launch_ray_kernel(bool backward, const RayArgs& a, int blocks, int block,
                              hipStream_t st) {
  if (!backward) {
    const size_t lds = LPR == 1 ? (size_t)(block / 64) * kStageBytesPerWave : 0;
    if constexpr (LPR == 1) {
      if (a.w.edge16) {
        hipLaunchKernelGGL((k_render_fwd<1, TEX, APP, true>), dim3(blocks), dim3(block), lds, st,
                           a);
        return;
      }
    }
    hipLaunchKernelGGL((k_render_fwd<LPR, TEX, APP, false>), dim3(blocks), dim3(block), lds, st, a);
    return;
  }
  if constexpr (APP != 2) {
    // (the comparison model of appearance 2 has no adjoint: refused on the host)
    hipLaunchKernelGGL((k_render_bwd<LPR, TEX, APP>), dim3(blocks), dim3(block), 0, st, a);
  }
}

template <int TEX, int APP>
static void dispatch_lpr(int lpr, bool backward, const RayArgs& a, int blocks, int block,
                         hipStream_t st) {
  switch (lpr) {
    case 1: launch_ray_kernel<1, TEX, APP>(backward, a, blocks, block, st); break;
    case 2: launch_ray_kernel<2, TEX, APP>(backward, a, blocks, block, st); break;
    case 4: launch_ray_kernel<4, TEX, APP>(backward, a, blocks, block, st); break;
    case 8: launch_ray_kernel<8, TEX, APP>(backward, a, blocks, block, st); break;
    default: launch_ray_kernel<16, TEX, APP>(backward, a, blocks, block, st); break;
  }
}

template <int APP>
static void dispatch_tex(int tex, int lpr, bool backward, const RayArgs& a, int blocks, int block,
                         hipStream_t st) {
  switch (tex) {
    case VORO_TEX_F32: dispatch_lpr<VORO_TEX_F32, APP>(lpr, backward, a, blocks, block, st); break;
    case VORO_TEX_F16: dispatch_lpr<VORO_TEX_F16, APP>(lpr, backward, a, blocks, block, st); break;
    default: dispatch_lpr<VORO_TEX_BF16, APP>(lpr, backward, a, blocks, block, st); break;
  }
}

static void dispatch_ray_kernel(int app, int tex, int lpr, bool backward, const RayArgs& a,
                                int blocks, int block, hipStream_t st) {
  if (app == 1)
    dispatch_tex<1>(tex, lpr, backward, a, blocks, block, st);
  else if (app == 2)
    dispatch_tex<2>(tex, lpr, backward, a, blocks, block, st);
  else
    dispatch_tex<0>(tex, lpr, backward, a, blocks, block, st);
}

float4* cell_grads(const voro_scene* s, void* ws);

DevScene dev_scene(const voro_scene* s, const void* ws) {
  const WsLayout L = ws_layout(s->n_sites, s->n_edges);
  DevScene d;
  d.cells = reinterpret_cast<const float4*>((const char*)ws + L.cells);
  d.edges = reinterpret_cast<const float4*>((const char*)ws + L.edges);
  d.edges16 = reinterpret_cast<const uint2*>((const char*)ws + L.edges16);
  d.texels = s->texels;
  d.n = s->n_sites;
  d.res = s->tex_res;
  return d;
}

WalkParams walk_params(const voro_params* p) {
  WalkParams w;
  w.t_stop = p->t_stop;
  w.skip_w = p->skip_w;
  w.tie_window = p->tie_window;
  w.max_steps = p->max_steps;
  w.edge16 = p->edge_fp16;
  return w;
}

static voro_status ray_launch(bool backward, const voro_scene* scene, const void* ws,
                              size_t ws_bytes, const float* o, const float* d, const float* tmax,
                              const int32_t* start, int32_t R, const voro_params* params,
                              RayArgs a, void* stream) {
  voro_status st;
  if ((st = check_scene(scene)) != VORO_OK) return st;
  if ((st = check_ws(scene, ws, ws_bytes)) != VORO_OK) return st;
  if ((st = check_params(params, backward)) != VORO_OK) return st;
  if ((st = check_appearance(scene, params)) != VORO_OK) return st;
  if (R < 0) return fail(VORO_EINVAL, "R must be >= 0");
  if (R == 0) return VORO_OK;
  if (!o || !d || !tmax || !start) return fail(VORO_EINVAL, "ray arrays must not be NULL");
  if (params->img_w > 0 && (R % params->img_w) != 0)
    return fail(VORO_EINVAL, "R (%d) must be a multiple of img_w (%d)", R, params->img_w);
  if ((st = check_device()) != VORO_OK) return st;
  const Launch L = resolve_launch(params);
  a.s = dev_scene(scene, ws);
  a.w = walk_params(params);
  a.o = o;
  a.d = d;
  a.tmax = tmax;
  a.start = start;
  a.map.n_rays = R;
  a.map.img_w = params->img_w;
  a.map.img_h = params->img_w > 0 ? R / params->img_w : 1;
  a.map.tile_w = L.tile_w;
  a.map.tile_h = L.tile_h;
  const int nwaves = L.block / 64;
  long blocks;
  if (params->img_w > 0) {
    const int wx = nwaves >= 2 ? 2 : 1;
    const int bw = L.tile_w * wx;
    const int bh = L.tile_h * (nwaves / wx);
    a.map.blocks_x = (params->img_w + bw - 1) / bw;
    blocks = (long)a.map.blocks_x * ((a.map.img_h + bh - 1) / bh);
  } else {
    a.map.blocks_x = 0;
    const long rays_per_block = (long)L.block / L.lpr;
    blocks = (R + rays_per_block - 1) / rays_per_block;
  }
  if (blocks > 0x7fffffff) return fail(VORO_EINVAL, "too many rays");
  dispatch_ray_kernel(params->appearance, scene->tex_dtype, L.lpr, backward, a, (int)blocks, L.block,
                      (hipStream_t)stream);
  return check_launch(backward ? "voro_render_bwd" : "voro_render_fwd");
}

}  // namespace voro

using namespace voro;

extern "C" {

voro_status voro_prepare(const voro_scene* scene, void* ws, size_t ws_bytes, uint64_t* stats,
                         void* stream) {
  voro_status st;
  if ((st = check_scene(scene)) != VORO_OK) return st;
  if ((st = check_ws(scene, ws, ws_bytes)) != VORO_OK) return st;
  if ((st = check_device()) != VORO_OK) return st;
  const WsLayout L = ws_layout(scene->n_sites, scene->n_edges);
  PrepArgs a;
  a.sites = scene->sites;
  a.density = scene->density;
  a.nbr_off = scene->nbr_off;
  a.nbr_idx = scene->nbr_idx;
  a.n = scene->n_sites;
  a.m = (int)scene->n_edges;
  a.cells = reinterpret_cast<float4*>((char*)ws + L.cells);
  a.edges = reinterpret_cast<float4*>((char*)ws + L.edges);
  a.edges16 = reinterpret_cast<uint2*>((char*)ws + L.edges16);
  a.cellg = reinterpret_cast<float4*>((char*)ws + L.cellg);
  a.stats = reinterpret_cast<unsigned long long*>(stats);
  const long threads = (long)scene->n_sites * 16;
  const int blocks = (int)((threads + 255) / 256);
  hipLaunchKernelGGL(k_prepare, dim3(blocks), dim3(256), 0, (hipStream_t)stream, a);
  return check_launch("voro_prepare");
}

voro_status voro_render_fwd(const voro_scene* scene, const void* ws, size_t ws_bytes,
                            const float* o, const float* d, const float* tmax,
                            const int32_t* start_cell, int32_t R, const voro_params* params,
                            float* rgb, float* T, int32_t* nsteps, int32_t* cells, float* dist,
                            int32_t* trace, int32_t trace_cap, uint64_t* stats, void* stream) {
  if (R > 0 && (!rgb || !T)) return fail(VORO_EINVAL, "rgb and T must not be NULL");
  if (params && params->max_record > 0 && !cells)
    return fail(VORO_EINVAL, "cells must not be NULL when max_record > 0");
  voro_status st0 = check_trace(trace, trace_cap);
  if (st0 != VORO_OK) return st0;
  RayArgs a = {};
  a.trace = reinterpret_cast<int2*>(trace);
  a.trace_cap = trace ? trace_cap : 0;
  a.rgb = rgb;
  a.T = T;
  a.nsteps = nsteps;
  a.cells_out = cells;
  a.max_record = params ? params->max_record : 0;
  a.dist_out = dist;
  a.stats = reinterpret_cast<unsigned long long*>(stats);
  return ray_launch(false, scene, ws, ws_bytes, o, d, tmax, start_cell, R, params, a, stream);
}

voro_status voro_render_bwd(const voro_scene* scene, void* ws, size_t ws_bytes,
                            const float* o, const float* d, const float* tmax,
                            const int32_t* start_cell, int32_t R, const voro_params* params,
                            const float* rgb, const float* T, const float* g_rgb,
                            const float* g_T, const float* dist, const float* g_dist,
                            const int32_t* trace, int32_t trace_cap, float* g_sites,
                            float* g_density, float* g_texels, uint64_t* stats, void* stream) {
  if (R > 0 && (!rgb || !T || !g_rgb))
    return fail(VORO_EINVAL, "rgb, T and g_rgb must not be NULL");
  if ((dist == nullptr) != (g_dist == nullptr))
    return fail(VORO_EINVAL, "dist and g_dist must both be given or both be NULL");
  if (R > 0 && (!g_sites || !g_density || !g_texels))
    return fail(VORO_EINVAL, "gradient outputs must not be NULL");
  if (g_texels && !aligned(g_texels, 16)) return fail(VORO_EINVAL, "g_texels must be 16-byte aligned");
  voro_status st0 = check_trace(trace, trace_cap);
  if (st0 != VORO_OK) return st0;
  RayArgs a = {};
  a.trace = reinterpret_cast<int2*>(const_cast<int32_t*>(trace));
  a.trace_cap = trace ? trace_cap : 0;
  a.rgb_in = rgb;
  a.T_in = T;
  a.g_rgb = g_rgb;
  a.g_T = g_T;
  a.dist_in = dist;
  a.g_dist = g_dist;
  a.g.texels = g_texels;
  a.g.maps = scene && scene->tex_maps == 2 ? 2 : 1;
  a.stats = reinterpret_cast<unsigned long long*>(stats);
  if (scene && ws) a.g.cell = cell_grads(scene, ws);
  voro_status st =
      ray_launch(true, scene, ws, ws_bytes, o, d, tmax, start_cell, R, params, a, stream);
  if (st != VORO_OK || R == 0) return st;
  return launch_fold_cell_grads(scene, ws, g_sites, g_density, (hipStream_t)stream);
}

}  // extern "C"
