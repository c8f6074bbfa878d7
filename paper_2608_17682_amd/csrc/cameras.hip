// Ray generation and the persistent multi-view launch (Sec. 6.5, App. D:
// several camera models rendered by the same walk; Sec. 5.6: waves take
// compact screen tiles so neighbouring lanes walk similar cells).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "camera_impl.hpp"
#include "host_common.hpp"
#include "locate_impl.hpp"
#include "voro_device.hpp"
#include "walk_impl.hpp"

namespace voro {

voro_status launch_locate_brute(const voro_scene* scene, void* partials, const float* origins,
                                int U, int32_t* out, hipStream_t st);
float4* cell_grads(const voro_scene* s, void* ws);

// ------------------------------------------------------------- gen_rays
__global__ void __launch_bounds__(256) k_gen_rays(CamTable ct, float* __restrict__ o,
                                                  float* __restrict__ d, float* __restrict__ tmax,
                                                  int n_rays) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rays) return;
  const int v = find_view(ct.ray_off, ct.V, i);
  const voro_camera& c = ct.cam[v];
  const int spp = c.spp;
  const int local = i - ct.ray_off[v];
  const int pix = local / spp;
  const int s = local - pix * spp;
  const int px = pix % c.width;
  const int py = pix / c.width;
  float ox, oy, oz, dx, dy, dz, tm;
  gen_ray(c, ct.g[v], ct.focal[v], px, py, s, ox, oy, oz, dx, dy, dz, tm);
  o[3 * (size_t)i] = ox;
  o[3 * (size_t)i + 1] = oy;
  o[3 * (size_t)i + 2] = oz;
  d[3 * (size_t)i] = dx;
  d[3 * (size_t)i + 1] = dy;
  d[3 * (size_t)i + 2] = dz;
  tmax[i] = tm;
}

// ------------------------------------------------------ multi-view launch
//
// Work unit: one wave-sized screen tile (tile_w x tile_h rays) of one view.
// A thin-lens view's samples form a (W g) x (H g) ray grid so a tile holds
// neighbouring samples.  Workgroup b runs on XCD b % 8; each XCD first
// drains its own contiguous eighth of the tile sequence (its L2 sees one
// image region), then helps the other XCDs.  Counters live in the workspace
// and are zeroed by k_views_setup before every launch.
constexpr int kXcd = 8;

struct ViewsArgs {
  DevScene s;
  WalkParams w;
  CamTable ct;
  const int32_t* center_cell;  // [V] cell of each camera centre
  unsigned int* counters;      // [kXcd]
  int total_tiles;
  int tile_w, tile_h;
  // refill schedule: strips of strip_tiles tiles inside one view
  int strip_off[VORO_MAX_VIEWS + 1];
  int strip_tiles;
  // forward
  float* rgb;
  float* T;
  float* ray_rgbT;
  int32_t* nsteps;
  // backward
  const float* rgb_in;
  const float* T_in;
  const float* ray_rgbT_in;
  const float* g_rgb;
  const float* g_T;
  Grads g;
  unsigned long long* stats;
  // stored exits, [trace_cap][n_rays] (null: the adjoint searches every step)
  int2* trace;
  int trace_cap;
  unsigned n_rays;
};

// the stored exits of one ray (none for a lane without a ray)
__device__ __forceinline__ ExitTrace ray_trace(const ViewsArgs& a, bool has, int ray) {
  ExitTrace x;
  x.p = a.trace && has ? a.trace + ray : nullptr;
  x.stride = a.n_rays;
  x.cap = a.trace_cap;
  return x;
}

struct Centers {
  float c[3 * VORO_MAX_VIEWS];
};

// camera centres into the workspace (they travel as kernel arguments, so no
// host-to-device copy is needed) and the tile counters zeroed
__global__ void k_views_setup(Centers c, float* dst, int n, unsigned int* ctr) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = c.c[i];
  if (i < kXcd) ctr[i] = 0u;
}

// Next work unit from the XCD-partitioned queue (one thread asks), or -1
// when every XCD's range is drained.  probe: how many ranges this caller has
// found empty so far.
__device__ __forceinline__ int next_unit(unsigned int* counters, int total, int xcd, int& probe) {
  while (probe < kXcd) {
    const int x = (xcd + probe) % kXcd;
    const int lo = (int)(((long)total * x) / kXcd);
    const int hi = (int)(((long)total * (x + 1)) / kXcd);
    const int t = (int)atomicAdd(&counters[x], 1u);
    if (lo + t < hi) return lo + t;
    ++probe;
  }
  return -1;
}

// per-wave claim: lane 0 asks, the wave shares the answer
__device__ __forceinline__ int next_tile(unsigned int* counters, int total, int xcd, int lane,
                                         int& probe) {
  int t = 0;
  if (lane == 0) t = next_unit(counters, total, xcd, probe);
  return __shfl(t, 0);
}

struct TileRay {
  int view, px, py, s, ray, pixel;
};

// Decode (work unit, wave's sub-tile, lane group) into a ray; false outside
// the view.  A unit is unit_w x unit_h rays; the wave covers the tile_w x
// tile_h sub-tile at (sx, sy) tiles inside it.
__device__ __forceinline__ bool tile_ray(const CamTable& ct, int unit, int sx, int sy, int grp,
                                         int tile_w, int tile_h, int unit_w, int unit_h,
                                         TileRay& tr) {
  // the unit is wave-uniform: keep the camera in scalar registers
  const int v = __builtin_amdgcn_readfirstlane(find_view(ct.tile_off, ct.V, unit));
  const voro_camera& c = ct.cam[v];
  const int gx = ct.gx[v];
  const int gy = ct.gy[v];
  const int gw = c.width * gx;
  const int gh = c.height * gy;
  const int units_x = (gw + unit_w - 1) / unit_w;
  const int local = unit - ct.tile_off[v];
  const int X = (local % units_x) * unit_w + sx * tile_w + grp % tile_w;
  const int Y = (local / units_x) * unit_h + sy * tile_h + grp / tile_w;
  if (X >= gw || Y >= gh) return false;
  tr.view = v;
  tr.px = X / gx;
  tr.py = Y / gy;
  tr.s = (X % gx) + gx * (Y % gy);
  tr.pixel = tr.py * c.width + tr.px;
  tr.ray = ct.ray_off[v] + tr.pixel * c.spp + tr.s;
  return true;
}

__device__ __forceinline__ RayIn views_ray(const ViewsArgs& a, const TileRay& tr, bool* capped) {
  const voro_camera& c = a.ct.cam[tr.view];
  RayIn r;
  gen_ray(c, a.ct.g[tr.view], a.ct.focal[tr.view], tr.px, tr.py, tr.s, r.ox, r.oy, r.oz, r.dx,
          r.dy, r.dz, r.tmax);
  r.start = a.center_cell[tr.view];
  const bool moved = c.model == VORO_CAM_ROLLING_SHUTTER || c.model == VORO_CAM_MOTION_BLUR ||
                     (c.model == VORO_CAM_THIN_LENS && c.lens_radius > 0.0f);
  if (moved && r.tmax > 0.0f && r.start >= 0 && r.start < a.s.n)
    r.start = nearest_walk(a.s, r.ox, r.oy, r.oz, r.start, capped);
  return r;
}

// one ray's forward outputs
template <int LPR>
__device__ __forceinline__ void write_ray_out(const ViewsArgs& a, const TileRay& tr,
                                              const RayOut& out) {
  const voro_camera& c = a.ct.cam[tr.view];
  if (c.spp == 1) {
    const size_t p = (size_t)a.ct.pix_off[tr.view] + tr.pixel;
    a.rgb[3 * p] = out.r;
    a.rgb[3 * p + 1] = out.g;
    a.rgb[3 * p + 2] = out.b;
    a.T[p] = out.T;
  }
  if (a.ray_rgbT) {
    reinterpret_cast<float4*>(a.ray_rgbT)[tr.ray] = make_float4(out.r, out.g, out.b, out.T);
  }
  if (a.nsteps) a.nsteps[tr.ray] = out.k;
}

// PERSIST: waves loop over the XCD-partitioned tile queue; otherwise each
// wave of the grid takes one tile (workgroups renumbered per XCD) and the
// hardware dispatcher balances the load.  One lane per ray walks with staged
// edge rows (dynamic LDS: kStageBytesPerWave per wave), also when gathered
// rows are ranked in half precision.  The persistent one-lane-per-ray exact walk is
// held to 96 VGPRs, five waves per SIMD instead of four (the registers come
// from the FP64 branch, the per-view focal length and the per-tile counters;
// its few spills, 48 bytes per lane, sit outside the walk loop); the extra
// wave hides more of the gathers' latency.
template <int LPR, int APP, bool PERSIST, bool E16>
struct FwdWaves {
  static constexpr int value = (LPR == 1 && APP == 0 && (PERSIST ? !E16 : E16)) ? 5 : 1;
};

template <int LPR, int TEX, int APP, bool PERSIST, bool E16>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(FwdWaves<LPR, APP, PERSIST, E16>::value, 8)))
    k_views_fwd(ViewsArgs a) {
  extern __shared__ float4 slabs[];
  __shared__ unsigned long long s_stats[kWgStats];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int grp = lane / LPR;
  const int sub = lane % LPR;
  const int xcd = blockIdx.x % kXcd;
  if constexpr (PERSIST) {
    wg_stats_clear(s_stats);
    __syncthreads();
  }
  int probe = 0;
  int tile = PERSIST ? -1 : xcd_block(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave;
  for (;;) {
    if constexpr (PERSIST) {
      tile = next_tile(a.counters, a.total_tiles, xcd, lane, probe);
      if (tile < 0) break;
    } else if (tile >= a.total_tiles) {
      break;
    }
    Counters cnt;
    bool capped = false;
    TileRay tr;
    const bool has = tile_ray(a.ct, tile, 0, 0, grp, a.tile_w, a.tile_h, a.tile_w, a.tile_h, tr);
    if constexpr (LPR == 1) {
      RayIn r{};
      if (has) r = views_ray(a, tr, &capped);
      const RayOut out = walk_forward_staged<TEX, APP, E16>(
          a.s, a.w, r, has, lane, slabs + wave * (kStageBytesPerWave / 16), nullptr, 0, cnt,
          false, ray_trace(a, has, tr.ray));
      if (has) write_ray_out<LPR>(a, tr, out);
    } else if (has) {
      const RayIn r = views_ray(a, tr, &capped);
      const RayOut out = walk_forward<LPR, TEX, APP, E16>(a.s, a.w, r, sub, nullptr, 0, cnt,
                                                          false, ray_trace(a, true, tr.ray));
      if (sub == 0) write_ray_out<LPR>(a, tr, out);
    }
    if (a.stats) {
      const bool mine = has && sub == 0;
      if constexpr (PERSIST) {
        tile_counters_to_lds(cnt, mine, capped, lane, s_stats);
      } else {
        flush_counters(cnt, mine, lane, a.stats);
        const uint32_t cp = wave_sum_u32(mine && capped ? 1u : 0u);
        if (lane == 0 && cp) atomicAdd(&a.stats[VORO_STAT_LOCATE_CAP], (unsigned long long)cp);
      }
    }
    if constexpr (!PERSIST) break;
  }
  if constexpr (PERSIST) {
    __syncthreads();
    if (a.stats) wg_stats_flush(s_stats, a.stats);
  }
}

// Refill schedule (one lane per ray): each wave owns a strip of tiles in one
// view and keeps its lanes busy across the strip: whenever at least
// kRefillMin lanes (or all of them) have finished their rays, the idle lanes
// take the strip's next rays in lane order (ballot + rank) and the walk goes
// on.  Every refill advances the strip cursor by the idle count and every
// ray ends within max_steps, so the loop ends.
constexpr int kRefillMin = 16;
constexpr int kStripTiles = 4;  // 256 rays per wave

template <int TEX, int APP, bool E16>
__global__ void __launch_bounds__(256) k_views_fwd_refill(ViewsArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  Counters cnt;
  uint32_t capped_n = 0;
  const int strip = xcd_block(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave;
  if (strip < a.strip_off[a.ct.V]) {
    const int v = find_view(a.strip_off, a.ct.V, strip);
    const int t0 = a.ct.tile_off[v] + (strip - a.strip_off[v]) * a.strip_tiles;
    const int nt = min(a.strip_tiles, a.ct.tile_off[v + 1] - t0);
    const int pool = nt * 64;
    int q = 0;  // next ray of the strip (wave-uniform)
    bool active = false;
    FwdState<APP> st;
    RayIn r = {};
    TileRay tr = {};
    for (;;) {
      const unsigned long long idle = __ballot(!active);
      const int n_idle = __popcll(idle);
      if (q < pool && (n_idle >= kRefillMin || n_idle == 64)) {
        const int idx = q + __popcll(idle & ((1ull << lane) - 1ull));
        if (!active && idx < pool &&
            tile_ray(a.ct, t0 + (idx >> 6), 0, 0, idx & 63, a.tile_w, a.tile_h, a.tile_w,
                     a.tile_h, tr)) {
          bool capped = false;
          r = views_ray(a, tr, &capped);
          capped_n += capped ? 1u : 0u;
          active = fwd_begin<APP>(st, a.s, r, cnt);
          if (!active) write_ray_out<1>(a, tr, fwd_end<APP>(st, false, cnt));
        }
        q += n_idle;
      }
      if (!__any(active)) {
        if (q >= pool) break;
        continue;
      }
      if (active && fwd_step<1, TEX, APP, E16>(st, a.s, a.w, r, 0, nullptr, 0, cnt, false, nullptr,
                                               ray_trace(a, true, tr.ray))) {
        write_ray_out<1>(a, tr, fwd_end<APP>(st, true, cnt));
        active = false;
      }
    }
  }
  if (a.stats) {
    flush_counters(cnt, true, lane, a.stats);
    const uint32_t cp = wave_sum_u32(capped_n);
    if (lane == 0 && cp) atomicAdd(&a.stats[VORO_STAT_LOCATE_CAP], (unsigned long long)cp);
  }
}

// Backward work unit: a workgroup tile (the waves' tiles side by side, 2
// wide), walked by the whole workgroup into one LDS gradient table that is
// flushed to global memory before the next unit.  The persistent
// one-lane-per-ray single-map adjoint is held to 128 VGPRs and a 528-entry
// table, four workgroups of four waves per CU instead of three (it spills
// 84 bytes per lane, a few of whose reloads fall inside the walk loop; the
// extra wave still wins); the other forms keep the larger table.
template <int LPR, int APP, bool PERSIST>
struct BwdShape {
  static constexpr bool quad = PERSIST && LPR == 1 && APP == 0;
  static constexpr int waves = quad ? 4 : 1;
  static constexpr int cap = quad ? kTableCapQuad : TableShape<APP>::cap;
};

template <int LPR, int TEX, int APP, bool PERSIST>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(BwdShape<LPR, APP, PERSIST>::waves, 8)))
    k_views_bwd(ViewsArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const int wx = nwaves >= 2 ? 2 : 1;
  const int grp = lane / LPR;
  const int sub = lane % LPR;
  const int xcd = blockIdx.x % kXcd;
  const int unit_w = a.tile_w * wx;
  const int unit_h = a.tile_h * (nwaves / wx);
  const int RR = a.s.res * a.s.res;
  constexpr int kCap = BwdShape<LPR, APP, PERSIST>::cap;
  constexpr int kOb = TableShape<APP>::outbox;
  __shared__ int s_keys[kCap];
  __shared__ float s_vals[16 * kCap];
  __shared__ int s_unit;
  __shared__ int s_okeys[4][kOb];
  __shared__ float s_ovals[4][kStageStride * kOb];
  GradTable<kCap> tab;
  tab.keys = s_keys;
  tab.vals = s_vals;
  const Outbox ob{s_okeys[wave], s_ovals[wave], kOb};
  __shared__ unsigned long long s_stats[kWgStats];
  table_clear(tab);
  if constexpr (PERSIST) wg_stats_clear(s_stats);
  int probe = 0;
  int unit = PERSIST ? -1 : xcd_block(blockIdx.x, gridDim.x);
  for (;;) {
    if constexpr (PERSIST) {
      if (threadIdx.x == 0) s_unit = next_unit(a.counters, a.total_tiles, xcd, probe);
      __syncthreads();
      unit = s_unit;
      if (unit < 0) break;
    } else {
      __syncthreads();
      if (unit >= a.total_tiles) break;
    }
    TileRay tr;
    const bool has = tile_ray(a.ct, unit, wave % wx, wave / wx, grp, a.tile_w, a.tile_h, unit_w,
                              unit_h, tr);
    RayIn r = {};
    Upstream u = {};
    if (has) {
      bool capped = false;
      r = views_ray(a, tr, &capped);
      const voro_camera& c = a.ct.cam[tr.view];
      const size_t p = (size_t)a.ct.pix_off[tr.view] + tr.pixel;
      const float share = 1.0f / (float)c.spp;
      if (c.spp == 1) {
        u.Cr = a.rgb_in[3 * p];
        u.Cg = a.rgb_in[3 * p + 1];
        u.Cb = a.rgb_in[3 * p + 2];
        u.Tf = a.T_in[p];
      } else {
        const float4 q = reinterpret_cast<const float4*>(a.ray_rgbT_in)[tr.ray];
        u.Cr = q.x;
        u.Cg = q.y;
        u.Cb = q.z;
        u.Tf = q.w;
      }
      u.gr = a.g_rgb[3 * p] * share;
      u.gg = a.g_rgb[3 * p + 1] * share;
      u.gb = a.g_rgb[3 * p + 2] * share;
      u.gT = a.g_T ? a.g_T[p] * share : 0.0f;
    }
    // the whole wave walks its tile together (gradient records merge across
    // lanes); its counters go to the workgroup's LDS stats after each unit
    Counters cnt;
    walk_backward<LPR, TEX, APP, kCap>(a.s, a.w, r, u, has, sub, lane, a.g, &tab, ob, cnt, false,
                                       ray_trace(a, has, tr.ray));
    if (a.stats) {
      if constexpr (PERSIST) {
        tile_counters_to_lds(cnt, has && sub == 0, false, lane, s_stats);
      } else {
        flush_counters(cnt, has && sub == 0, lane, a.stats);
      }
    }
    __syncthreads();
    table_flush(tab, a.g, RR, a.s.res);
    __syncthreads();
    if constexpr (!PERSIST) break;
  }
  if constexpr (PERSIST) {
    __syncthreads();
    if (a.stats) wg_stats_flush(s_stats, a.stats);
  }
}

// pixel = mean of its samples, in sample order
__global__ void __launch_bounds__(256) k_views_resolve(CamTable ct, const float4* __restrict__ ray_rgbT,
                                                       float* __restrict__ rgb, float* __restrict__ T,
                                                       int n_pixels) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pixels) return;
  const int v = find_view(ct.pix_off, ct.V, p);
  const int spp = ct.cam[v].spp;
  if (spp == 1) return;
  const int base = ct.ray_off[v] + (p - ct.pix_off[v]) * spp;
  float r = 0.0f, g = 0.0f, b = 0.0f, t = 0.0f;
  for (int s = 0; s < spp; ++s) {
    const float4 q = ray_rgbT[base + s];
    r += q.x;
    g += q.y;
    b += q.z;
    t += q.w;
  }
  const float inv = 1.0f / (float)spp;
  rgb[3 * (size_t)p] = r * inv;
  rgb[3 * (size_t)p + 1] = g * inv;
  rgb[3 * (size_t)p + 2] = b * inv;
  T[p] = t * inv;
}

static CamTable make_table(const voro_camera* cams, int V, int tile_w, int tile_h) {
  CamTable ct;
  std::memset(&ct, 0, sizeof(ct));
  ct.V = V;
  int ro = 0, po = 0, to = 0;
  for (int v = 0; v < V; ++v) {
    ct.cam[v] = cams[v];
    const int g = (int)std::lround(std::sqrt((double)cams[v].spp));
    ct.g[v] = g;
    // thin-lens samples tile the pixel as g x g; time samples as a row
    ct.gx[v] = cams[v].model == VORO_CAM_THIN_LENS ? g : cams[v].spp;
    ct.gy[v] = cams[v].model == VORO_CAM_THIN_LENS ? g : 1;
    ct.focal[v] = camera_focal(cams[v]);
    ct.ray_off[v] = ro;
    ct.pix_off[v] = po;
    ct.tile_off[v] = to;
    ro += cams[v].width * cams[v].height * cams[v].spp;
    po += cams[v].width * cams[v].height;
    if (tile_w > 0) {
      const int gw = cams[v].width * ct.gx[v], gh = cams[v].height * ct.gy[v];
      to += ((gw + tile_w - 1) / tile_w) * ((gh + tile_h - 1) / tile_h);
    }
  }
  for (int v = V; v <= VORO_MAX_VIEWS; ++v) {
    ct.ray_off[v] = ro;
    ct.pix_off[v] = po;
    ct.tile_off[v] = to;
  }
  return ct;
}

// dynamic LDS of a forward launch: the staged edge rows of each wave
template <int LPR>
static size_t fwd_lds(int block) {
  return LPR == 1 ? (size_t)(block / 64) * kStageBytesPerWave : 0;
}

template <int LPR, int TEX, int APP, bool E16 = false>
static int persistent_blocks(bool backward, int block) {
  static int cached[2][3] = {};
  int& c = cached[backward ? 1 : 0][block == 64 ? 0 : (block == 128 ? 1 : 2)];
  if (c) return c;
  int dev = 0, cus = 0, occ = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if constexpr (APP == 2) {
    (void)backward;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_views_fwd<LPR, TEX, APP, true, E16>,
                                                       block, fwd_lds<LPR>(block));
  } else if (backward) {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_views_bwd<LPR, TEX, APP, true>, block, 0);
  } else {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_views_fwd<LPR, TEX, APP, true, E16>,
                                                       block, fwd_lds<LPR>(block));
  }
  (void)hipGetLastError();
  c = max(kXcd, max(1, cus) * max(1, occ));
  c = (c / kXcd) * kXcd;
  return c;
}

// forward launches: lane refill, persistent queue or grid
template <int LPR, int TEX, int APP, bool E16>
static void launch_views_fwd_t(bool persist, const ViewsArgs& a, int block, hipStream_t st) {
  const int nwaves = block / 64;
  if constexpr (LPR == 1) {
    if (a.strip_tiles > 0) {
      const int strips = a.strip_off[a.ct.V];
      hipLaunchKernelGGL((k_views_fwd_refill<TEX, APP, E16>),
                         dim3(max(1, (strips + nwaves - 1) / nwaves)), dim3(block), 0, st, a);
      return;
    }
  }
  if (persist) {
    const int blocks = persistent_blocks<LPR, TEX, APP, E16>(false, block);
    hipLaunchKernelGGL((k_views_fwd<LPR, TEX, APP, true, E16>), dim3(blocks), dim3(block),
                       fwd_lds<LPR>(block), st, a);
  } else {
    const int blocks = max(1, (a.total_tiles + nwaves - 1) / nwaves);
    hipLaunchKernelGGL((k_views_fwd<LPR, TEX, APP, false, E16>), dim3(blocks), dim3(block),
                       fwd_lds<LPR>(block), st, a);
  }
}

template <int LPR, int TEX, int APP>
static void launch_views_t(bool backward, bool persist, const ViewsArgs& a, int block,
                           hipStream_t st) {
  if (!backward) {
    if constexpr (LPR == 1) {
      if (a.w.edge16) {
        launch_views_fwd_t<1, TEX, APP, true>(persist, a, block, st);
        return;
      }
    }
    launch_views_fwd_t<LPR, TEX, APP, false>(persist, a, block, st);
    return;
  }
  if constexpr (APP != 2) {
    // (the comparison model of appearance 2 has no adjoint: refused on the host)
    if (persist) {
      const int blocks = persistent_blocks<LPR, TEX, APP>(true, block);
      hipLaunchKernelGGL((k_views_bwd<LPR, TEX, APP, true>), dim3(blocks), dim3(block), 0, st, a);
    } else {
      hipLaunchKernelGGL((k_views_bwd<LPR, TEX, APP, false>), dim3(max(1, a.total_tiles)),
                         dim3(block), 0, st, a);
    }
  }
}

template <int TEX, int APP>
static void launch_views_lpr(int lpr, bool backward, bool persist, const ViewsArgs& a, int block,
                             hipStream_t st) {
  switch (lpr) {
    case 1: launch_views_t<1, TEX, APP>(backward, persist, a, block, st); break;
    case 2: launch_views_t<2, TEX, APP>(backward, persist, a, block, st); break;
    case 4: launch_views_t<4, TEX, APP>(backward, persist, a, block, st); break;
    case 8: launch_views_t<8, TEX, APP>(backward, persist, a, block, st); break;
    default: launch_views_t<16, TEX, APP>(backward, persist, a, block, st); break;
  }
}

template <int APP>
static void launch_views_tex(int tex, int lpr, bool backward, bool persist, const ViewsArgs& a,
                             int block, hipStream_t st) {
  switch (tex) {
    case VORO_TEX_F32: launch_views_lpr<VORO_TEX_F32, APP>(lpr, backward, persist, a, block, st); break;
    case VORO_TEX_F16: launch_views_lpr<VORO_TEX_F16, APP>(lpr, backward, persist, a, block, st); break;
    default: launch_views_lpr<VORO_TEX_BF16, APP>(lpr, backward, persist, a, block, st); break;
  }
}

// Scratch of a multi-view launch: the tile-queue counters, the camera
// centres and their cells, and the brute-force search's partial results.
constexpr size_t kViewsScratchCounters = 0;
constexpr size_t kViewsScratchCenters = 256;
constexpr size_t kViewsScratchOrigins = 512;
constexpr size_t kViewsScratchPartials = 768;
constexpr size_t kViewsScratchBytes =
    kViewsScratchPartials + (size_t)VORO_MAX_VIEWS * kLocateChunks * 16;
static_assert(kViewsScratchCenters >= kXcd * 4 && kViewsScratchOrigins - kViewsScratchCenters >=
              VORO_MAX_VIEWS * 4 && kViewsScratchPartials - kViewsScratchOrigins >=
              3 * VORO_MAX_VIEWS * 4, "views scratch layout");

// Where a launch keeps its scratch: counters, centres and their cells at
// `base` (kViewsScratchPartials bytes), the partial results at `partials`.
struct ViewsScratch {
  char* base;
  void* partials;
};

// static_scratch null: the scratch lives in the workspace (counter region and
// the nearest-site search's region), which must then hold voro_workspace_size
// bytes; otherwise the workspace is only read and must hold the prepared
// records.
static voro_status views_common(bool backward, const voro_scene* scene, const void* ws,
                                size_t ws_bytes, const ViewsScratch* static_scratch,
                                const voro_camera* cams, int32_t V, const voro_params* params,
                                ViewsArgs& a, int64_t* n_rays, int64_t* n_pixels, bool* any_spp,
                                int32_t* trace, int32_t trace_cap, void* stream) {
  voro_status st;
  if ((st = check_scene(scene)) != VORO_OK) return st;
  static_assert(kViewsScratchPartials <= 4096, "counter region");
  const WsLayout W = ws_layout(scene->n_sites, scene->n_edges);
  const size_t ws_needed = static_scratch ? W.locate : W.total;
  if (!ws) return fail(VORO_EWORKSPACE, "workspace is NULL");
  if (!aligned(ws, 256)) return fail(VORO_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < ws_needed)
    return fail(VORO_EWORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, ws_needed);
  const ViewsScratch sc = static_scratch
      ? *static_scratch
      : ViewsScratch{(char*)const_cast<void*>(ws) + W.counters,
                     (char*)const_cast<void*>(ws) + W.locate};
  if ((st = check_params(params, backward)) != VORO_OK) return st;
  if ((st = check_appearance(scene, params)) != VORO_OK) return st;
  if ((st = check_cameras(cams, V, n_rays, n_pixels)) != VORO_OK) return st;
  bool spp = false;
  for (int v = 0; v < V; ++v) spp = spp || cams[v].spp > 1;
  *any_spp = spp;
  if ((st = check_device()) != VORO_OK) return st;
  const Launch L = resolve_launch(params);
  a.trace = reinterpret_cast<int2*>(trace);
  a.trace_cap = trace ? trace_cap : 0;
  a.n_rays = (unsigned)*n_rays;
  a.counters = reinterpret_cast<unsigned int*>(sc.base + kViewsScratchCounters);
  int32_t* centers = reinterpret_cast<int32_t*>(sc.base + kViewsScratchCenters);
  float* origins = reinterpret_cast<float*>(sc.base + kViewsScratchOrigins);
  a.center_cell = centers;
  a.s = dev_scene(scene, ws);
  a.w = walk_params(params);
  // forward work units are wave tiles, backward units workgroup tiles
  const int nw = L.block / 64;
  const int wxu = nw >= 2 ? 2 : 1;
  a.ct = backward ? make_table(cams, V, L.tile_w * wxu, L.tile_h * (nw / wxu))
                  : make_table(cams, V, L.tile_w, L.tile_h);
  a.total_tiles = a.ct.tile_off[V];
  a.tile_w = L.tile_w;
  a.tile_h = L.tile_h;
  const hipStream_t s = (hipStream_t)stream;
  // camera centres -> device (through kernel arguments), then their cells
  Centers cc;
  for (int v = 0; v < V; ++v) {
    cc.c[3 * v] = cams[v].c2w[3];
    cc.c[3 * v + 1] = cams[v].c2w[7];
    cc.c[3 * v + 2] = cams[v].c2w[11];
  }
  hipLaunchKernelGGL(k_views_setup, dim3(1), dim3(64), 0, s, cc, origins, 3 * V, a.counters);
  if ((st = check_launch("views: setup")) != VORO_OK) return st;
  if ((st = launch_locate_brute(scene, sc.partials, origins, V, centers, s)) != VORO_OK) return st;
  const int block = L.block;
  // the refill schedule drives the one-lane-per-ray forward; the adjoint
  // (whose work unit is a workgroup tile) takes the persistent queue then
  const bool refill = params->schedule == VORO_SCHEDULE_REFILL;
  const bool persist = params->schedule == VORO_SCHEDULE_PERSISTENT || (refill && backward);
  a.strip_tiles = 0;
  if (refill && !backward && L.lpr == 1) {
    a.strip_tiles = kStripTiles;
    int so = 0;
    for (int v = 0; v < V; ++v) {
      a.strip_off[v] = so;
      const int tiles = a.ct.tile_off[v + 1] - a.ct.tile_off[v];
      so += (tiles + kStripTiles - 1) / kStripTiles;
    }
    for (int v = V; v <= VORO_MAX_VIEWS; ++v) a.strip_off[v] = so;
  }
  if (params->appearance == 1)
    launch_views_tex<1>(scene->tex_dtype, L.lpr, backward, persist, a, block, s);
  else if (params->appearance == 2)
    launch_views_tex<2>(scene->tex_dtype, L.lpr, backward, persist, a, block, s);
  else
    launch_views_tex<0>(scene->tex_dtype, L.lpr, backward, persist, a, block, s);
  return check_launch(backward ? "voro_render_views_bwd" : "voro_render_views_fwd");
}

// ------------------------------------------------- allocation-free launch
//
// voro_render_views_fwd_noalloc keeps the launch's scratch in a file-scope
// device array instead of the caller's workspace.  Each GPU holds its own
// copy until the process ends; host code never passes the array's name to a
// kernel (on the host it only stands in for the symbol) but the device
// address that hipGetSymbolAddress returns for the current device.
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kViewsScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxScratchDevices] = {};

// The current device's scratch address (looked up once per device).
static voro_status static_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(VORO_ENODEV, "no current HIP device");
  }
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(VORO_EUNSUPPORTED, "device %d: the static scratch covers devices 0..%d", dev,
                kMaxScratchDevices - 1);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(VORO_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return VORO_OK;
}

}  // namespace voro

using namespace voro;

extern "C" {

voro_status voro_render_views_fwd_noalloc(const voro_scene* scene, const void* ws,
                                          size_t ws_bytes, const voro_camera* cams, int32_t V,
                                          const voro_params* params, float* rgb, float* T,
                                          float* ray_rgbT, int32_t* nsteps, uint64_t* stats,
                                          void* stream) {
  if (!rgb || !T) return fail(VORO_EINVAL, "rgb and T must not be NULL");
  if (ray_rgbT && !aligned(ray_rgbT, 16)) return fail(VORO_EINVAL, "ray_rgbT must be 16-byte aligned");
  if (V > VORO_MAX_VIEWS)
    return fail(VORO_EINVAL, "V = %d views exceeds the static scratch's maximum of %d", V,
                VORO_MAX_VIEWS);
  int64_t nr = 0, np = 0;
  voro_status st = check_cameras(cams, V, &nr, &np);
  if (st != VORO_OK) return st;
  for (int v = 0; v < V; ++v)
    if (cams[v].spp > 1 && !ray_rgbT)
      return fail(VORO_EINVAL, "ray_rgbT is required when a view has spp > 1");
  if ((st = check_device()) != VORO_OK) return st;
  void* base = nullptr;
  if ((st = static_scratch(&base)) != VORO_OK) return st;
  const ViewsScratch sc{(char*)base, (char*)base + kViewsScratchPartials};
  ViewsArgs a = {};
  a.rgb = rgb;
  a.T = T;
  a.ray_rgbT = ray_rgbT;
  a.nsteps = nsteps;
  a.stats = reinterpret_cast<unsigned long long*>(stats);
  bool any_spp = false;
  st = views_common(false, scene, ws, ws_bytes, &sc, cams, V, params, a, &nr, &np, &any_spp,
                    nullptr, 0, stream);
  if (st != VORO_OK) return st;
  if (any_spp) {
    const int n = (int)np;
    hipLaunchKernelGGL(k_views_resolve, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       a.ct, reinterpret_cast<const float4*>(ray_rgbT), rgb, T, n);
    st = check_launch("voro_render_views_fwd_noalloc: resolve");
  }
  return st;
}

voro_status voro_gen_rays(const voro_camera* cams, int32_t V, float* o, float* d, float* tmax,
                          void* stream) {
  int64_t nr = 0, np = 0;
  voro_status st = check_cameras(cams, V, &nr, &np);
  if (st != VORO_OK) return st;
  if (!o || !d || !tmax) return fail(VORO_EINVAL, "ray outputs must not be NULL");
  if ((st = check_device()) != VORO_OK) return st;
  const CamTable ct = make_table(cams, V, 0, 0);
  const int n = (int)nr;
  hipLaunchKernelGGL(k_gen_rays, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, ct, o,
                     d, tmax, n);
  return check_launch("voro_gen_rays");
}

voro_status voro_render_views_fwd(const voro_scene* scene, void* ws, size_t ws_bytes,
                                  const voro_camera* cams, int32_t V, const voro_params* params,
                                  float* rgb, float* T, float* ray_rgbT, int32_t* nsteps,
                                  int32_t* trace, int32_t trace_cap, uint64_t* stats,
                                  void* stream) {
  if (!rgb || !T) return fail(VORO_EINVAL, "rgb and T must not be NULL");
  if (ray_rgbT && !aligned(ray_rgbT, 16)) return fail(VORO_EINVAL, "ray_rgbT must be 16-byte aligned");
  voro_status st0 = check_trace(trace, trace_cap);
  if (st0 != VORO_OK) return st0;
  ViewsArgs a = {};
  a.rgb = rgb;
  a.T = T;
  a.ray_rgbT = ray_rgbT;
  a.nsteps = nsteps;
  a.stats = reinterpret_cast<unsigned long long*>(stats);
  int64_t nr = 0, np = 0;
  bool any_spp = false;
  // validate everything (including ray_rgbT's presence) before enqueueing
  voro_status st = check_cameras(cams, V, &nr, &np);
  if (st != VORO_OK) return st;
  for (int v = 0; v < V; ++v)
    if (cams[v].spp > 1 && !ray_rgbT)
      return fail(VORO_EINVAL, "ray_rgbT is required when a view has spp > 1");
  st = views_common(false, scene, ws, ws_bytes, nullptr, cams, V, params, a, &nr, &np, &any_spp,
                    trace, trace_cap, stream);
  if (st != VORO_OK) return st;
  if (any_spp) {
    const int n = (int)np;
    hipLaunchKernelGGL(k_views_resolve, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       a.ct, reinterpret_cast<const float4*>(ray_rgbT), rgb, T, n);
    st = check_launch("voro_render_views_fwd: resolve");
  }
  return st;
}

voro_status voro_render_views_bwd(const voro_scene* scene, void* ws, size_t ws_bytes,
                                  const voro_camera* cams, int32_t V, const voro_params* params,
                                  const float* rgb, const float* T, const float* ray_rgbT,
                                  const int32_t* trace, int32_t trace_cap, const float* g_rgb,
                                  const float* g_T, float* g_sites, float* g_density,
                                  float* g_texels, uint64_t* stats, void* stream) {
  if (!rgb || !T || !g_rgb) return fail(VORO_EINVAL, "rgb, T and g_rgb must not be NULL");
  voro_status st0 = check_trace(trace, trace_cap);
  if (st0 != VORO_OK) return st0;
  if (!g_sites || !g_density || !g_texels)
    return fail(VORO_EINVAL, "gradient outputs must not be NULL");
  if (ray_rgbT && !aligned(ray_rgbT, 16)) return fail(VORO_EINVAL, "ray_rgbT must be 16-byte aligned");
  if (!aligned(g_texels, 16)) return fail(VORO_EINVAL, "g_texels must be 16-byte aligned");
  int64_t nr = 0, np = 0;
  voro_status st = check_cameras(cams, V, &nr, &np);
  if (st != VORO_OK) return st;
  for (int v = 0; v < V; ++v)
    if (cams[v].spp > 1 && !ray_rgbT)
      return fail(VORO_EINVAL, "ray_rgbT is required when a view has spp > 1");
  ViewsArgs a = {};
  a.rgb_in = rgb;
  a.T_in = T;
  a.ray_rgbT_in = ray_rgbT;
  a.g_rgb = g_rgb;
  a.g_T = g_T;
  a.g.texels = g_texels;
  a.g.maps = scene && scene->tex_maps == 2 ? 2 : 1;
  a.stats = reinterpret_cast<unsigned long long*>(stats);
  if (scene && ws) a.g.cell = cell_grads(scene, ws);
  bool any_spp = false;
  st = views_common(true, scene, ws, ws_bytes, nullptr, cams, V, params, a, &nr, &np, &any_spp,
                    const_cast<int32_t*>(trace), trace_cap, stream);
  if (st != VORO_OK) return st;
  return launch_fold_cell_grads(scene, ws, g_sites, g_density, (hipStream_t)stream);
}

}  // extern "C"
