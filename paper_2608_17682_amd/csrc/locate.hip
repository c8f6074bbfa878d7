// The cell containing each ray origin: its nearest site (Sec. 3.1, the single
// nearest-neighbour query that starts the walk).  Distances are compared in
// FP64 from the FP32 inputs, ties going to the smallest index.
//
// Two exact strategies:
//  * brute force (few origins, e.g. one per pinhole view): a grid of
//    (chunk, origin) workgroups each reduce a chunk of sites, a second pass
//    reduces the chunks;
//  * greedy walk over the Delaunay adjacency from a hint (many origins, e.g.
//    thin-lens samples): move to the closest neighbour while one is closer.
//    Exact because a site that is not the nearest to x always has a Delaunay
//    neighbour closer to x; with (distance, index) ordered lexicographically
//    the walk strictly descends, so it ends after at most N moves.
#include <hip/hip_runtime.h>

#include "host_common.hpp"
#include "locate_impl.hpp"
#include "voro_device.hpp"
#include "walk_impl.hpp"

namespace voro {

struct BestD {
  double d2;
  int idx;
  int pad;
};

__device__ __forceinline__ bool better(double da, int ia, double db, int ib) {
  return (da < db) || (da == db && (unsigned)ia < (unsigned)ib);
}

__global__ void __launch_bounds__(256) k_locate_brute(const float* __restrict__ sites, int n,
                                                      const float* __restrict__ origins,
                                                      BestD* __restrict__ partial, int chunks) {
  const int u = blockIdx.y;
  const int chunk = blockIdx.x;
  const long per = ((long)n + chunks - 1) / chunks;
  const long lo = (long)chunk * per;
  const long hi = min((long)n, lo + per);
  const double ox = origins[3 * (size_t)u];
  const double oy = origins[3 * (size_t)u + 1];
  const double oz = origins[3 * (size_t)u + 2];
  double bd = __builtin_huge_val();
  int bi = 0x7fffffff;
  for (long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const double dx = (double)sites[3 * i] - ox;
    const double dy = (double)sites[3 * i + 1] - oy;
    const double dz = (double)sites[3 * i + 2] - oz;
    const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    if (better(d2, (int)i, bd, bi)) {
      bd = d2;
      bi = (int)i;
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const double od = __shfl_xor(bd, m);
    const int oi = __shfl_xor(bi, m);
    if (better(od, oi, bd, bi)) {
      bd = od;
      bi = oi;
    }
  }
  __shared__ double sd[16];
  __shared__ int si[16];
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sd[wave] = bd;
    si[wave] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < nw; ++k)
      if (better(sd[k], si[k], bd, bi)) {
        bd = sd[k];
        bi = si[k];
      }
    BestD r;
    r.d2 = bd;
    r.idx = bi;
    r.pad = 0;
    partial[(size_t)u * chunks + chunk] = r;
  }
}

__global__ void __launch_bounds__(64) k_locate_final(const BestD* __restrict__ partial, int chunks,
                                                     int32_t* __restrict__ out) {
  const int u = blockIdx.x;
  double bd = __builtin_huge_val();
  int bi = 0x7fffffff;
  for (int c = threadIdx.x; c < chunks; c += 64) {
    const BestD r = partial[(size_t)u * chunks + c];
    if (better(r.d2, r.idx, bd, bi)) {
      bd = r.d2;
      bi = r.idx;
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const double od = __shfl_xor(bd, m);
    const int oi = __shfl_xor(bi, m);
    if (better(od, oi, bd, bi)) {
      bd = od;
      bi = oi;
    }
  }
  if (threadIdx.x == 0) out[u] = bi;
}

__global__ void __launch_bounds__(256) k_locate_walk(DevScene s, const float* __restrict__ origins,
                                                     const int32_t* __restrict__ hint, int U,
                                                     int32_t* __restrict__ out,
                                                     unsigned long long* stats) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t capped = 0;
  if (u < U) {
    int h = hint ? hint[u] : 0;
    if (h < 0 || h >= s.n) h = 0;
    bool cap = false;
    out[u] = nearest_walk(s, origins[3 * (size_t)u], origins[3 * (size_t)u + 1],
                          origins[3 * (size_t)u + 2], h, &cap);
    capped = cap ? 1u : 0u;
  }
  if (stats) {
    const uint32_t c = wave_sum_u32(capped);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(&stats[VORO_STAT_LOCATE_CAP], (unsigned long long)c);
  }
}

// Brute-force nearest sites of U <= kLocateBruteMax origins into out (device);
// partials: U * kLocateChunks * 16 bytes of device scratch.
voro_status launch_locate_brute(const voro_scene* scene, void* partials, const float* origins,
                                int U, int32_t* out, hipStream_t st) {
  BestD* partial = reinterpret_cast<BestD*>(partials);
  int chunks = (scene->n_sites + 4095) / 4096;
  chunks = max(1, min(chunks, kLocateChunks));
  hipLaunchKernelGGL(k_locate_brute, dim3(chunks, U), dim3(256), 0, st, scene->sites,
                     scene->n_sites, origins, partial, chunks);
  hipLaunchKernelGGL(k_locate_final, dim3(U), dim3(64), 0, st, partial, chunks, out);
  return check_launch("voro_locate_origins (brute force)");
}

}  // namespace voro

using namespace voro;

extern "C" voro_status voro_locate_origins(const voro_scene* scene, const void* ws,
                                           size_t ws_bytes, const float* origins,
                                           const int32_t* hint, int32_t U, int32_t* cell_out,
                                           uint64_t* stats, void* stream) {
  voro_status st;
  if ((st = check_scene(scene)) != VORO_OK) return st;
  if ((st = check_ws(scene, ws, ws_bytes)) != VORO_OK) return st;
  if (U < 0) return fail(VORO_EINVAL, "U must be >= 0");
  if (U == 0) return VORO_OK;
  if (!origins || !cell_out) return fail(VORO_EINVAL, "origins and cell_out must not be NULL");
  if ((st = check_device()) != VORO_OK) return st;
  const hipStream_t s = (hipStream_t)stream;
  if (!hint && U <= kLocateBruteMax) {
    const WsLayout L = ws_layout(scene->n_sites, scene->n_edges);
    // the partials' region of the workspace is scratch (const only in the signature)
    return launch_locate_brute(scene, (char*)const_cast<void*>(ws) + L.locate, origins, U, cell_out, s);
  }
  const DevScene d = dev_scene(scene, ws);
  hipLaunchKernelGGL(k_locate_walk, dim3((U + 255) / 256), dim3(256), 0, s, d, origins, hint, U,
                     cell_out, reinterpret_cast<unsigned long long*>(stats));
  return check_launch("voro_locate_origins (walk)");
}
