// Greedy nearest-site walk over the packed Delaunay adjacency (device).
#pragma once

#include <hip/hip_runtime.h>

#include "voro_device.hpp"

namespace voro {

__device__ __forceinline__ double dist2_64(const float4 p, double ox, double oy, double oz) {
  const double dx = (double)p.x - ox;
  const double dy = (double)p.y - oy;
  const double dz = (double)p.z - oz;
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

// From `start`, move to the neighbour that is closest to x (FP64 squared
// distances, ties to the smaller index) while it beats the current site.
// Terminates: (distance, index) strictly decreases, so at most N moves.
__device__ __forceinline__ int nearest_walk(const DevScene& s, float fx, float fy, float fz,
                                            int start, bool* capped) {
  const double ox = fx, oy = fy, oz = fz;
  int cur = start;
  double dc = dist2_64(s.cells[2 * (size_t)cur], ox, oy, oz);
  for (int it = 0; it < s.n; ++it) {
    const Cell c = load_cell(s.cells, cur);
    int best = cur;
    double bd = dc;
    for (int e = 0; e < c.deg; ++e) {
      const int j = __float_as_int(s.edges[c.off + e].w);
      const double d2 = dist2_64(s.cells[2 * (size_t)j], ox, oy, oz);
      if (d2 < bd || (d2 == bd && j < best)) {
        bd = d2;
        best = j;
      }
    }
    if (best == cur) return cur;
    cur = best;
    dc = bd;
  }
  *capped = true;
  return cur;
}

}  // namespace voro
