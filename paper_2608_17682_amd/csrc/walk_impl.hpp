// The per-ray walk, forward and adjoint, as device functions shared by the
// explicit-ray kernels and the persistent multi-view kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "voro.h"
#include "voro_device.hpp"

namespace voro {

struct WalkParams {
  float t_stop;
  float skip_w;
  float tie_window;
  int max_steps;
};

struct RayIn {
  float ox, oy, oz;
  float dx, dy, dz;
  float tmax;
  int start;
};

struct RayOut {
  float r, g, b, T;
  int k;
};

// saved forward totals and upstream gradient of one ray
struct Upstream {
  float Cr, Cg, Cb, Tf;
  float gr, gg, gb, gT;
};

struct Grads {
  float* sites;    // [N,3]
  float* density;  // [N]
  float* texels;   // [N,R,R,4]
};

struct Counters {
  uint32_t rays = 0, steps = 0, deg = 0, maxsteps = 0, nan = 0, bad = 0, redecide = 0,
           skipped = 0;
};

// wave-reduce the per-lane counters and add them to stats (one lane per
// counter and wave).  Every lane of the wave must call this.
__device__ __forceinline__ void flush_counters(Counters c, bool contribute, int lane,
                                               unsigned long long* stats) {
  if (!contribute) c = Counters();
  const uint32_t v[8] = {c.rays, c.steps, c.deg, c.maxsteps, c.nan, c.bad, c.redecide, c.skipped};
  const int idx[8] = {VORO_STAT_RAYS,  VORO_STAT_STEPS,     VORO_STAT_DEGREE_SUM,
                      VORO_STAT_MAX_STEPS, VORO_STAT_NAN, VORO_STAT_BAD_START,
                      VORO_STAT_FP64_REDECIDE, VORO_STAT_SKIPPED};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t s = wave_sum_u32(v[k]);
    if (lane == 0 && s) atomicAdd(&stats[idx[k]], (unsigned long long)s);
  }
}

// One step of the walk: the exit of cell `cur` entered at t_in.
template <int LPR>
__device__ __forceinline__ Exit step_exit(const DevScene& s, const WalkParams& w, const RayIn& r,
                                          const Cell& c, int cur, float t_in, int sub) {
  const float qx = fmaf(t_in, r.dx, r.ox) - c.px;
  const float qy = fmaf(t_in, r.dy, r.oy) - c.py;
  const float qz = fmaf(t_in, r.dz, r.oz) - c.pz;
  const Top2 t2 = exit_search<LPR>(s.edges, c.off, c.deg, sub, qx, qy, qz, r.dx, r.dy, r.dz);
  return decide_exit(t2, s.cells, cur, t_in, w.tie_window, r.ox, r.oy, r.oz, r.dx, r.dy, r.dz);
}

template <int LPR, int TEX>
__device__ __forceinline__ RayOut walk_forward(const DevScene& s, const WalkParams& w,
                                               const RayIn& r, int sub, int32_t* rec,
                                               int max_record, Counters& cnt) {
  RayOut out;
  out.r = out.g = out.b = 0.0f;
  out.T = 1.0f;
  out.k = 0;
  if (!(r.tmax > 0.0f)) return out;
  if (r.start < 0 || r.start >= s.n) {
    cnt.bad++;
    return out;
  }
  cnt.rays++;
  const Taps tp = make_taps(r.dx, r.dy, r.dz, s.res);
  float T = 1.0f, Cr = 0.0f, Cg = 0.0f, Cb = 0.0f, t_in = 0.0f;
  int cur = r.start;
  int k = 0;
  for (;;) {
    const Cell c = load_cell(s.cells, cur);
    const Exit ex = step_exit<LPR>(s, w, r, c, cur, t_in, sub);
    cnt.redecide += ex.redecided ? 1u : 0u;
    cnt.deg += (uint32_t)c.deg;
    const Segment sg = segment(ex.t, r.tmax, t_in, c.sigma);
    const float wk = T * sg.alpha;
    if (wk >= w.skip_w) {
      float cr, cg, cb;
      texel_rgb<TEX>(s.texels, cur, s.res, tp, cr, cg, cb);
      Cr = fmaf(wk, cr, Cr);
      Cg = fmaf(wk, cg, Cg);
      Cb = fmaf(wk, cb, Cb);
    } else {
      cnt.skipped++;
    }
    T = T * sg.trans;
    if (rec && sub == 0 && k < max_record) rec[k] = cur;
    ++k;
    if (T < w.t_stop) break;
    if (!(ex.t < r.tmax) || ex.next < 0) break;
    if (k >= w.max_steps) {
      cnt.maxsteps++;
      break;
    }
    t_in = fmaxf(t_in, fminf(ex.t, r.tmax));
    cur = ex.next;
  }
  cnt.steps += (uint32_t)k;
  if (T != T) cnt.nan++;
  out.r = Cr;
  out.g = Cg;
  out.b = Cb;
  out.T = T;
  out.k = k;
  return out;
}

// dL/dt of the bisector crossing between cells a (left) and b (entered) at
// parameter t, pushed to both sites: dt/dp_a = (x - p_a)/beta,
// dt/dp_b = (p_b - x)/beta, x = o + t w, beta = (p_b - p_a).w.
__device__ __forceinline__ void flush_face(const DevScene& s, const Grads& g, const RayIn& r,
                                           int a, int b, float t, float coef) {
  const float4 A = s.cells[2 * (size_t)a];
  const float4 B = s.cells[2 * (size_t)b];
  const float nx = B.x - A.x;
  const float ny = B.y - A.y;
  const float nz = B.z - A.z;
  const float beta = dot3(nx, ny, nz, r.dx, r.dy, r.dz);
  const float xx = fmaf(t, r.dx, r.ox);
  const float xy = fmaf(t, r.dy, r.oy);
  const float xz = fmaf(t, r.dz, r.oz);
  const float c = coef / beta;
  atomicAdd(&g.sites[3 * (size_t)a], c * (xx - A.x));
  atomicAdd(&g.sites[3 * (size_t)a + 1], c * (xy - A.y));
  atomicAdd(&g.sites[3 * (size_t)a + 2], c * (xz - A.z));
  atomicAdd(&g.sites[3 * (size_t)b], c * (B.x - xx));
  atomicAdd(&g.sites[3 * (size_t)b + 1], c * (B.y - xy));
  atomicAdd(&g.sites[3 * (size_t)b + 2], c * (B.z - xz));
}

// Adjoint of walk_forward (replays it with identical decisions).
//   dL/dtau_k = g.(T_{k+1} c_k - S_k) - g_T T_final, S_k = C - sum_{j<=k} w_j c_j
//   dL/dsigma += dL/dtau_k delta_k, dL/dtexel_q += w_k b_q g,
//   each segment end moves with its bisector: +sigma_k dL/dtau_k at the exit
//   face, -sigma_k dL/dtau_k at the entry face (the crossing that last
//   advanced t); a face's two contributions are summed before it is flushed.
template <int LPR, int TEX>
__device__ __forceinline__ void walk_backward(const DevScene& s, const WalkParams& w,
                                              const RayIn& r, const Upstream& u, int sub,
                                              const Grads& g, Counters& cnt) {
  if (!(r.tmax > 0.0f)) return;
  if (r.start < 0 || r.start >= s.n) {
    cnt.bad++;
    return;
  }
  cnt.rays++;
  const int R = s.res;
  const Taps tp = make_taps(r.dx, r.dy, r.dz, R);
  float T = 1.0f, Pr = 0.0f, Pg = 0.0f, Pb = 0.0f, t_in = 0.0f;
  int cur = r.start;
  int k = 0;
  int fa = -1, fb = -1;
  float ft = 0.0f, fg = 0.0f;
  for (;;) {
    const Cell c = load_cell(s.cells, cur);
    const Exit ex = step_exit<LPR>(s, w, r, c, cur, t_in, sub);
    cnt.redecide += ex.redecided ? 1u : 0u;
    cnt.deg += (uint32_t)c.deg;
    const Segment sg = segment(ex.t, r.tmax, t_in, c.sigma);
    const float wk = T * sg.alpha;
    float cr, cg, cb;
    texel_rgb<TEX>(s.texels, cur, R, tp, cr, cg, cb);
    Pr = fmaf(wk, cr, Pr);
    Pg = fmaf(wk, cg, Pg);
    Pb = fmaf(wk, cb, Pb);
    const float Tn = T * sg.trans;
    const float Sr = u.Cr - Pr;
    const float Sg = u.Cg - Pg;
    const float Sb = u.Cb - Pb;
    const float dtau =
        fmaf(u.gb, Tn * cb - Sb, fmaf(u.gg, Tn * cg - Sg, u.gr * (Tn * cr - Sr))) - u.gT * u.Tf;
    if (sub == 0) {
      atomicAdd(&g.density[cur], dtau * sg.delta);
      float* tq = g.texels + ((size_t)cur * (size_t)(R * R) + (size_t)tp.base) * 4;
      const float q00 = wk * tp.w00, q01 = wk * tp.w01, q10 = wk * tp.w10, q11 = wk * tp.w11;
      atomicAdd(tq + 0, q00 * u.gr);
      atomicAdd(tq + 1, q00 * u.gg);
      atomicAdd(tq + 2, q00 * u.gb);
      atomicAdd(tq + 4, q01 * u.gr);
      atomicAdd(tq + 5, q01 * u.gg);
      atomicAdd(tq + 6, q01 * u.gb);
      float* tr = tq + 4 * R;
      atomicAdd(tr + 0, q10 * u.gr);
      atomicAdd(tr + 1, q10 * u.gg);
      atomicAdd(tr + 2, q10 * u.gb);
      atomicAdd(tr + 4, q11 * u.gr);
      atomicAdd(tr + 5, q11 * u.gg);
      atomicAdd(tr + 6, q11 * u.gb);
    }
    if (sg.delta > 0.0f) {
      const float dd = c.sigma * dtau;
      if (fa >= 0) fg -= dd;
      if (ex.t < r.tmax && ex.next >= 0) {
        if (fa >= 0 && sub == 0) flush_face(s, g, r, fa, fb, ft, fg);
        fa = cur;
        fb = ex.next;
        ft = ex.t;
        fg = dd;
      }
    }
    T = Tn;
    ++k;
    if (T < w.t_stop) break;
    if (!(ex.t < r.tmax) || ex.next < 0) break;
    if (k >= w.max_steps) {
      cnt.maxsteps++;
      break;
    }
    t_in = fmaxf(t_in, fminf(ex.t, r.tmax));
    cur = ex.next;
  }
  if (fa >= 0 && sub == 0) flush_face(s, g, r, fa, fb, ft, fg);
  cnt.steps += (uint32_t)k;
  if (T != T) cnt.nan++;
}

}  // namespace voro

namespace voro {
// host helpers (defined in walk.hip)
DevScene dev_scene(const voro_scene* s, const void* ws);
WalkParams walk_params(const voro_params* p);
}  // namespace voro
