// Device-side building blocks of the Voronoi walk, shared by every kernel so
// that all launches (explicit rays, persistent multi-view, forward and
// adjoint) take bit-identical decisions for the same ray.
//
// Compiled with -ffp-contract=off: every fused multiply-add below is written
// out with fmaf, so no launch context can change the rounding.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "voro.h"

namespace voro {

constexpr float kInf = __builtin_huge_valf();

// ----------------------------------------------------------- packed scene
//
// Cell record, 32 bytes = two float4: {x, y, z, sigma}, {edge_off, deg, 0, 0}
// (the ints stored by bit pattern).  Edge record, 16 bytes: {m.x, m.y, m.z, j}
// with m = n / |n|^2, n = p_j - p_i (the quotient formed in FP64 from the FP32
// positions and rounded once) and j the neighbour id (bit pattern).  Row i
// holds deg consecutive records from edge_off = nbr_off[i]; an exit search
// reads groups of four, the last 0-3 records under a per-lane mask.
struct DevScene {
  const float4* __restrict__ cells;
  const float4* __restrict__ edges;
  const uint2* __restrict__ edges16;  // {m.x, m.y | m.z, 0} as binary16, same slots
  const void* __restrict__ texels;
  int n;
  int res;
};

struct Cell {
  float px, py, pz, sigma;
  int off, deg;
};

__device__ __forceinline__ Cell load_cell(const float4* __restrict__ cells, int i) {
  const float4 a = cells[2 * (size_t)i];
  const float4 b = cells[2 * (size_t)i + 1];
  Cell c;
  c.px = a.x;
  c.py = a.y;
  c.pz = a.z;
  c.sigma = a.w;
  c.off = __float_as_int(b.x);
  c.deg = __float_as_int(b.y);
  return c;
}

__device__ __forceinline__ float dot3(float ax, float ay, float az, float bx, float by, float bz) {
  return fmaf(az, bz, fmaf(ay, by, ax * bx));
}

// ----------------------------------------------------- exit-face search
//
// Among the Delaunay neighbours j of the current cell i, the ray leaves
// through the bisector it reaches first moving forward (Sec. 3.1).  With
// x_in = o + t_in w the entry point, q = x_in - p_i and n = p_j - p_i, the
// bisector of (p_i, p_j) is crossed at t_in + (|n|^2/2 - n.q) / (n.w), and
// only faces with n.w > 0 lie ahead.  Measuring from x_in keeps the numerator
// small (cell-sized), and an error in t_in cancels: the result is the plane's
// own crossing parameter.  Dividing numerator and denominator by |n|^2, the
// packed record m = n/|n|^2 gives u = (1 - m.(2q)) / (m.w), twice the
// distance from t_in, in three FMAs, three FMAs and a reciprocal.
//
// Inside a lane the search keeps the best u with its id and the second-best
// u by value; lanes sharing a ray merge lexicographically in (u, id).  When
// the best two lie within the tie window, every face whose FP32 crossing is
// within the window of the best is re-decided in FP64 (exact ties to the
// smaller id), so the result does not depend on the order or the lane split
// of the neighbour list.
struct Best {
  float t1;  // best crossing offset
  int j1;    // its neighbour (-1: none ahead)
  float t2;  // second-best crossing offset (value only)
};

__device__ __forceinline__ float cross_u(const float4& E, float q2x, float q2y, float q2z,
                                         float dx, float dy, float dz) {
  const float b = dot3(E.x, E.y, E.z, dx, dy, dz);
  const float a = fmaf(-E.z, q2z, fmaf(-E.y, q2y, fmaf(-E.x, q2x, 1.0f)));
  return b > 0.0f ? a * __builtin_amdgcn_rcpf(b) : kInf;
}

__device__ __forceinline__ void best_push(Best& r, float u, int j) {
  const bool lt = u < r.t1;
  r.t2 = __builtin_amdgcn_fmed3f(r.t1, r.t2, u);  // second smallest of {t1, t2, u}
  r.t1 = lt ? u : r.t1;
  r.j1 = lt ? j : r.j1;
}

// merge another lane's summary; symmetric, so both lanes of a pair agree
__device__ __forceinline__ void best_merge(Best& r, float u1, int k1, float u2) {
  const bool take = u1 < r.t1 || (u1 == r.t1 && (unsigned)k1 < (unsigned)r.j1);
  const float loser = take ? r.t1 : u1;
  const float s2 = u2 < r.t2 ? u2 : r.t2;
  r.t2 = loser < s2 ? loser : s2;
  r.t1 = take ? u1 : r.t1;
  r.j1 = take ? k1 : r.j1;
}

template <int LPR>
__device__ __forceinline__ Best exit_search(const float4* __restrict__ edges, int off, int deg,
                                            int sub, float qx, float qy, float qz, float dx,
                                            float dy, float dz) {
  const float q2x = 2.0f * qx, q2y = 2.0f * qy, q2z = 2.0f * qz;
  Best r;
  r.t1 = kInf;
  r.j1 = -1;
  r.t2 = kInf;
  const float4* e = edges + off;
  if constexpr (LPR == 1) {
    const int full = deg & ~3;
    for (int k = 0; k < full; k += 4) {
      const float4 E0 = e[k], E1 = e[k + 1], E2 = e[k + 2], E3 = e[k + 3];
      best_push(r, cross_u(E0, q2x, q2y, q2z, dx, dy, dz), __float_as_int(E0.w));
      best_push(r, cross_u(E1, q2x, q2y, q2z, dx, dy, dz), __float_as_int(E1.w));
      best_push(r, cross_u(E2, q2x, q2y, q2z, dx, dy, dz), __float_as_int(E2.w));
      best_push(r, cross_u(E3, q2x, q2y, q2z, dx, dy, dz), __float_as_int(E3.w));
    }
    const int rem = deg - full;
    if (rem > 0) {
      const float4 E0 = e[full];
      best_push(r, cross_u(E0, q2x, q2y, q2z, dx, dy, dz), __float_as_int(E0.w));
      if (rem > 1) {
        const float4 E1 = e[full + 1];
        best_push(r, cross_u(E1, q2x, q2y, q2z, dx, dy, dz), __float_as_int(E1.w));
        if (rem > 2) {
          const float4 E2 = e[full + 2];
          best_push(r, cross_u(E2, q2x, q2y, q2z, dx, dy, dz), __float_as_int(E2.w));
        }
      }
    }
  } else {
#pragma unroll 2
    for (int k = sub; k < deg; k += LPR) {
      const float4 E = e[k];
      best_push(r, cross_u(E, q2x, q2y, q2z, dx, dy, dz), __float_as_int(E.w));
    }
#pragma unroll
    for (int m = 1; m < LPR; m <<= 1) {
      const float u1 = __shfl_xor(r.t1, m);
      const int k1 = __shfl_xor(r.j1, m);
      const float u2 = __shfl_xor(r.t2, m);
      best_merge(r, u1, k1, u2);
    }
  }
  r.t1 *= 0.5f;
  r.t2 *= 0.5f;
  return r;
}

// ---- half-precision ranking (inference variant, Sec. 5.6 "fp16 edge
// vectors"): the same u from binary16 copies of m, two records per 16-byte
// load (one 8-byte load first when the row starts on an odd slot), with a
// bound on how far each face's u can lie from the u that the FP32 record
// gives.  With M = max |m16_c|, Q = |2q|_1, W = |w|_1 and the binary16
// rounding of m at most 2^-11 |m| per component:
//   |b32 - b16| <= Eb = 2^-10 M W,   |a32 - a16| <= Ea = 2^-10 M Q + 2^-21
// (the FP32 roundings of both sides are inside the doubled constants), so
// a face with b16 > 2 Eb certainly lies ahead, one with b16 <= -Eb certainly
// does not, and for the first kind
//   |u32 - u16| <= e = 2 (Ea + |u16| Eb) / b16 + 2^-20 |u16|
// (the last term for the approximate reciprocals).  Anything else (a face
// too close to parallel, a record out of the binary16 range) is `unsure`.
struct Rank16 {
  float lo1;   // smallest lower bound u16 - e
  int k1;      // its slot in the row
  float lo2;   // second smallest lower bound
  float hi;    // smallest upper bound u16 + e
  bool unsure;
};

__device__ __forceinline__ void rank16_push(Rank16& r, unsigned xy, unsigned z0, float q2x,
                                            float q2y, float q2z, float dx, float dy, float dz,
                                            float cQ, float cW, int k) {
  const float mx = (float)__builtin_bit_cast(_Float16, (uint16_t)(xy & 0xffffu));
  const float my = (float)__builtin_bit_cast(_Float16, (uint16_t)(xy >> 16));
  const float mz = (float)__builtin_bit_cast(_Float16, (uint16_t)(z0 & 0xffffu));
  const float b = dot3(mx, my, mz, dx, dy, dz);
  const float a = fmaf(-mz, q2z, fmaf(-my, q2y, fmaf(-mx, q2x, 1.0f)));
  const float M = fmaxf(fabsf(mx), fmaxf(fabsf(my), fabsf(mz)));
  const float Eb = M * cW;
  const float Ea = fmaf(M, cQ, 0x1p-21f);
  const bool ahead = b > 2.0f * Eb;        // false for NaN / inf records too
  const bool behind = b <= -Eb;
  r.unsure = r.unsure || !(ahead || behind);
  if (ahead) {
    const float rb = __builtin_amdgcn_rcpf(b);
    const float u = a * rb;
    const float au = fabsf(u);
    const float e = fmaf(au, 0x1p-20f, 2.0f * fmaf(au, Eb, Ea) * rb);
    const float lo = u - e;
    r.hi = fminf(r.hi, u + e);
    const bool lt = lo < r.lo1;
    r.lo2 = __builtin_amdgcn_fmed3f(r.lo1, r.lo2, lo);
    r.lo1 = lt ? lo : r.lo1;
    r.k1 = lt ? k : r.k1;
  }
}

// The slot that certainly holds the row's smallest FP32 crossing offset
// (doubled), or -1 when the half-precision bounds cannot tell.
__device__ __forceinline__ Rank16 rank16(const uint2* __restrict__ edges16, int off, int deg,
                                         float qx, float qy, float qz, float dx, float dy,
                                         float dz) {
  const float q2x = 2.0f * qx, q2y = 2.0f * qy, q2z = 2.0f * qz;
  const float cQ = 0x1p-10f * (fabsf(q2x) + fabsf(q2y) + fabsf(q2z));
  const float cW = 0x1p-10f * (fabsf(dx) + fabsf(dy) + fabsf(dz));
  Rank16 r;
  r.lo1 = kInf;
  r.k1 = -1;
  r.lo2 = kInf;
  r.hi = kInf;
  r.unsure = false;
  const uint2* e = edges16 + off;
  int k = 0;
  if ((off & 1) && deg > 0) {
    const uint2 h = e[0];
    rank16_push(r, h.x, h.y, q2x, q2y, q2z, dx, dy, dz, cQ, cW, 0);
    k = 1;
  }
  for (; k + 4 <= deg; k += 4) {
    const uint4 A = *reinterpret_cast<const uint4*>(e + k);
    const uint4 B = *reinterpret_cast<const uint4*>(e + k + 2);
    rank16_push(r, A.x, A.y, q2x, q2y, q2z, dx, dy, dz, cQ, cW, k);
    rank16_push(r, A.z, A.w, q2x, q2y, q2z, dx, dy, dz, cQ, cW, k + 1);
    rank16_push(r, B.x, B.y, q2x, q2y, q2z, dx, dy, dz, cQ, cW, k + 2);
    rank16_push(r, B.z, B.w, q2x, q2y, q2z, dx, dy, dz, cQ, cW, k + 3);
  }
  if (k + 2 <= deg) {
    const uint4 A = *reinterpret_cast<const uint4*>(e + k);
    rank16_push(r, A.x, A.y, q2x, q2y, q2z, dx, dy, dz, cQ, cW, k);
    rank16_push(r, A.z, A.w, q2x, q2y, q2z, dx, dy, dz, cQ, cW, k + 1);
    k += 2;
  }
  if (k < deg) {
    const uint2 h = e[k];
    rank16_push(r, h.x, h.y, q2x, q2y, q2z, dx, dy, dz, cQ, cW, k);
  }
  return r;
}

// Crossing parameter of the bisector of (p_i, p_j) in FP64 from the FP32
// inputs: t = n.(m - o) / (n.w), n = p_j - p_i, m = (p_i + p_j)/2; +inf
// when the face does not lie ahead.
__device__ __forceinline__ double cross64(const float4* __restrict__ cells, int i, int j, double ox,
                                          double oy, double oz, double dx, double dy, double dz) {
  const float4 a = cells[2 * (size_t)i];
  const float4 c = cells[2 * (size_t)j];
  const double nx = (double)c.x - (double)a.x;
  const double ny = (double)c.y - (double)a.y;
  const double nz = (double)c.z - (double)a.z;
  const double b = __dadd_rn(__dadd_rn(__dmul_rn(nx, dx), __dmul_rn(ny, dy)), __dmul_rn(nz, dz));
  if (!(b > 0.0)) return __builtin_huge_val();
  const double mx = 0.5 * ((double)a.x + (double)c.x);
  const double my = 0.5 * ((double)a.y + (double)c.y);
  const double mz = 0.5 * ((double)a.z + (double)c.z);
  const double num = __dadd_rn(__dadd_rn(__dmul_rn(nx, mx - ox), __dmul_rn(ny, my - oy)),
                               __dmul_rn(nz, mz - oz));
  return num / b;
}

// The exit of cell i: absolute exit parameter and the next cell (-1: none).
// Near ties of the FP32 search are re-decided in FP64.
struct Exit {
  float t;
  int next;
  bool redecided;
};

__device__ __forceinline__ Exit decide_exit(const Best& r, const float4* __restrict__ cells,
                                            const float4* __restrict__ edges, int i, int off,
                                            int deg, float t_in, float tie_window, float ox,
                                            float oy, float oz, float dx, float dy, float dz,
                                            float qx, float qy, float qz) {
  Exit x;
  x.redecided = false;
  if (r.j1 < 0) {
    x.t = kInf;
    x.next = -1;
    return x;
  }
  x.t = t_in + r.t1;
  x.next = r.j1;
  const float win = tie_window * fmaxf(1.0f, fabsf(x.t));
  if (r.t2 - r.t1 <= win) {
    // the same FP32 crossings as the search (halving is exact), so the best
    // and the runner-up are always among the candidates
    const float q2x = 2.0f * qx, q2y = 2.0f * qy, q2z = 2.0f * qz;
    double tb = __builtin_huge_val();
    int jb = -1;
    for (int k = 0; k < deg; ++k) {
      const float4 E = edges[off + k];
      const float u = 0.5f * cross_u(E, q2x, q2y, q2z, dx, dy, dz);
      if (u - r.t1 <= win) {
        const int j = __float_as_int(E.w);
        // The empty asm makes the ray's coordinates look redefined here, so
        // their FP64 conversions stay in this rarely taken branch; hoisted
        // out of the walk they would hold 12 VGPRs for the whole walk.
        float o0 = ox, o1 = oy, o2 = oz, d0 = dx, d1 = dy, d2 = dz;
        asm volatile("" : "+v"(o0), "+v"(o1), "+v"(o2), "+v"(d0), "+v"(d1), "+v"(d2));
        const double t = cross64(cells, i, j, o0, o1, o2, d0, d1, d2);
        if (t < tb || (t == tb && t < __builtin_huge_val() && j < jb)) {
          tb = t;
          jb = j;
        }
      }
    }
    if (jb >= 0) {
      x.t = (float)tb;
      x.next = jb;
    }
    x.redecided = true;
  }
  return x;
}

// ------------------------------------------------------ octahedral taps
//
// Sec. 5.1: q = d / |d|_1; upper hemisphere (d_z >= 0) -> (q_x, q_y), lower
// -> ((1-|q_y|) sgn q_x, (1-|q_x|) sgn q_y) with sgn(0) = +1.  Texel space
// is corner-aligned: x = (u+1)/2 (R-1), column c0 = min(floor x, R-2),
// fraction x - c0 (rows likewise from v).  The four taps are
// (r0,c0), (r0,c0+1), (r0+1,c0), (r0+1,c0+1).
struct Taps {
  int base;  // r0 * R + c0
  float w00, w01, w10, w11;
};

__device__ __forceinline__ float sgn_nz(float x) { return x >= 0.0f ? 1.0f : -1.0f; }

__device__ __forceinline__ Taps make_taps(float dx, float dy, float dz, int R) {
  const float s = fabsf(dx) + fabsf(dy) + fabsf(dz);
  const float qx = dx / s;
  const float qy = dy / s;
  float u, v;
  if (dz >= 0.0f) {
    u = qx;
    v = qy;
  } else {
    u = (1.0f - fabsf(qy)) * sgn_nz(qx);
    v = (1.0f - fabsf(qx)) * sgn_nz(qy);
  }
  const float x = (u + 1.0f) * 0.5f * (float)(R - 1);
  const float y = (v + 1.0f) * 0.5f * (float)(R - 1);
  int c0 = (int)floorf(x);
  int r0 = (int)floorf(y);
  c0 = max(0, min(c0, R - 2));
  r0 = max(0, min(r0, R - 2));
  const float fx = x - (float)c0;
  const float fy = y - (float)r0;
  Taps t;
  t.base = r0 * R + c0;
  t.w00 = (1.0f - fx) * (1.0f - fy);
  t.w01 = fx * (1.0f - fy);
  t.w10 = (1.0f - fx) * fy;
  t.w11 = fx * fy;
  return t;
}

// texel storage
template <int TEX>
struct TexelT;

template <>
struct TexelT<VORO_TEX_F32> {
  __device__ __forceinline__ static float4 load(const void* __restrict__ p, size_t idx) {
    return reinterpret_cast<const float4*>(p)[idx];
  }
};

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

template <>
struct TexelT<VORO_TEX_BF16> {
  __device__ __forceinline__ static float4 load(const void* __restrict__ p, size_t idx) {
    const uint2 v = reinterpret_cast<const uint2*>(p)[idx];
    return make_float4(bf16_to_f32(v.x & 0xffffu), bf16_to_f32(v.x >> 16),
                       bf16_to_f32(v.y & 0xffffu), bf16_to_f32(v.y >> 16));
  }
};

template <>
struct TexelT<VORO_TEX_F16> {
  __device__ __forceinline__ static float4 load(const void* __restrict__ p, size_t idx) {
    const uint2 v = reinterpret_cast<const uint2*>(p)[idx];
    const _Float16 a = __builtin_bit_cast(_Float16, (uint16_t)(v.x & 0xffffu));
    const _Float16 b = __builtin_bit_cast(_Float16, (uint16_t)(v.x >> 16));
    const _Float16 c = __builtin_bit_cast(_Float16, (uint16_t)(v.y & 0xffffu));
    const _Float16 d = __builtin_bit_cast(_Float16, (uint16_t)(v.y >> 16));
    return make_float4((float)a, (float)b, (float)c, (float)d);
  }
};

// Bilinear colour of cell i at the ray's taps.
template <int TEX>
__device__ __forceinline__ void texel_rgb(const void* __restrict__ tex, int i, int R, const Taps& tp,
                                          float& r, float& g, float& b) {
  const size_t base = (size_t)i * (size_t)(R * R) + (size_t)tp.base;
  const float4 a = TexelT<TEX>::load(tex, base);
  const float4 c = TexelT<TEX>::load(tex, base + 1);
  const float4 e = TexelT<TEX>::load(tex, base + R);
  const float4 f = TexelT<TEX>::load(tex, base + R + 1);
  r = fmaf(tp.w11, f.x, fmaf(tp.w10, e.x, fmaf(tp.w01, c.x, tp.w00 * a.x)));
  g = fmaf(tp.w11, f.y, fmaf(tp.w10, e.y, fmaf(tp.w01, c.y, tp.w00 * a.y)));
  b = fmaf(tp.w11, f.z, fmaf(tp.w10, e.z, fmaf(tp.w01, c.z, tp.w00 * a.z)));
}

// ------------------------------------------------ full appearance model
//
// Sec. 5.1/5.2: each cell holds two maps of RGB logits, [N, 2, R, R, 4]
// (map 0 = surface map, map 1 = view map); the colour is sigmoid(surface
// map at oct(x - p_i) + view map at oct(-w)), x the point where the ray
// meets the cell (its entry point; the exit point in the start cell).  The
// octahedral map is unchanged by positive scaling, so the surface taps take
// x - p_i as it is.

constexpr float kLog2e = 1.44269504088896341f;

__device__ __forceinline__ float sigmoid_f(float l) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-l * kLog2e));
}

// logits of cell i: surface map at taps ts (its four texels returned for the
// adjoint), view map at taps tv
template <int TEX>
__device__ __forceinline__ void full_logits(const void* __restrict__ tex, int i, int R,
                                            const Taps& ts, const Taps& tv, float& lr, float& lg,
                                            float& lb, float4& a, float4& b, float4& e,
                                            float4& f) {
  const size_t base = (size_t)(2 * i) * (size_t)(R * R) + (size_t)ts.base;
  a = TexelT<TEX>::load(tex, base);
  b = TexelT<TEX>::load(tex, base + 1);
  e = TexelT<TEX>::load(tex, base + R);
  f = TexelT<TEX>::load(tex, base + R + 1);
  float vr, vg, vb;
  texel_rgb<TEX>(tex, 2 * i + 1, R, tv, vr, vg, vb);
  lr = fmaf(ts.w11, f.x, fmaf(ts.w10, e.x, fmaf(ts.w01, b.x, ts.w00 * a.x))) + vr;
  lg = fmaf(ts.w11, f.y, fmaf(ts.w10, e.y, fmaf(ts.w01, b.y, ts.w00 * a.y))) + vg;
  lb = fmaf(ts.w11, f.z, fmaf(ts.w10, e.z, fmaf(ts.w01, b.z, ts.w00 * a.z))) + vb;
}

// d(u, v)/d(d) of the octahedral map at any direction d != 0: with
// s = |d|_1, q = d/s, dq_a/dd = (e_a - q_a sgn d)/s (sgn(0) = +1); upper
// hemisphere (u, v) = (qx, qy); lower du = -sgn qx sgn qy dqy and
// dv = -sgn qx sgn qy dqx.
__device__ __forceinline__ void oct_jacobian(float dx, float dy, float dz, float ju[3],
                                             float jv[3]) {
  const float inv = 1.0f / (fabsf(dx) + fabsf(dy) + fabsf(dz));
  const float qx = dx * inv, qy = dy * inv;
  const float sx = sgn_nz(dx), sy = sgn_nz(dy), sz = sgn_nz(dz);
  const float ax[3] = {(1.0f - qx * sx) * inv, -qx * sy * inv, -qx * sz * inv};
  const float ay[3] = {-qy * sx * inv, (1.0f - qy * sy) * inv, -qy * sz * inv};
  if (dz >= 0.0f) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ju[k] = ax[k];
      jv[k] = ay[k];
    }
  } else {
    const float m = -sx * sy;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ju[k] = m * ay[k];
      jv[k] = m * ax[k];
    }
  }
}

// --------------------------------------- spherical-harmonic comparison
//
// Sec. 3.3: c = sum_{l<=3} sum_m k_lm Y_l^m(w) with the real orthonormal
// harmonics (no Condon-Shortley phase), coefficient i = l^2 + l + m, stored
// per cell as 48 values (coefficient-major RGB).  The constants are the
// normalisations of the polynomial forms: 1/(2 sqrt(pi)); sqrt(3/(4 pi));
// sqrt(15/pi)/2, sqrt(5/pi)/4, sqrt(15/pi)/4; sqrt(35/(2 pi))/4,
// sqrt(105/pi)/2, sqrt(21/(2 pi))/4, sqrt(7/pi)/4, sqrt(105/pi)/4.
__device__ __forceinline__ void sh3_basis(float x, float y, float z, float Y[16]) {
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[0] = 0.28209479177387814f;
  Y[1] = 0.48860251190291992f * y;
  Y[2] = 0.48860251190291992f * z;
  Y[3] = 0.48860251190291992f * x;
  Y[4] = 1.0925484305920792f * (x * y);
  Y[5] = 1.0925484305920792f * (y * z);
  Y[6] = 0.31539156525252005f * fmaf(3.0f, zz, -1.0f);
  Y[7] = 1.0925484305920792f * (x * z);
  Y[8] = 0.54627421529603959f * (xx - yy);
  Y[9] = 0.59004358992664352f * (y * fmaf(3.0f, xx, -yy));
  Y[10] = 2.8906114426405538f * (x * y * z);
  Y[11] = 0.45704579946446572f * (y * fmaf(5.0f, zz, -1.0f));
  Y[12] = 0.37317633259011540f * (z * fmaf(5.0f, zz, -3.0f));
  Y[13] = 0.45704579946446572f * (x * fmaf(5.0f, zz, -1.0f));
  Y[14] = 1.4453057213202769f * (z * (xx - yy));
  Y[15] = 0.59004358992664352f * (x * fmaf(-3.0f, yy, xx));
}

// the 48 coefficients of cell i, streamed in 16-byte loads (12 for f32, 6
// for f16/bf16), dotted with the basis
template <int TEX>
__device__ __forceinline__ void sh3_colour(const void* __restrict__ tex, int i, const float Y[16],
                                           float& r, float& g, float& b) {
  float v[48];
  if constexpr (TEX == VORO_TEX_F32) {
    const float4* p = reinterpret_cast<const float4*>(tex) + (size_t)i * 12;
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      const float4 a = p[q];
      v[4 * q] = a.x;
      v[4 * q + 1] = a.y;
      v[4 * q + 2] = a.z;
      v[4 * q + 3] = a.w;
    }
  } else {
    const uint4* p = reinterpret_cast<const uint4*>(tex) + (size_t)i * 6;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const uint4 a = p[q];
      const uint2 lo = make_uint2(a.x, a.y), hi = make_uint2(a.z, a.w);
      const float4 fl = TexelT<TEX>::load(&lo, 0);
      const float4 fh = TexelT<TEX>::load(&hi, 0);
      v[8 * q] = fl.x;
      v[8 * q + 1] = fl.y;
      v[8 * q + 2] = fl.z;
      v[8 * q + 3] = fl.w;
      v[8 * q + 4] = fh.x;
      v[8 * q + 5] = fh.y;
      v[8 * q + 6] = fh.z;
      v[8 * q + 7] = fh.w;
    }
  }
  r = Y[0] * v[0];
  g = Y[0] * v[1];
  b = Y[0] * v[2];
#pragma unroll
  for (int k = 1; k < 16; ++k) {
    r = fmaf(Y[k], v[3 * k], r);
    g = fmaf(Y[k], v[3 * k + 1], g);
    b = fmaf(Y[k], v[3 * k + 2], b);
  }
}

// ---------------------------------------------------------- segment math
//
// Sec. 3.2: delta = max(min(exit, tmax) - t_in, 0), alpha = 1 - exp(-sigma
// delta), w = T alpha, T <- T exp(-sigma delta).
struct Segment {
  float delta;
  float trans;  // exp(-sigma delta)
  float alpha;
};

__device__ __forceinline__ Segment segment(float exit_t, float tmax, float t_in, float sigma) {
  Segment s;
  const float t_out = fminf(exit_t, tmax);
  s.delta = fmaxf(t_out - t_in, 0.0f);
  // exp(-x) = 2^(-x log2 e) on the transcendental unit (relative error a
  // few ulp, far inside the 1e-4 tolerance)
  s.trans = __builtin_amdgcn_exp2f(-(sigma * s.delta) * 1.44269504088896341f);
  s.alpha = 1.0f - s.trans;
  return s;
}

// ------------------------------------------------------- launch geometry
//
// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Renumber them so that each XCD walks one contiguous range of
// screen tiles and its L2 sees spatially coherent cells.
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  constexpr int X = 8;
  const int q = nblocks / X;
  const int r = nblocks % X;
  const int x = b % X;
  const int k = b / X;
  return x * q + min(x, r) + k;
}

// Map (logical block, wave, lane group) to a ray index, or -1.
struct RayMap {
  int n_rays;
  int img_w;   // 0: linear order
  int img_h;
  int tile_w;
  int tile_h;
  int blocks_x;  // image blocks per row (tiled mode)
};

template <int LPR>
__device__ __forceinline__ int map_ray(const RayMap& m, int lblock, int wave, int nwaves, int grp) {
  constexpr int RPW = 64 / LPR;  // rays per wave
  if (m.img_w <= 0) {
    const long r = ((long)lblock * nwaves + wave) * RPW + grp;
    return r < m.n_rays ? (int)r : -1;
  }
  // waves of a block form a wx x wy grid of tiles
  const int wx = nwaves >= 2 ? 2 : 1;
  const int bw = m.tile_w * wx;
  const int bh = m.tile_h * (nwaves / wx);
  const int bx = lblock % m.blocks_x;
  const int by = lblock / m.blocks_x;
  const int x = bx * bw + (wave % wx) * m.tile_w + grp % m.tile_w;
  const int y = by * bh + (wave / wx) * m.tile_h + grp / m.tile_w;
  if (x >= m.img_w || y >= m.img_h) return -1;
  return y * m.img_w + x;
}

// wave-wide sum of a 32-bit counter
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

}  // namespace voro
