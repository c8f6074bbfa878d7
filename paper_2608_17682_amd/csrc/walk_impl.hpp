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
  int edge16;  // rank neighbours from the half-precision edge vectors
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
  float dist, dist_a, dist_w;  // distortion loss and its running totals (when asked for)
};

// saved forward totals and upstream gradient of one ray; with the
// distortion loss also its saved value and totals sum w sbar, sum w, and
// its upstream gradient
struct Upstream {
  float Cr, Cg, Cb, Tf;
  float gr, gg, gb, gT;
  float D, DA, DW, gD;
};

// Distortion loss (Sec. 5.3): s(t) = t / (1 + t) maps depth into [0, 1).
// Along a ray the intervals are ordered, so the pair sum runs on prefix
// sums: segment k adds 2 w_k (sbar_k W - A) + w_k^2 ds_k / 3, with W, A the
// sums of w and w sbar over the earlier segments.
__device__ __forceinline__ float dist_s(float t) { return t / (1.0f + t); }

// Gradient targets of the adjoint kernels.  Position and density gradients
// go to a per-cell accumulator in the workspace, dp in xyz and dsigma in w,
// so that one 16-byte slot (one cache line) takes all four terms of a cell;
// a second kernel then adds it into the caller's arrays.  Texel gradients go
// straight to the caller's array.
struct Grads {
  float4* cell;    // [N] workspace accumulator: (dp.x, dp.y, dp.z, dsigma)
  float* texels;   // [N,R,R,4], or [N,2,R,R,4] for the full appearance model
  int maps;        // texture maps per cell (1 or 2)
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

// Per-workgroup stats in LDS (index = VORO_STAT_*) for the persistent
// kernels, whose waves walk one ray per lane group per tile: after each tile
// the lanes add their counters there (per-ray events as one ballot count per
// wave, per-step sums as LDS atomics), so no counter and no cross-lane
// shuffle address stays live across the tile loop.
constexpr int kWgStats = 10;

__device__ __forceinline__ void wg_stats_clear(unsigned long long* s) {
  if (threadIdx.x < kWgStats) s[threadIdx.x] = 0ull;
}

// Every lane of the wave must call this; a lane's counters cover at most one
// ray since they were zeroed.
__device__ __forceinline__ void tile_counters_to_lds(const Counters& c, bool contribute,
                                                     bool capped, int lane,
                                                     unsigned long long* s) {
  const unsigned n_rays = __popcll(__ballot(contribute && c.rays != 0u));
  const unsigned n_bad = __popcll(__ballot(contribute && c.bad != 0u));
  const unsigned n_max = __popcll(__ballot(contribute && c.maxsteps != 0u));
  const unsigned n_nan = __popcll(__ballot(contribute && c.nan != 0u));
  const unsigned n_cap = __popcll(__ballot(contribute && capped));
  if (contribute) {
    if (c.steps) atomicAdd(&s[VORO_STAT_STEPS], (unsigned long long)c.steps);
    if (c.deg) atomicAdd(&s[VORO_STAT_DEGREE_SUM], (unsigned long long)c.deg);
    if (c.redecide) atomicAdd(&s[VORO_STAT_FP64_REDECIDE], (unsigned long long)c.redecide);
    if (c.skipped) atomicAdd(&s[VORO_STAT_SKIPPED], (unsigned long long)c.skipped);
  }
  if (lane == 0) {
    if (n_rays) atomicAdd(&s[VORO_STAT_RAYS], (unsigned long long)n_rays);
    if (n_bad) atomicAdd(&s[VORO_STAT_BAD_START], (unsigned long long)n_bad);
    if (n_max) atomicAdd(&s[VORO_STAT_MAX_STEPS], (unsigned long long)n_max);
    if (n_nan) atomicAdd(&s[VORO_STAT_NAN], (unsigned long long)n_nan);
    if (n_cap) atomicAdd(&s[VORO_STAT_LOCATE_CAP], (unsigned long long)n_cap);
  }
}

// after a barrier that follows every wave's last tile.  The thread index is
// read afresh (empty asm) so that the slot address is not kept live, or
// spilled, from the kernel's start.
__device__ __forceinline__ void wg_stats_flush(const unsigned long long* s,
                                               unsigned long long* stats) {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  if (t < kWgStats && s[t]) atomicAdd(&stats[t], s[t]);
}

// One step of the walk: the exit of cell `cur` entered at t_in.  lrow: the
// cell's edge row staged in LDS by the wave (one lane per ray), or null to
// gather it from global memory.  E16: rank a gathered row from its
// half-precision copy first (a template switch, so the exact walk's kernels
// do not carry that code's registers); a staged row is searched in FP32
// either way, which reads it from LDS and costs less than the ranking.
template <int LPR, bool E16 = false>
__device__ __forceinline__ Exit step_exit(const DevScene& s, const WalkParams& w, const RayIn& r,
                                          const Cell& c, int cur, float t_in, int sub,
                                          const float4* lrow = nullptr) {
  const float qx = fmaf(t_in, r.dx, r.ox) - c.px;
  const float qy = fmaf(t_in, r.dy, r.oy) - c.py;
  const float qz = fmaf(t_in, r.dz, r.oz) - c.pz;
  Best b;
  bool searched = false;
  if constexpr (LPR == 1 && E16) if (!lrow) {
    // Rank in half precision.  When the bounds leave a single face that can
    // hold the smallest FP32 crossing, and every other face lies beyond the
    // tie window from it, that face's FP32 record gives exactly what the
    // FP32 search would (its crossing, its id, no FP64 re-decision);
    // otherwise the row is searched in FP32.  Either way the walk is the
    // exact walk.
    const Rank16 h = rank16(s.edges16, c.off, c.deg, qx, qy, qz, r.dx, r.dy, r.dz);
    if (!h.unsure && h.k1 >= 0 && h.lo2 > h.hi) {
      const float4 E = s.edges[c.off + h.k1];
      const float u = cross_u(E, 2.0f * qx, 2.0f * qy, 2.0f * qz, r.dx, r.dy, r.dz);
      const float t1 = 0.5f * u;
      const float win = w.tie_window * fmaxf(1.0f, fabsf(t_in + t1));
      if (0.5f * h.lo2 - t1 > win) {
        b.t1 = t1;
        b.j1 = __float_as_int(E.w);
        b.t2 = 0.5f * h.lo2;
        searched = true;
      }
    } else if (!h.unsure && h.k1 < 0) {
      b.t1 = kInf;  // no face lies ahead
      b.j1 = -1;
      b.t2 = kInf;
      searched = true;
    }
  }
  if (searched) {
  } else if (LPR == 1 && lrow) {
    b = exit_search<1>(lrow, 0, c.deg, 0, qx, qy, qz, r.dx, r.dy, r.dz);
  } else {
    b = exit_search<LPR>(s.edges, c.off, c.deg, sub, qx, qy, qz, r.dx, r.dy, r.dz);
  }
  return decide_exit(b, s.cells, s.edges, cur, c.off, c.deg, t_in, w.tie_window, r.ox, r.oy, r.oz,
                     r.dx, r.dy, r.dz, qx, qy, qz);
}

// Full appearance model: the vector from the site to the point where the ray
// meets cell c (its entry point t_in; the clipped exit point in the start
// cell, step k = 0).  Zero when that point is the site itself.
__device__ __forceinline__ void hit_vector(const RayIn& r, const Cell& c, int k, float t_in,
                                           float exit_t, float& hx, float& hy, float& hz) {
  const float th = k > 0 ? t_in : fminf(exit_t, r.tmax);
  hx = fmaf(th, r.dx, r.ox) - c.px;
  hy = fmaf(th, r.dy, r.oy) - c.py;
  hz = fmaf(th, r.dz, r.oz) - c.pz;
}

// The taps a ray uses for every cell: the single map at +w (appearance 0)
// or the view map at -w (appearance 1; unused by appearance 2).
template <int APP>
__device__ __forceinline__ Taps ray_taps(const RayIn& r, int R) {
  return APP ? make_taps(-r.dx, -r.dy, -r.dz, R) : make_taps(r.dx, r.dy, r.dz, R);
}

// Forward walk state of one ray, so that a lane can hold a ray across the
// steps of a loop it shares with other rays (fwd_begin, fwd_step, fwd_end).
template <int APP>
struct FwdState {
  Taps tp;
  float Ysh[APP == 2 ? 16 : 1];
  float T, Cr, Cg, Cb, t_in;
  float dP, dQ, dW, dA, s0;
  int cur, k;
  // the record of cell cur, loaded as soon as cur is known (the exit
  // decision of the previous step), so that its latency overlaps that
  // step's texel lookup and compositing
  Cell nc;
};

// false: nothing to walk (tmax <= 0 or an invalid start cell)
template <int APP>
__device__ __forceinline__ bool fwd_begin(FwdState<APP>& st, const DevScene& s, const RayIn& r,
                                          Counters& cnt) {
  st.T = 1.0f;
  st.Cr = st.Cg = st.Cb = 0.0f;
  st.t_in = 0.0f;
  st.dP = st.dQ = st.dW = st.dA = st.s0 = 0.0f;
  st.k = 0;
  st.cur = r.start;
  if (!(r.tmax > 0.0f)) return false;
  if (r.start < 0 || r.start >= s.n) {
    cnt.bad++;
    return false;
  }
  cnt.rays++;
  st.nc = load_cell(s.cells, r.start);
  st.tp = ray_taps<APP>(r, s.res);
  if constexpr (APP == 2) sh3_basis(r.dx, r.dy, r.dz, st.Ysh);
  return true;
}

// Stored exits of a ray: step k's exit (parameter t by bit pattern, next
// cell) at p[k * stride] for k < cap, written by the forward and read by the
// adjoint instead of searching the step's edge row again (null: none).
using i32x2 = int __attribute__((ext_vector_type(2)));
struct ExitTrace {
  int2* p;
  unsigned stride;
  int cap;
};

// One visited cell (lrow: its edge row staged in LDS, or null); true when
// the ray has ended.
template <int LPR, int TEX, int APP, bool E16 = false>
__device__ __forceinline__ bool fwd_step(FwdState<APP>& st, const DevScene& s,
                                         const WalkParams& w, const RayIn& r, int sub,
                                         int32_t* rec, int max_record, Counters& cnt,
                                         bool dist_on, const float4* lrow = nullptr,
                                         const ExitTrace& xt = {}) {
  const int cur = st.cur;
  const float t_in = st.t_in;
  const Cell c = st.nc;
  const Exit ex = step_exit<LPR, E16>(s, w, r, c, cur, t_in, sub, lrow);
  if (xt.p && sub == 0 && st.k < xt.cap) {
    // streamed out (only the adjoint reads it back): a non-temporal store
    // leaves the caches to the walk's records
    const i32x2 e = {__float_as_int(ex.t), ex.next};
    __builtin_nontemporal_store(e, reinterpret_cast<i32x2*>(xt.p + (size_t)st.k * xt.stride));
  }
  if (ex.next >= 0) st.nc = load_cell(s.cells, ex.next);
  cnt.redecide += ex.redecided ? 1u : 0u;
  cnt.deg += (uint32_t)c.deg;
  const Segment sg = segment(ex.t, r.tmax, t_in, c.sigma);
  const float wk = st.T * sg.alpha;
  if (dist_on) {
    const float s1 = dist_s(fmaxf(t_in, fminf(ex.t, r.tmax)));
    const float sb = 0.5f * (st.s0 + s1);
    st.dP = fmaf(2.0f * wk, fmaf(sb, st.dW, -st.dA), st.dP);
    st.dQ = fmaf(wk * wk, s1 - st.s0, st.dQ);
    st.dW += wk;
    st.dA = fmaf(wk, sb, st.dA);
    st.s0 = s1;
  }
  if (wk >= w.skip_w) {
    float cr, cg, cb;
    if constexpr (APP == 0) {
      texel_rgb<TEX>(s.texels, cur, s.res, st.tp, cr, cg, cb);
    } else if constexpr (APP == 2) {
      sh3_colour<TEX>(s.texels, cur, st.Ysh, cr, cg, cb);
    } else {
      float hx, hy, hz;
      hit_vector(r, c, st.k, t_in, ex.t, hx, hy, hz);
      const bool on_site = hx == 0.0f && hy == 0.0f && hz == 0.0f;
      const Taps ts = make_taps(on_site ? r.dx : hx, on_site ? r.dy : hy,
                                on_site ? r.dz : hz, s.res);
      float lr, lg, lb;
      float4 ta, tb, te, tf;
      full_logits<TEX>(s.texels, cur, s.res, ts, st.tp, lr, lg, lb, ta, tb, te, tf);
      cr = sigmoid_f(lr);
      cg = sigmoid_f(lg);
      cb = sigmoid_f(lb);
    }
    st.Cr = fmaf(wk, cr, st.Cr);
    st.Cg = fmaf(wk, cg, st.Cg);
    st.Cb = fmaf(wk, cb, st.Cb);
  } else {
    cnt.skipped++;
  }
  st.T = st.T * sg.trans;
  if (rec && sub == 0 && st.k < max_record) rec[st.k] = cur;
  ++st.k;
  if (st.T < w.t_stop) return true;
  if (!(ex.t < r.tmax) || ex.next < 0) return true;
  if (st.k >= w.max_steps) {
    cnt.maxsteps++;
    return true;
  }
  st.t_in = fmaxf(t_in, fminf(ex.t, r.tmax));
  st.cur = ex.next;
  return false;
}

template <int APP>
__device__ __forceinline__ RayOut fwd_end(const FwdState<APP>& st, bool walked, Counters& cnt) {
  RayOut out;
  out.r = st.Cr;
  out.g = st.Cg;
  out.b = st.Cb;
  out.T = st.T;
  out.k = st.k;
  out.dist = fmaf(st.dQ, 1.0f / 3.0f, st.dP);
  out.dist_a = st.dA;
  out.dist_w = st.dW;
  if (walked) {
    cnt.steps += (uint32_t)st.k;
    if (st.T != st.T) cnt.nan++;
  }
  return out;
}

template <int LPR, int TEX, int APP, bool E16 = false>
__device__ __forceinline__ RayOut walk_forward(const DevScene& s, const WalkParams& w,
                                               const RayIn& r, int sub, int32_t* rec,
                                               int max_record, Counters& cnt,
                                               bool dist_on = false, const ExitTrace& xt = {}) {
  FwdState<APP> st;
  const bool walk = fwd_begin<APP>(st, s, r, cnt);
  if (walk)
    while (!fwd_step<LPR, TEX, APP, E16>(st, s, w, r, sub, rec, max_record, cnt, dist_on,
                                         nullptr, xt)) {
    }
  return fwd_end<APP>(st, walk, cnt);
}

// Wave-cooperative staging of edge rows (one lane per ray).  Rays of a
// coherent tile often stand in the same few cells: when the live lanes of
// the wave sit in at most kStageCells distinct cells whose rows (at most 64
// faces each) fit the wave's LDS slab together, the wave copies those rows
// into the slab, one coalesced load per row, and every live lane reads its
// row from there; otherwise each lane gathers its own row from global
// memory.  The choice is per wave and step (mixing both within one step was
// slower: the two loops then run one after the other), and the exit search
// sees the same records in the same order either way.
constexpr int kStageCells = 8;
constexpr int kStageRecords = 256;
constexpr int kStageBytesPerWave = kStageRecords * 16;
constexpr int kStageMaxGap = 8;

// Every lane of the wave must call this; alive: the lane's walk goes on, at
// cell cur with record c.  Returns the lane's staged row, or null when the
// wave's rows were not staged (then staged = false on every lane).
__device__ __forceinline__ const float4* stage_rows(const float4* __restrict__ edges, float4* slab,
                                                    bool alive, int cur, const Cell& c, int lane,
                                                    bool& staged) {
  unsigned long long pend = __ballot(alive);
  int mine = 0;
  int offs[kStageCells], degs[kStageCells];
  int n = 0, used = 0;
  bool fits = true;
#pragma unroll
  for (int q = 0; q < kStageCells; ++q) {
    if (pend == 0ull) break;
    const int leader = __ffsll((long long)pend) - 1;  // wave-uniform
    const int cl = __builtin_amdgcn_readlane(cur, leader);
    offs[q] = __builtin_amdgcn_readlane(c.off, leader);
    degs[q] = __builtin_amdgcn_readlane(c.deg, leader);
    const bool same = alive && cur == cl;
    pend &= ~__ballot(same);
    if (same) mine = used;
    fits = fits && degs[q] <= 64;
    used += degs[q];
    n = q + 1;
  }
  staged = pend == 0ull && fits && used <= kStageRecords;
  if (!staged) return nullptr;
  // the slab's previous rows have been read by every lane (LDS operations of
  // one wave complete in order)
  __builtin_amdgcn_wave_barrier();
  int base = 0;
#pragma unroll
  for (int q = 0; q < kStageCells; ++q) {
    if (q < n && lane < degs[q]) slab[base + lane] = edges[offs[q] + lane];
    base += q < n ? degs[q] : 0;
  }
  __builtin_amdgcn_wave_barrier();
  return slab + mine;
}

// walk_forward with one lane per ray and staged rows.  Every lane of the
// wave must call this (has_ray = false for lanes without a ray); slab: the
// wave's kStageBytesPerWave of LDS.
template <int TEX, int APP, bool E16 = false>
__device__ __forceinline__ RayOut walk_forward_staged(const DevScene& s, const WalkParams& w,
                                                      const RayIn& r, bool has_ray, int lane,
                                                      float4* slab, int32_t* rec, int max_record,
                                                      Counters& cnt, bool dist_on = false,
                                                      const ExitTrace& xt = {}) {
  FwdState<APP> st;
  const bool walk = has_ray && fwd_begin<APP>(st, s, r, cnt);
  bool alive = walk;
  // after a step whose rows could not be staged the wave waits `wait` steps
  // before it tries again, doubling the wait up to kStageMaxGap while it
  // keeps failing (rays that have spread apart seldom meet again soon, and
  // each failed try costs a full pass over kStageCells ballots)
  int wait = 0, gap = 1;
  while (__any(alive)) {
    const float4* row = nullptr;
    if (wait == 0) {
      // the row bounds for the staging (the record fwd_step will use)
      Cell c;
      if (alive) c = st.nc;
      bool staged;
      row = stage_rows(s.edges, slab, alive, st.cur, c, lane, staged);
      if (staged) {
        gap = 1;
      } else {
        wait = gap;
        gap = min(2 * gap, kStageMaxGap);
      }
    } else {
      --wait;
    }
    if (alive) {
      if (row)
        alive = !fwd_step<1, TEX, APP, E16>(st, s, w, r, 0, rec, max_record, cnt, dist_on, row, xt);
      else
        alive =
            !fwd_step<1, TEX, APP, E16>(st, s, w, r, 0, rec, max_record, cnt, dist_on, nullptr, xt);
    }
  }
  return fwd_end<APP>(st, walk, cnt);
}

// ------------------------------------------------------------- adjoint
//
// Adjoint of walk_forward for L = g.C + g_T T_final.  The walk is replayed
// with identical decisions (each exit searched again, or read from the
// forward's stored exits) and, per segment k (App. X of the derivation in
// the oracle's adjoint module):
//   dL/dtau_k  = g.(T_{k+1} c_k - S_k) - g_T T_final,  S_k = C - sum_{j<=k} w_j c_j
//   dL/dsigma  += dL/dtau_k delta_k,    dL/dtexel_q += w_k b_q g
//   the exit end of the segment moves with its bisector crossing (+D) and
//   the entry end, the crossing that last advanced t, with -D, where
//   D = sigma_k dL/dtau_k; for the bisector of (a, b) crossed at t,
//   dt/dp_a = (x - p_a)/beta, dt/dp_b = (p_b - x)/beta, beta = (p_b - p_a).w.
//
// Gradient traffic.  A visited cell receives contributions from its own
// segment and from its two faces on the ray, i.e. from three consecutive
// steps.  Each lane keeps a sliding window (previous cell, current cell, next
// cell) and emits a cell's finished record - dsigma, dp (3), 12 texel terms -
// once, one step after leaving it.  Before the atomics, the records of the
// whole wave are merged on a butterfly: partner lanes (lane ^ m) holding the
// same key (cell, texel quad) add up and one of them retires, so coherent
// rays crossing the same cell issue one set of atomics instead of one per
// lane.  Faces whose far cell has already been emitted (only after zero-length
// segments) go straight to the atomics.

__device__ __forceinline__ void atomic_site(const Grads& g, int cell, float x, float y, float z) {
  float* p = reinterpret_cast<float*>(g.cell + cell);
  atomicAdd(p, x);
  atomicAdd(p + 1, y);
  atomicAdd(p + 2, z);
}

// A record's key is (cell * maps + map) * R^2 + texel quad.  Address of term
// c (0..15): 0 dsigma, 1-3 dp, 4-15 the texel terms of taps (r0,c0),
// (r0,c0+1), (r0+1,c0), (r0+1,c0+1) x RGB of that map.
__device__ __forceinline__ float* record_addr(const Grads& g, int key, int c, int RR, int R) {
  const int cm = key / RR;
  const int base = key - cm * RR;
  const int cell = g.maps == 2 ? (cm >> 1) : cm;
  if (c < 4) return reinterpret_cast<float*>(g.cell + cell) + (c == 0 ? 3 : c - 1);
  const int t = (c - 4) / 3;
  const int ch = (c - 4) - 3 * t;
  return g.texels + ((size_t)cm * (size_t)RR + (size_t)base) * 4 + (t & 1) * 4 + (t >> 1) * 4 * R +
         ch;
}

// Per-wave LDS staging of records bound for global memory: 16 lanes then
// write one record's 16 terms with one instruction, so a record costs about
// four cache-line requests at the memory-side atomic units instead of
// sixteen.  The area holds `cap` records; more senders go in turns.  With
// the full appearance model the same area also stages the survivors bound
// for the workgroup table (see emit_records), laid out [record][kStageStride],
// and then holds a whole wave (64 records).
constexpr int kStageStride = 17;  // odd: both access patterns spread over the banks
struct Outbox {
  int* keys;    // [cap]
  float* vals;  // [kStageStride * cap]
  int cap;
};

// Every lane of the wave must call this; `send` lanes hand over (key, v).
__device__ __forceinline__ void outbox_send(const Outbox& ob, bool send, int key, const float* v,
                                            int lane, const Grads& g, int RR, int R) {
  const unsigned long long m = __ballot(send);
  if (m == 0ull) return;
  const int pos = __popcll(m & ((1ull << lane) - 1ull));
  const int total = __popcll(m);
  const int cap = ob.cap;
  for (int b0 = 0; b0 < total; b0 += cap) {
    if (send && pos >= b0 && pos < b0 + cap) {
      ob.keys[pos - b0] = key;
#pragma unroll
      for (int c = 0; c < 16; ++c) ob.vals[c * cap + pos - b0] = v[c];
    }
    __builtin_amdgcn_wave_barrier();
    const int n = min(cap, total - b0);
    for (int b = 0; b < n; b += 4) {
      const int r = b + (lane >> 4);
      const int c = lane & 15;
      if (r < n) {
        const float x = ob.vals[c * cap + r];
        if (x != 0.0f) atomicAdd(record_addr(g, ob.keys[r], c, RR, R), x);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Workgroup gradient table in LDS: open addressing on the record key
// (cell * R^2 + texel quad), 16 FP32 sums per entry stored term-major so
// that lanes adding to different entries hit different banks.  Records are
// added with LDS float atomics while the workgroup walks its rays; every
// entry then reaches global memory once, when the workgroup flushes.  A
// record that finds no slot within kTableProbes goes straight to global
// memory.  Capacity: as many entries as leave room for three workgroups
// of four waves per CU (a larger table that costs a workgroup, or more
// probes, measured slower; so did a smaller table with four workgroups).
constexpr int kTableProbes = 8;
constexpr int kTableCapSingle = 704;  // one texture map: 16-record outboxes beside it
// the persistent one-lane-per-ray single-map adjoint runs four workgroups of
// four waves per CU: 528 entries is the most that leaves LDS for four
constexpr int kTableCapQuad = 528;
constexpr int kTableCapFull = 512;    // two maps: the outboxes also stage a whole wave
constexpr int kOutboxSingle = 16;
constexpr int kOutboxFull = 64;

template <int APP>
struct TableShape {
  static constexpr int cap = APP == 1 ? kTableCapFull : kTableCapSingle;
  static constexpr int outbox = APP == 1 ? kOutboxFull : kOutboxSingle;
};

// The capacity is a compile-time constant: a run-time one made the adjoint
// spill registers to scratch memory.
template <int CAP>
struct GradTable {
  static constexpr int cap = CAP;
  int* keys;    // [cap], -1 = empty
  float* vals;  // [16][cap]
};

// home slot of a key: multiplicative hash scaled to [0, cap)
template <int CAP>
__device__ __forceinline__ int table_home(const GradTable<CAP>& t, int key) {
  const unsigned h = (unsigned)key * 2654435761u;
  return (int)(((unsigned long long)h * (unsigned)CAP) >> 32);
}

// all threads of the workgroup; needs a barrier before the table is used
template <int CAP>
__device__ __forceinline__ void table_clear(const GradTable<CAP>& t) {
  for (int i = threadIdx.x; i < t.cap; i += blockDim.x) {
    t.keys[i] = -1;
#pragma unroll
    for (int c = 0; c < 16; ++c) t.vals[c * t.cap + i] = 0.0f;
  }
}

// the record's table slot (claimed if new), or -1 when kTableProbes probes
// (linear, wrapping) find neither the key nor an empty slot
template <int CAP>
__device__ __forceinline__ int table_slot(const GradTable<CAP>& t, int key) {
  int slot = table_home(t, key);
  for (int p = 0; p < kTableProbes; ++p) {
    int k = __hip_atomic_load(&t.keys[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (k == -1) k = atomicCAS(&t.keys[slot], -1, key);
    if (k == -1 || k == key) return slot;
    slot = slot + 1 == t.cap ? 0 : slot + 1;
  }
  return -1;
}

// C0: the first term that may be nonzero (texel-only records start at 4)
template <int C0, int CAP>
__device__ __forceinline__ bool table_add(const GradTable<CAP>& t, int key, const float* v) {
  const int slot = table_slot(t, key);
  if (slot < 0) return false;
#pragma unroll
  for (int c = C0; c < 16; ++c)
    if (v[c] != 0.0f) atomicAdd(&t.vals[c * t.cap + slot], v[c]);
  return true;
}

// all threads of the workgroup, after a barrier: every entry to global
// memory once (16 consecutive threads per entry, one term each), and the
// table left empty (a barrier must follow)
template <int CAP>
__device__ __forceinline__ void table_flush(const GradTable<CAP>& t, const Grads& g, int RR,
                                            int R) {
  for (int i = threadIdx.x; i < t.cap * 16; i += blockDim.x) {
    const int slot = i >> 4;
    const int c = i & 15;
    const int key = t.keys[slot];
    if (key < 0) continue;
    const float x = t.vals[c * t.cap + slot];
    t.vals[c * t.cap + slot] = 0.0f;
    if (x != 0.0f) atomicAdd(record_addr(g, key, c, RR, R), x);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < t.cap; i += blockDim.x) t.keys[i] = -1;
}

// Value of lane ^ M, exchanged without the LDS: DPP quad permutations
// (xor 1, 2), a half-row mirror followed by a quad reversal (xor 7 then
// xor 3, i.e. xor 4), DPP row rotation by 8 (xor 8 within a row of 16) and
// the row/half swaps of permlane16/32 (xor 16, 32; element 0 holds the even
// row / lower half, element 1 the other).  Every lane of the wave must take
// part.  (A ds_swizzle for xor 4 goes through the LDS, which the gradient
// table keeps busy: the two DPP moves made the adjoint 2-6% faster.)
template <int M>
__device__ __forceinline__ int xor_lane(int x, int lane) {
  if constexpr (M == 1) {
    return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  } else if constexpr (M == 2) {
    return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  } else if constexpr (M == 4) {
    const int h = __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false);  // row_half_mirror
    return __builtin_amdgcn_update_dpp(0, h, 0x1B, 0xF, 0xF, false);  // quad_perm [3,2,1,0]
  } else if constexpr (M == 8) {
    return __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false); // row_ror:8
  } else if constexpr (M == 16) {
    const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return (lane & 16) ? (int)p[0] : (int)p[1];
  } else {
    const auto p = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (lane & 32) ? (int)p[0] : (int)p[1];
  }
}

// One butterfly level: partners holding the same key add up and the upper
// one retires (terms below C0 are zero by construction and not exchanged).
// Every lane of the wave must call this.
template <int M, int C0>
__device__ __forceinline__ void merge_level(int& key, float (&v)[16], int lane) {
  const int pk = xor_lane<M>(key, lane);
  const bool match = key >= 0 && pk == key;
  if (!__any(match)) return;
  // each partner term is added as it arrives (two registers in flight, not
  // sixteen)
  const bool add = match && (lane & M) == 0;
#pragma unroll
  for (int i = C0; i < 16; ++i) {
    const float p = __int_as_float(xor_lane<M>(__float_as_int(v[i]), lane));
    v[i] = add ? v[i] + p : v[i];
  }
  if (match && (lane & M) != 0) key = -1;
}

// Merge equal-key records of butterfly partners across the wave (lane ^ m
// for m = LPR .. 32), then add the survivors to the workgroup table (or, with
// no table, to global memory).  Every lane of the wave must call this (key <
// 0: no record).
// The texel term of tap t and channel ch is tap weight t x m_ch.  C0 = 4
// marks a texel-only record (ds and dp are zero and skipped).
// SPREAD: each survivor only claims its table slot and stages its terms;
// then 16 lanes per record add them, so one LDS add instruction covers four
// records instead of one term of every survivor.  It needs a few more
// registers: a win for the full appearance model, whose two records per step
// already hold it at two waves per SIMD (3.58 -> 3.02 ms per frame), a loss
// for the single map, which it would push from three waves to two.
template <int LPR, int C0, bool SPREAD, int CAP>
__device__ __forceinline__ void emit_records(int key, float ds, float px, float py, float pz,
                                             const Taps& tp, float mr, float mg, float mb, int lane,
                                             int RR, int R, const Grads& g,
                                             const GradTable<CAP>* tab,
                                             const Outbox& ob) {
  float v[16];
  v[0] = ds;
  v[1] = px;
  v[2] = py;
  v[3] = pz;
  const float q[4] = {tp.w00, tp.w01, tp.w10, tp.w11};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    v[4 + 3 * t] = q[t] * mr;
    v[5 + 3 * t] = q[t] * mg;
    v[6 + 3 * t] = q[t] * mb;
  }
  if constexpr (LPR <= 1) merge_level<1, C0>(key, v, lane);
  if constexpr (LPR <= 2) merge_level<2, C0>(key, v, lane);
  if constexpr (LPR <= 4) merge_level<4, C0>(key, v, lane);
  if constexpr (LPR <= 8) merge_level<8, C0>(key, v, lane);
  if constexpr (LPR <= 16) merge_level<16, C0>(key, v, lane);
  merge_level<32, C0>(key, v, lane);
  if constexpr (SPREAD) {
    int slot = -1;
    if (key >= 0 && tab) slot = table_slot(*tab, key);
    const unsigned long long m = __ballot(slot >= 0);
    if (m) {
      const int pos = __popcll(m & ((1ull << lane) - 1ull));
      if (slot >= 0) {
        ob.keys[pos] = slot;
#pragma unroll
        for (int c = C0; c < 16; ++c) ob.vals[pos * kStageStride + c] = v[c];
      }
      __builtin_amdgcn_wave_barrier();
      const int n = __popcll(m);
      for (int b = 0; b < n; b += 4) {
        const int r = b + (lane >> 4);
        const int c = lane & 15;
        if (r < n && c >= C0) {
          const float x = ob.vals[r * kStageStride + c];
          if (x != 0.0f) atomicAdd(&tab->vals[c * tab->cap + ob.keys[r]], x);
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    outbox_send(ob, key >= 0 && slot < 0, key, v, lane, g, RR, R);
  } else {
    const bool over = key >= 0 && !(tab && table_add<C0, CAP>(*tab, key, v));
    outbox_send(ob, over, key, v, lane, g, RR, R);
  }
}

// Every lane of the wave must call this; has_ray = false for lanes without a
// ray.  The loop runs until every lane's walk has ended, so the record merge
// always sees the full wave.
//
// Full appearance model (APP = 1): with c = sigmoid(l), dL/dl = w_k g c(1-c)
// per channel feeds the surface-map taps (in the cell's delayed record) and
// the view-map taps (a record of its own, sent at once).  The surface
// direction adds dL/dx = J^T dL/d(u,v) for the hit point x, J the
// octahedral map's Jacobian at x - p_i: -dL/dx goes to the site, and
// dL/dt_hit = dL/dx . w to the crossing that placed x (the entry face, or
// the start cell's exit face) through the same dt/dp as the segment ends.
//
// Distortion loss (dist_on): with G_k = dL_dist/dw_k, the chain through
// w_k = T_k - T_{k+1} gives dL_dist/dtau_k = G_k T_{k+1} - sum_{j>k} G_j w_j,
// and sum_j G_j w_j = 2 L_dist, so the suffix follows from the saved loss;
// the interval ends move with their crossings through
// dL_dist/dt = (dL/dsbar / 2 -+ dL/dds) s'(t), s'(t) = 1/(1+t)^2.
template <int LPR, int TEX, int APP, int CAP = TableShape<APP>::cap>
__device__ __forceinline__ void walk_backward(const DevScene& s, const WalkParams& w, const RayIn& r,
                                              const Upstream& u, bool has_ray, int sub, int lane,
                                              const Grads& g, const GradTable<CAP>* tab,
                                              const Outbox& ob, Counters& cnt,
                                              bool dist_on = false, const ExitTrace& xt = {}) {
  const int R = s.res;
  const int RR = R * R;
  constexpr int MAPS = APP ? 2 : 1;
  bool active = has_ray && r.tmax > 0.0f;
  if (active && (r.start < 0 || r.start >= s.n)) {
    cnt.bad++;
    active = false;
  }
  if (active) cnt.rays++;
  const bool lead = sub == 0;
  const Taps tp = ray_taps<APP>(r, R);
  float T = 1.0f, Pr = 0.0f, Pg = 0.0f, Pb = 0.0f, t_in = 0.0f;
  float dW = 0.0f, dA = 0.0f, dGW = 0.0f, s0 = 0.0f;  // distortion prefix sums
  int cur = active ? r.start : 0;
  // the current cell's position and density: loaded with the previous
  // step's exit (a step with a stored exit needs nothing else of its cell).
  // Single map only: the full model's adjoint would lose a wave per SIMD to
  // the registers it holds.
  constexpr bool kCarry = APP == 0;
  float4 here = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (kCarry && active) here = s.cells[2 * (size_t)cur];

  int k = 0;
  // previous cell's record (emitted one step late): its texel multipliers
  // and, for APP = 1, its surface taps
  int a_cell = -1;
  float a_ds = 0.0f, a_px = 0.0f, a_py = 0.0f, a_pz = 0.0f;
  float a_mr = 0.0f, a_mg = 0.0f, a_mb = 0.0f;
  Taps a_tp = tp;
  // position gradient already received by the cell entered next
  int c_cell = -1;
  float c_px = 0.0f, c_py = 0.0f, c_pz = 0.0f;
  // the entry face: cells (fa, fb) and dt/dp_fa, dt/dp_fb
  int fa = -1, fb = -1;
  float uax = 0.0f, uay = 0.0f, uaz = 0.0f, ubx = 0.0f, uby = 0.0f, ubz = 0.0f;
  for (;;) {
    if (!__any(active)) break;
    int e_key = -1;
    float e_ds = 0.0f, e_px = 0.0f, e_py = 0.0f, e_pz = 0.0f;
    float e_mr = 0.0f, e_mg = 0.0f, e_mb = 0.0f;
    Taps e_tp = tp;
    int v_key = -1;  // APP = 1: this cell's view-map record
    float v_mr = 0.0f, v_mg = 0.0f, v_mb = 0.0f;
    if (active) {
      Cell c;
      Exit ex;
      const bool stored = xt.p && k < xt.cap;
      if (stored) {
        // the forward's exit of this step (a next cell outside the scene,
        // which only a trace from another walk could hold, ends the ray)
        const int2 e = xt.p[(size_t)k * xt.stride];
        ex.t = __int_as_float(e.x);
        ex.next = e.y >= 0 && e.y < s.n ? e.y : -1;
        ex.redecided = false;
      }
      if (kCarry && stored) {
        c.px = here.x;
        c.py = here.y;
        c.pz = here.z;
        c.sigma = here.w;
        c.off = 0;
        c.deg = 0;
      } else {
        c = load_cell(s.cells, cur);
        if (!stored) ex = step_exit<LPR>(s, w, r, c, cur, t_in, sub);
      }
      float4 pn = here;
      if constexpr (kCarry) pn = ex.next >= 0 ? s.cells[2 * (size_t)ex.next] : here;
      cnt.redecide += ex.redecided ? 1u : 0u;
      cnt.deg += (uint32_t)c.deg;
      const Segment sg = segment(ex.t, r.tmax, t_in, c.sigma);
      const float wk = T * sg.alpha;
      float cr, cg, cb;
      Taps ts = tp;
      float gxx = 0.0f, gxy = 0.0f, gxz = 0.0f, dldt = 0.0f;
      float glr = 0.0f, glg = 0.0f, glb = 0.0f;
      if constexpr (APP == 0) {
        texel_rgb<TEX>(s.texels, cur, R, tp, cr, cg, cb);
      } else {
        float hx, hy, hz;
        hit_vector(r, c, k, t_in, ex.t, hx, hy, hz);
        const bool on_site = hx == 0.0f && hy == 0.0f && hz == 0.0f;
        ts = make_taps(on_site ? r.dx : hx, on_site ? r.dy : hy, on_site ? r.dz : hz, R);
        float lr, lg, lb;
        float4 ta, tb, te, tf;
        full_logits<TEX>(s.texels, cur, R, ts, tp, lr, lg, lb, ta, tb, te, tf);
        cr = sigmoid_f(lr);
        cg = sigmoid_f(lg);
        cb = sigmoid_f(lb);
        glr = wk * u.gr * cr * (1.0f - cr);
        glg = wk * u.gg * cg * (1.0f - cg);
        glb = wk * u.gb * cb * (1.0f - cb);
        if (!on_site) {
          // dL/d(u,v) of the bilinear surface lookup (taps held fixed)
          const float kR = 0.5f * (float)(R - 1);
          const float fx = ts.w01 + ts.w11;
          const float fy = ts.w10 + ts.w11;
          const float dur = kR * fmaf(fy, tf.x - te.x, (1.0f - fy) * (tb.x - ta.x));
          const float dug = kR * fmaf(fy, tf.y - te.y, (1.0f - fy) * (tb.y - ta.y));
          const float dub = kR * fmaf(fy, tf.z - te.z, (1.0f - fy) * (tb.z - ta.z));
          const float dvr = kR * fmaf(fx, tf.x - tb.x, (1.0f - fx) * (te.x - ta.x));
          const float dvg = kR * fmaf(fx, tf.y - tb.y, (1.0f - fx) * (te.y - ta.y));
          const float dvb = kR * fmaf(fx, tf.z - tb.z, (1.0f - fx) * (te.z - ta.z));
          const float gu = dot3(glr, glg, glb, dur, dug, dub);
          const float gv = dot3(glr, glg, glb, dvr, dvg, dvb);
          float ju[3], jv[3];
          oct_jacobian(hx, hy, hz, ju, jv);
          gxx = fmaf(gu, ju[0], gv * jv[0]);
          gxy = fmaf(gu, ju[1], gv * jv[1]);
          gxz = fmaf(gu, ju[2], gv * jv[2]);
          dldt = dot3(gxx, gxy, gxz, r.dx, r.dy, r.dz);
        }
      }
      Pr = fmaf(wk, cr, Pr);
      Pg = fmaf(wk, cg, Pg);
      Pb = fmaf(wk, cb, Pb);
      const float Tn = T * sg.trans;
      const float Sr = u.Cr - Pr;
      const float Sg = u.Cg - Pg;
      const float Sb = u.Cb - Pb;
      float dtau =
          fmaf(u.gb, Tn * cb - Sb, fmaf(u.gg, Tn * cg - Sg, u.gr * (Tn * cr - Sr))) - u.gT * u.Tf;
      float dist_in = 0.0f, dist_ex = 0.0f;  // dL_dist/dt of the interval's ends
      if (dist_on) {
        const float t1 = fmaxf(t_in, fminf(ex.t, r.tmax));
        const float s1 = dist_s(t1);
        const float sb = 0.5f * (s0 + s1);
        const float dsv = s1 - s0;
        const float Wle = dW + wk;
        const float Ale = fmaf(wk, sb, dA);
        const float Gk = 2.0f * (fmaf(sb, dW, -dA) + (u.DA - Ale) - sb * (u.DW - Wle)) +
                         (2.0f / 3.0f) * wk * dsv;
        const float GWle = fmaf(Gk, wk, dGW);
        dtau = fmaf(u.gD, fmaf(Gk, Tn, -(2.0f * u.D - GWle)), dtau);
        const float gsb = 2.0f * wk * (dW - (u.DW - Wle));
        const float gds = wk * wk * (1.0f / 3.0f);
        const float i0 = 1.0f / (1.0f + t_in);
        const float i1 = 1.0f / (1.0f + t1);
        dist_in = u.gD * fmaf(0.5f, gsb, -gds) * (i0 * i0);
        dist_ex = u.gD * fmaf(0.5f, gsb, gds) * (i1 * i1);
        dW = Wle;
        dA = Ale;
        dGW = GWle;
        s0 = s1;
      }
      // this cell's record starts with what its entry face already sent it,
      // less the hit point's own pull on the site
      float m_px = (c_cell == cur ? c_px : 0.0f) - gxx;
      float m_py = (c_cell == cur ? c_py : 0.0f) - gxy;
      float m_pz = (c_cell == cur ? c_pz : 0.0f) - gxz;
      int n_cell = -1;
      float n_px = 0.0f, n_py = 0.0f, n_pz = 0.0f;
      if (sg.delta > 0.0f) {
        const float D = c.sigma * dtau;
        // dL/dt of the entry end (the hit point rides on it when k > 0) and
        // of the exit end (the start cell's hit point rides on it)
        const float Din = (k > 0 ? dldt : 0.0f) - D + dist_in;
        const float Dex = D + (k == 0 ? dldt : 0.0f) + dist_ex;
        if (fa >= 0) {
          if (fa == a_cell) {
            a_px = fmaf(Din, uax, a_px);
            a_py = fmaf(Din, uay, a_py);
            a_pz = fmaf(Din, uaz, a_pz);
          } else if (lead) {
            atomic_site(g, fa, Din * uax, Din * uay, Din * uaz);
          }
          if (fb == cur) {
            m_px = fmaf(Din, ubx, m_px);
            m_py = fmaf(Din, uby, m_py);
            m_pz = fmaf(Din, ubz, m_pz);
          } else if (fb == a_cell) {
            a_px = fmaf(Din, ubx, a_px);
            a_py = fmaf(Din, uby, a_py);
            a_pz = fmaf(Din, ubz, a_pz);
          } else if (lead) {
            atomic_site(g, fb, Din * ubx, Din * uby, Din * ubz);
          }
        }
        if (ex.t < r.tmax && ex.next >= 0) {
          // exit end: along the exit face (cur -> next)
          if constexpr (!kCarry) pn = s.cells[2 * (size_t)ex.next];
          const float nx = pn.x - c.px;
          const float ny = pn.y - c.py;
          const float nz = pn.z - c.pz;
          const float beta = dot3(nx, ny, nz, r.dx, r.dy, r.dz);
          const float xx = fmaf(ex.t, r.dx, r.ox);
          const float xy = fmaf(ex.t, r.dy, r.oy);
          const float xz = fmaf(ex.t, r.dz, r.oz);
          const float ib = 1.0f / beta;
          uax = (xx - c.px) * ib;
          uay = (xy - c.py) * ib;
          uaz = (xz - c.pz) * ib;
          ubx = (pn.x - xx) * ib;
          uby = (pn.y - xy) * ib;
          ubz = (pn.z - xz) * ib;
          fa = cur;
          fb = ex.next;
          m_px = fmaf(Dex, uax, m_px);
          m_py = fmaf(Dex, uay, m_py);
          m_pz = fmaf(Dex, uaz, m_pz);
          n_cell = ex.next;
          n_px = Dex * ubx;
          n_py = Dex * uby;
          n_pz = Dex * ubz;
        }
      }
      // the previous cell is complete: emit it
      if (lead && a_cell >= 0) {
        e_key = (a_cell * MAPS) * RR + a_tp.base;
        e_ds = a_ds;
        e_px = a_px;
        e_py = a_py;
        e_pz = a_pz;
        e_mr = a_mr;
        e_mg = a_mg;
        e_mb = a_mb;
        e_tp = a_tp;
      }
      if constexpr (APP == 1) {
        if (lead) {
          v_key = (2 * cur + 1) * RR + tp.base;
          v_mr = glr;
          v_mg = glg;
          v_mb = glb;
        }
      }
      a_cell = cur;
      a_ds = dtau * sg.delta;
      a_px = m_px;
      a_py = m_py;
      a_pz = m_pz;
      if constexpr (APP == 0) {
        a_mr = wk * u.gr;
        a_mg = wk * u.gg;
        a_mb = wk * u.gb;
      } else {
        a_mr = glr;
        a_mg = glg;
        a_mb = glb;
        a_tp = ts;
      }
      c_cell = n_cell;
      c_px = n_px;
      c_py = n_py;
      c_pz = n_pz;
      T = Tn;
      ++k;
      bool stop = T < w.t_stop || !(ex.t < r.tmax) || ex.next < 0;
      if (!stop && k >= w.max_steps) {
        cnt.maxsteps++;
        stop = true;
      }
      if (stop) {
        active = false;
        cnt.steps += (uint32_t)k;
        if (T != T) cnt.nan++;
      } else {
        t_in = fmaxf(t_in, fminf(ex.t, r.tmax));
        cur = ex.next;
        if constexpr (kCarry) here = pn;
      }
    }
    emit_records<LPR, 0, APP == 1, CAP>(e_key, e_ds, e_px, e_py, e_pz, e_tp, e_mr, e_mg, e_mb, lane,
                                   RR, R, g, tab, ob);
    if constexpr (APP == 1)
      emit_records<LPR, 4, true, CAP>(v_key, 0.0f, 0.0f, 0.0f, 0.0f, tp, v_mr, v_mg, v_mb, lane, RR, R,
                                 g, tab, ob);
  }
  // the last visited cell, and the unvisited cell behind an early-stopped ray's exit face
  emit_records<LPR, 0, APP == 1, CAP>(lead && a_cell >= 0 ? (a_cell * MAPS) * RR + a_tp.base : -1,
                                 a_ds, a_px, a_py, a_pz, a_tp, a_mr, a_mg, a_mb, lane, RR, R, g,
                                 tab, ob);
  emit_records<LPR, 0, APP == 1, CAP>(lead && c_cell >= 0 ? (c_cell * MAPS) * RR + tp.base : -1, 0.0f,
                                 c_px, c_py, c_pz, tp, 0.0f, 0.0f, 0.0f, lane, RR, R, g, tab, ob);
}

}  // namespace voro

namespace voro {
// host helpers (defined in walk.hip)
DevScene dev_scene(const voro_scene* s, const void* ws);
WalkParams walk_params(const voro_params* p);
}  // namespace voro
