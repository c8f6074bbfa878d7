// Scene preprocessing of Sec. 5.6: Morton (Z-order) reordering of cells so
// that cells close in space get close addresses, and half-precision texel
// storage.  Both run once per scene, outside a frame's timed work.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "host_common.hpp"

namespace voro {

struct ReorderScratch {
  size_t codes_in, codes_out, vals_in, deg, bbox, prim, total;
  size_t prim_bytes;  // rocPRIM's temporary storage (sort and scan share it)
};

static ReorderScratch reorder_layout(int n, int64_t m) {
  (void)m;
  ReorderScratch L;
  size_t sort_bytes = 0, scan_bytes = 0;
  (void)rocprim::radix_sort_pairs(nullptr, sort_bytes, (const unsigned*)nullptr, (unsigned*)nullptr,
                                  (const int*)nullptr, (int*)nullptr, (size_t)n, 0u, 30u);
  (void)rocprim::inclusive_scan(nullptr, scan_bytes, (const int*)nullptr, (int*)nullptr, (size_t)n,
                                rocprim::plus<int>());
  L.prim_bytes = sort_bytes > scan_bytes ? sort_bytes : scan_bytes;
  L.codes_in = 0;
  L.codes_out = align256(L.codes_in + (size_t)n * 4);
  L.vals_in = align256(L.codes_out + (size_t)n * 4);
  L.deg = align256(L.vals_in + (size_t)n * 4);
  L.bbox = align256(L.deg + (size_t)n * 4);
  L.prim = align256(L.bbox + 256 * 8 * 4);
  L.total = align256(L.prim + L.prim_bytes);
  return L;
}

constexpr int kBBoxBlocks = 256;

// per-block min/max of the sites -> partial[block][6]
__global__ void __launch_bounds__(256) k_bbox_partial(const float* __restrict__ sites, int n,
                                                      float* __restrict__ partial) {
  float lo[3] = {__builtin_huge_valf(), __builtin_huge_valf(), __builtin_huge_valf()};
  float hi[3] = {-__builtin_huge_valf(), -__builtin_huge_valf(), -__builtin_huge_valf()};
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float v = sites[3 * i + a];
      lo[a] = fminf(lo[a], v);
      hi[a] = fmaxf(hi[a], v);
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], m));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], m));
    }
  __shared__ float s[4][6];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 3; ++a) {
      s[w][a] = lo[a];
      s[w][3 + a] = hi[a];
    }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    float v = s[0][a];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) v = a < 3 ? fminf(v, s[k][a]) : fmaxf(v, s[k][a]);
    partial[blockIdx.x * 6 + a] = v;
  }
}

__device__ __forceinline__ unsigned spread3(unsigned x) {
  // insert two zero bits between the low 10 bits of x
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000ffu;
  x = (x | (x << 8)) & 0x0300f00fu;
  x = (x | (x << 4)) & 0x030c30c3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

__global__ void __launch_bounds__(256) k_morton(const float* __restrict__ sites, int n,
                                                const float* __restrict__ partial,
                                                unsigned* __restrict__ codes,
                                                int* __restrict__ vals) {
  __shared__ float bb[6];
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    float v = partial[a];
    for (int k = 1; k < kBBoxBlocks; ++k)
      v = a < 3 ? fminf(v, partial[k * 6 + a]) : fmaxf(v, partial[k * 6 + a]);
    bb[a] = v;
  }
  __syncthreads();
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned q[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float ext = bb[3 + a] - bb[a];
    const float t = ext > 0.0f ? (sites[3 * i + a] - bb[a]) / ext : 0.0f;
    int k = (int)(t * 1024.0f);
    k = k < 0 ? 0 : (k > 1023 ? 1023 : k);
    q[a] = (unsigned)k;
  }
  codes[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
  vals[i] = (int)i;
}

// gather the per-cell arrays in the new order; inverse permutation; degrees
__global__ void __launch_bounds__(256) k_permute_cells(
    const int* __restrict__ perm, int n, const float* __restrict__ sites_in,
    const float* __restrict__ dens_in, const int* __restrict__ off_in, float* __restrict__ sites_out,
    float* __restrict__ dens_out, int* __restrict__ inv_perm, int* __restrict__ deg) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int o = perm[k];
  sites_out[3 * k] = sites_in[3 * (size_t)o];
  sites_out[3 * k + 1] = sites_in[3 * (size_t)o + 1];
  sites_out[3 * k + 2] = sites_in[3 * (size_t)o + 2];
  dens_out[k] = dens_in[o];
  inv_perm[o] = (int)k;
  deg[k] = max(0, off_in[o + 1] - off_in[o]);
}

// texels of the new cell k are those of perm[k]; copied as 16-byte words
__global__ void __launch_bounds__(256) k_permute_texels(const int* __restrict__ perm, long n_words,
                                                        int words_per_cell,
                                                        const uint4* __restrict__ in,
                                                        uint4* __restrict__ out) {
  const long w = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= n_words) return;
  const long k = w / words_per_cell;
  const long r = w - k * words_per_cell;
  out[w] = in[(size_t)perm[k] * words_per_cell + r];
}

// 16 lanes per new row: copy and renumber its neighbour ids
__global__ void __launch_bounds__(256) k_permute_rows(const int* __restrict__ perm,
                                                      const int* __restrict__ inv_perm, int n,
                                                      int m, const int* __restrict__ off_in,
                                                      const int* __restrict__ idx_in,
                                                      int* __restrict__ off_out,
                                                      int* __restrict__ idx_out) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long k = gid >> 4;
  const int l = threadIdx.x & 15;
  if (k >= n) return;
  const int o = perm[k];
  const int s = off_in[o];
  const int e = off_in[o + 1];
  const int dst = off_out[k];
  // a malformed input row (offsets out of order or range) is left empty
  if (s < 0 || e < s || e > m || dst < 0 || dst > m - (e - s)) return;
  for (int t = l; t < e - s; t += 16) {
    const int j = idx_in[s + t];
    idx_out[dst + t] = (j >= 0 && j < n) ? inv_perm[j] : j;
  }
}

__global__ void k_set_first_zero(int* off) { off[0] = 0; }

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);  // round half to even on the dropped 16 bits
  return (uint16_t)(u >> 16);
}

__global__ void __launch_bounds__(256) k_cast(const float* __restrict__ src, uint16_t* __restrict__ dst,
                                              long count, int dtype) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float x = src[i];
  if (dtype == VORO_TEX_F16) {
    const _Float16 h = (_Float16)x;  // IEEE round to nearest even
    dst[i] = __builtin_bit_cast(uint16_t, h);
  } else {
    dst[i] = f32_to_bf16_rne(x);
  }
}

}  // namespace voro

using namespace voro;

extern "C" {

voro_status voro_reorder_scratch_size(int32_t n_sites, int64_t n_edges, size_t* bytes) {
  if (n_sites < 1 || n_edges < 0 || !bytes) return fail(VORO_EINVAL, "bad reorder size query");
  *bytes = reorder_layout(n_sites, n_edges).total;
  return VORO_OK;
}

voro_status voro_morton_reorder(const voro_scene* in, const voro_scene* out, int32_t* perm,
                                int32_t* inv_perm, void* scratch, size_t scratch_bytes,
                                void* stream) {
  voro_status st;
  if ((st = check_scene(in)) != VORO_OK) return st;
  if ((st = check_scene(out)) != VORO_OK) return st;
  if (out->n_sites != in->n_sites || out->n_edges != in->n_edges ||
      out->tex_res != in->tex_res || out->tex_dtype != in->tex_dtype ||
      (out->tex_maps == 2) != (in->tex_maps == 2) || (out->tex_maps == 3) != (in->tex_maps == 3))
    return fail(VORO_EINVAL, "out scene must match in scene sizes and texel type");
  if (!perm || !inv_perm) return fail(VORO_EINVAL, "perm and inv_perm must not be NULL");
  const int n = in->n_sites;
  const ReorderScratch L = reorder_layout(n, in->n_edges);
  if (!scratch || scratch_bytes < L.total)
    return fail(VORO_EWORKSPACE, "reorder scratch too small: %zu < %zu", scratch_bytes, L.total);
  if (!aligned(scratch, 256)) return fail(VORO_EINVAL, "scratch must be 256-byte aligned");
  if ((st = check_device()) != VORO_OK) return st;
  const hipStream_t s = (hipStream_t)stream;
  char* base = (char*)scratch;
  unsigned* codes_in = (unsigned*)(base + L.codes_in);
  unsigned* codes_out = (unsigned*)(base + L.codes_out);
  int* vals_in = (int*)(base + L.vals_in);
  int* deg = (int*)(base + L.deg);
  float* bbox = (float*)(base + L.bbox);
  void* prim = base + L.prim;
  const int blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_bbox_partial, dim3(kBBoxBlocks), dim3(256), 0, s, in->sites, n, bbox);
  hipLaunchKernelGGL(k_morton, dim3(blocks), dim3(256), 0, s, in->sites, n, bbox, codes_in, vals_in);
  if ((st = check_launch("voro_morton_reorder: codes")) != VORO_OK) return st;
  // stable LSD radix sort on the 30 code bits: equal codes keep their order
  size_t pb = L.prim_bytes;
  if (rocprim::radix_sort_pairs(prim, pb, codes_in, codes_out, vals_in, perm, (size_t)n, 0u, 30u,
                                s) != hipSuccess)
    return fail(VORO_EHIP, "voro_morton_reorder: radix sort failed");
  hipLaunchKernelGGL(k_permute_cells, dim3(blocks), dim3(256), 0, s, perm, n, in->sites,
                     in->density, in->nbr_off, const_cast<float*>(out->sites),
                     const_cast<float*>(out->density), inv_perm, deg);
  int* off_out = const_cast<int*>(out->nbr_off);
  pb = L.prim_bytes;
  if (rocprim::inclusive_scan(prim, pb, deg, off_out + 1, (size_t)n, rocprim::plus<int>(), s) !=
      hipSuccess)
    return fail(VORO_EHIP, "voro_morton_reorder: scan failed");
  hipLaunchKernelGGL(k_set_first_zero, dim3(1), dim3(1), 0, s, off_out);
  hipLaunchKernelGGL(k_permute_rows, dim3((int)(((long)n * 16 + 255) / 256)), dim3(256), 0, s, perm,
                     inv_perm, n, (int)in->n_edges, in->nbr_off, in->nbr_idx, off_out, const_cast<int*>(out->nbr_idx));
  const int esz = in->tex_dtype == VORO_TEX_F32 ? 4 : 2;
  // texel maps [R,R,4] per map, or 48 spherical-harmonic coefficients
  const int maps = in->tex_maps == 2 ? 2 : 1;
  const long bytes_per_cell = in->tex_maps == 3 ? 48L * esz
                                                : (long)maps * in->tex_res * in->tex_res * 4 * esz;
  const int words = (int)(bytes_per_cell / 16);
  const long n_words = (long)n * words;
  hipLaunchKernelGGL(k_permute_texels, dim3((int)((n_words + 255) / 256)), dim3(256), 0, s, perm,
                     n_words, words, reinterpret_cast<const uint4*>(in->texels),
                     reinterpret_cast<uint4*>(const_cast<void*>(out->texels)));
  return check_launch("voro_morton_reorder");
}

voro_status voro_cast_texels(const float* src, void* dst, int64_t count, int32_t dtype,
                             void* stream) {
  if (count < 0) return fail(VORO_EINVAL, "count must be >= 0");
  if (dtype != VORO_TEX_F16 && dtype != VORO_TEX_BF16)
    return fail(VORO_EINVAL, "dtype must be VORO_TEX_F16 or VORO_TEX_BF16");
  if (count == 0) return VORO_OK;
  if (!src || !dst) return fail(VORO_EINVAL, "src and dst must not be NULL");
  voro_status st;
  if ((st = check_device()) != VORO_OK) return st;
  hipLaunchKernelGGL(k_cast, dim3((int)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     src, reinterpret_cast<uint16_t*>(dst), (long)count, dtype);
  return check_launch("voro_cast_texels");
}

}  // extern "C"
