/*
 * voro.h - C ABI of libvoro.so: the per-ray Voronoi cell walk of
 * differentiable Voronoi ray tracing, as hand-written HIP kernels for
 * MI355X (gfx950).
 *
 * What the library computes (paper sections in parentheses):
 *   - the cell containing a ray origin, i.e. the nearest site (Sec. 3.1,
 *     "Adjacency-Based Traversal": a single nearest-neighbour query);
 *   - the walk from that cell across the nearest forward crossing of the
 *     bisector planes between the current site and its Delaunay neighbours
 *     (Sec. 3.1 and the adjacency-walk figure);
 *   - per visited cell, opacity alpha = 1 - exp(-sigma * delta) and
 *     front-to-back compositing C = sum T_k alpha_k c_k with early
 *     termination on transmittance (Sec. 3.2 equations);
 *   - the cell colour c as a bilinear lookup of the cell's octahedral
 *     texture at the ray direction (Sec. 5.1 octahedral map; indexed by the
 *     ray direction, identity activation);
 *   - the adjoint of all of the above with respect to site positions,
 *     densities and texels (the quantities Sec. 5.5 optimises);
 *   - ray generation for pinhole, equidistant fisheye, rolling-shutter and
 *     thin-lens cameras (Sec. 6.5, App. D), and a persistent launch that
 *     renders several such views at once;
 *   - the Morton reordering of cells and the half-precision texel storage
 *     of Sec. 5.6 (inference optimisations).
 *
 * Conventions shared by every entry point:
 *   - Every pointer argument named *device* is caller-owned device memory
 *     of the current HIP device; the library allocates nothing, keeps no
 *     pointer after returning and never synchronises: work is enqueued on
 *     the given stream (NULL = the legacy default stream).  The caller
 *     keeps buffers alive until the stream has passed the work.
 *   - Arrays are dense, C order, without padding.  float = IEEE binary32.
 *   - Arguments are validated on the host before anything is enqueued; an
 *     invalid argument returns VORO_EINVAL (VORO_EUNSUPPORTED for features
 *     outside this build) and enqueues nothing.  voro_last_error() returns
 *     a description of the last failure on the calling thread.
 *   - Anomalies met on the device (walk step limit reached, NaN, start cell
 *     out of range, FP64 re-decisions, skipped texel lookups, malformed
 *     adjacency entries) are not errors: they are counted in the optional
 *     uint64 `stats` array (VORO_STAT_COUNT entries, accumulated with +=).
 *   - Calls on different streams may run concurrently as long as they do
 *     not share output or workspace buffers.
 */
#ifndef VORO_H
#define VORO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t voro_status;
enum {
  VORO_OK = 0,
  VORO_EINVAL = -1,       /* null pointer, bad size/enum/alignment/range */
  VORO_ENODEV = -2,       /* no usable HIP device */
  VORO_EHIP = -3,         /* a HIP runtime call or kernel launch failed */
  VORO_EUNSUPPORTED = -4, /* valid request outside this build's features */
  VORO_EWORKSPACE = -5    /* workspace missing or smaller than required */
};

/* texel storage types; compositing and gradients are always FP32 */
enum { VORO_TEX_F32 = 0, VORO_TEX_F16 = 1, VORO_TEX_BF16 = 2 };

/* camera models (Sec. 6.5 / App. D) */
enum {
  VORO_CAM_PINHOLE = 0,         /* f = (W/2)/tan(fov/2), fov horizontal */
  VORO_CAM_FISHEYE = 1,         /* equidistant: theta = r/f, f = (W/2)/(fov/2) */
  VORO_CAM_ROLLING_SHUTTER = 2, /* row y exposed at centre c + y/(H-1) * rs_delta */
  VORO_CAM_THIN_LENS = 3,       /* spp aperture samples per pixel, averaged */
  VORO_CAM_MOTION_BLUR = 4      /* spp time samples over the exposure, averaged */
};

/* indices into the optional uint64 stats array */
enum {
  VORO_STAT_RAYS = 0,          /* rays walked (tmax > 0 and valid start) */
  VORO_STAT_STEPS = 1,         /* cells visited, summed over rays (sum K(r)) */
  VORO_STAT_DEGREE_SUM = 2,    /* Delaunay degree of visited cells whose exit was
                                  searched (every step, unless a stored exit
                                  stood in for the search), summed */
  VORO_STAT_MAX_STEPS = 3,     /* rays cut by params.max_steps */
  VORO_STAT_NAN = 4,           /* rays whose transmittance became NaN */
  VORO_STAT_BAD_START = 5,     /* rays whose start cell was out of range */
  VORO_STAT_FP64_REDECIDE = 6, /* exit faces re-decided in FP64 (in searched steps) */
  VORO_STAT_SKIPPED = 7,       /* texel lookups skipped (weight < skip_w) */
  VORO_STAT_BAD_CSR = 8,       /* adjacency rows/entries found malformed by voro_prepare */
  VORO_STAT_LOCATE_CAP = 9,    /* nearest-site walks stopped by their step cap */
  VORO_STAT_COUNT = 16
};

#define VORO_MAX_VIEWS 16
#define VORO_MAX_TEX_RES 16
#define VORO_MIN_TEX_RES 2

/*
 * The scene.  All pointers are device memory.
 *   sites   [N,3] float   site positions p_i (Sec. 3.1)
 *   density [N]   float   sigma_i >= 0 (the caller applies sigma = exp(rho), Sec. 5.4)
 *   nbr_off [N+1] int32   CSR offsets of the symmetric Delaunay adjacency
 *   nbr_idx [M]   int32   CSR neighbour ids (no self loops)
 *   texels  [N,R,R,4]     per-cell octahedral texture, RGBA with A unused,
 *                         row index follows v, column index follows u;
 *                         float (16-byte aligned) or f16/bf16 (8-byte aligned);
 *           [N,2,R,R,4]   with tex_maps = 2: map 0 = surface map T_vi, map 1 =
 *                         view map T_vd, both RGB logits (Sec. 5.1, 5.2;
 *                         appearance 1)
 *           [N,48]        with tex_maps = 3: degree-3 spherical-harmonic RGB
 *                         coefficients, coefficient-major, index l^2 + l + m
 *                         (Sec. 3.3; appearance 2, forward only; 16-byte
 *                         aligned; tex_res is not used but must be valid)
 */
typedef struct voro_scene {
  int32_t n_sites;   /* N >= 1 */
  int32_t tex_res;   /* R in [VORO_MIN_TEX_RES, VORO_MAX_TEX_RES] */
  int32_t tex_dtype; /* VORO_TEX_* */
  int32_t tex_maps;  /* per-cell appearance: 0/1 = one map, 2 = surface + view, 3 = SH */
  int64_t n_edges;   /* M = nbr_off[N] < 2^31 */
  const float* sites;
  const float* density;
  const int32_t* nbr_off;
  const int32_t* nbr_idx;
  const void* texels;
} voro_scene;

/*
 * Render parameters; voro_default_params() fills the defaults.
 *   t_stop      early termination once T < t_stop after a segment (Sec. 3.2)  [1e-4]
 *   skip_w      skip the texel lookup of a segment whose compositing weight
 *               T*alpha < skip_w, still updating T (Sec. 5.6); 0 = never  [0]
 *   max_steps   cap on cells visited per ray (flagged in stats)         [4096]
 *   tie_window  exit faces whose FP32 crossings lie within
 *               tie_window * max(1, |t|) are re-decided in FP64          [1e-6]
 *   appearance  0 = single texture indexed by the ray direction, colour =
 *               the interpolated texel (needs tex_maps 0 or 1)            [0]
 *               1 = the full model of Sec. 5.1/5.2 (needs tex_maps = 2):
 *               c = sigmoid(T_vi(oct(x - p_i)) + T_vd(oct(-d))), x the point
 *               where the ray meets the cell - its entry point, or in the
 *               start cell (which holds the origin) its exit point clipped
 *               at tmax; x = p_i uses the ray direction instead of x - p_i
 *               2 = degree-3 spherical harmonics at the ray direction, the
 *               comparison model of Sec. 3.3 (needs tex_maps = 3; forward
 *               only)
 *   lanes_per_ray  1, 2, 4, 8 or 16 lanes cooperate on one ray's
 *               neighbour tests (0 = library default)                   [0]
 *   tile_w, tile_h  screen tile walked by one 64-lane wave, in rays;
 *               tile_w * tile_h * lanes_per_ray must equal 64 (0 = default)
 *   img_w       voro_render_fwd/bwd: when > 0 the R rays are row-major
 *               images of this width and waves take screen tiles; 0 = rays
 *               are walked in index order                               [0]
 *   max_record  cells recorded per ray in voro_render_fwd's `cells`     [0]
 *   block       threads per workgroup: 64, 128 or 256 (0 = 256)          [0]
 *   edge_fp16   forward-only inference variant (Sec. 5.6 "fp16 edge
 *               vectors"): neighbours are ranked from half-precision copies
 *               of the packed edge vectors (two per 16-byte load) and the
 *               winner's crossing is taken from its full-precision record;
 *               one lane per ray only.  A ray may take a different exit
 *               where two faces are within half-precision error.         [0]
 *   schedule    multi-view launches: VORO_SCHEDULE_GRID (one work tile per
 *               wave, hardware dispatch), VORO_SCHEDULE_PERSISTENT (waves
 *               loop over an XCD-partitioned tile queue) or
 *               VORO_SCHEDULE_REFILL (forward with one lane per ray: a wave
 *               owns a strip of 4 tiles and refills lanes whose ray ended,
 *               by ballot, once 16 are idle; the adjoint then uses the
 *               persistent queue); 0 = grid                            [0]
 */
typedef struct voro_params {
  float t_stop;
  float skip_w;
  int32_t max_steps;
  float tie_window;
  int32_t appearance;
  int32_t lanes_per_ray;
  int32_t tile_w;
  int32_t tile_h;
  int32_t img_w;
  int32_t max_record;
  int32_t block;
  int32_t schedule;
  int32_t edge_fp16;
  int32_t reserved[3]; /* must be 0 */
} voro_params;

enum {
  VORO_SCHEDULE_DEFAULT = 0,
  VORO_SCHEDULE_GRID = 1,
  VORO_SCHEDULE_PERSISTENT = 2,
  VORO_SCHEDULE_REFILL = 3
};

/*
 * A camera (Sec. 6.5 / App. D: only ray generation changes).  c2w is the
 * row-major 3x4 camera-to-world matrix whose columns are the camera's +x
 * (right), +y (down) and +z (forward) axes and its centre.  Pixel (x, y)
 * is sampled at its centre (x + 0.5, y + 0.5).  tmax is the ray extent.
 * Thin lens: spp = g*g stratum-centre samples mapped to the lens disk by the
 * concentric map (Shirley and Chiu 1997), each aimed at the pixel's pinhole
 * point on the plane at focus_dist along the axis.  Motion blur (Sec. 6.5:
 * time samples over the exposure, averaged): pinhole rays, sample s taken at
 * tau = (s + 0.5)/spp with the centre moved to c + tau * rs_delta (the
 * translation over the exposure; orientation fixed).  Fisheye pixels outside
 * the image circle emit no ray (tmax = 0: rgb = 0, T = 1).
 */
typedef struct voro_camera {
  int32_t model;   /* VORO_CAM_* */
  int32_t width;   /* >= 1 */
  int32_t height;  /* >= 1 (>= 2 for rolling shutter) */
  int32_t spp;     /* 1; a square <= 64 for THIN_LENS; 1..64 for MOTION_BLUR */
  float c2w[12];
  float fov;       /* radians, in (0, pi) for pinhole-type, (0, 2pi) fisheye */
  float tmax;      /* > 0 */
  float lens_radius;
  float focus_dist;
  float rs_delta[3]; /* rolling shutter: first -> last row; motion blur: over the exposure */
  int32_t reserved; /* must be 0 */
} voro_camera;

/* ---------------------------------------------------------------- info */

/* Library version string, e.g. "voro 0.1.0 gfx950". */
const char* voro_version(void);

/* Description of the last failing call on this thread ("" if none). */
const char* voro_last_error(void);

/* Fill *p with the defaults listed above.  VORO_EINVAL if p is NULL. */
voro_status voro_default_params(voro_params* p);

/* ---------------------------------------------------------- workspace */

/*
 * Bytes of device workspace the scene needs: packed cell records
 * (32 B per cell: position, density, adjacency row), packed edge records
 * (16 B per adjacency entry: (p_j - p_i)/|p_j - p_i|^2 and j, stored at the
 * adjacency's own offsets with no padding, so M records), their binary16
 * copies (8 B per entry, for the edge_fp16 variant), the nearest-site
 * search's partial results, the persistent launch's work counters and the
 * adjoint's per-cell gradient accumulator (16 B per cell; cleared by
 * voro_prepare and left clear by every adjoint call).  Host-only; needs no
 * device.
 */
voro_status voro_workspace_size(const voro_scene* scene, size_t* bytes);

/*
 * Pack the scene into the workspace (ws: device, 256-byte aligned, at least
 * voro_workspace_size bytes).  Must run (on the same stream, or ordered
 * before) after every change of sites, density or adjacency and before any
 * locate/render call that uses this workspace.  Malformed adjacency rows or
 * entries (offsets out of order or range, ids out of range, self loops) are
 * neutralised (never followed) and counted in stats[VORO_STAT_BAD_CSR].
 * stats may be NULL.
 */
voro_status voro_prepare(const voro_scene* scene, void* ws, size_t ws_bytes,
                         uint64_t* stats, void* stream);

/* ------------------------------------------------------------- locate */

/*
 * Nearest site to each origin (the cell containing it, Sec. 3.1), distances
 * compared in FP64 from the FP32 inputs; ties go to the smallest index.
 *   origins  [U,3] float device
 *   hint     [U] int32 device or NULL.  With a hint (or U > 64) each origin
 *            is found by a greedy walk over the Delaunay adjacency from the
 *            hint (from cell 0 without one): step to the closest neighbour
 *            while one is closer - exact, since a site that is not the
 *            nearest always has a closer Delaunay neighbour.  Without a hint
 *            and U <= 64, by a brute-force search over all sites.
 *   cell_out [U] int32 device
 * Requires voro_prepare on ws.  U = 0 is a no-op.
 */
voro_status voro_locate_origins(const voro_scene* scene, const void* ws, size_t ws_bytes,
                                const float* origins, const int32_t* hint, int32_t U,
                                int32_t* cell_out, uint64_t* stats, void* stream);

/* ------------------------------------------------------------- render */

/*
 * Forward render of R explicit rays (Sec. 3.1 walk, Sec. 3.2 compositing,
 * Sec. 5.1 appearance).
 *   o [R,3], d [R,3] (unit within 1e-6; not renormalised), tmax [R]
 *   start_cell [R] int32: the cell containing o (voro_locate_origins)
 *   rgb [R,3] out: premultiplied colour sum_k T_k alpha_k c_k (no background)
 *   T   [R]   out: transmittance after the last composited segment
 *   nsteps [R] int32 out or NULL: cells visited K(r)
 *   cells [R, params.max_record] int32 out or NULL: the first max_record
 *         visited cells per ray, -1 padded
 *   dist [R,3] float out or NULL: the ray's distortion loss (Sec. 5.3,
 *         eq. distortion-loss) sum_{k,l} w_k w_l |sbar_k - sbar_l| +
 *         1/3 sum_k w_k^2 ds_k over its segments, s(t) = 1 - 1/(1+t), then
 *         sum_k w_k sbar_k and sum_k w_k (kept for voro_render_bwd)
 *   trace [trace_cap][R][2] int32 out or NULL: each ray's first trace_cap
 *         exits, laid out and validated as for voro_render_views_fwd, for
 *         voro_render_bwd
 * Rays with tmax <= 0 return rgb = 0, T = 1, K = 0.  Start cells out of
 * range return rgb = 0, T = 1 and are counted.  Requires voro_prepare.
 */
voro_status voro_render_fwd(const voro_scene* scene, const void* ws, size_t ws_bytes,
                            const float* o, const float* d, const float* tmax,
                            const int32_t* start_cell, int32_t R, const voro_params* params,
                            float* rgb, float* T, int32_t* nsteps, int32_t* cells, float* dist,
                            int32_t* trace, int32_t trace_cap, uint64_t* stats, void* stream);

/*
 * Adjoint of voro_render_fwd for L = sum_r g_rgb[r].rgb[r] + g_T[r] T[r]
 * (+ g_dist[r] L_dist[r]).
 * Replays each ray's walk (same code, same cell sequence) and recovers the
 * back-to-front colour suffix from the saved forward totals rgb and T, so
 * nothing per step needs storing between the passes; with `trace` (the
 * exits voro_render_fwd stored for the same rays, scene and walk
 * parameters) the steps it holds are taken from it instead of searched,
 * as in voro_render_views_bwd.  Accumulates (+=) into
 *   g_sites [N,3], g_density [N] (dL/dsigma), g_texels [N,R,R,4] float
 *   ([N,2,R,R,4] with tex_maps = 2; A channel untouched), whatever the
 *   texel storage type.  Texel gradients are added with FP32 atomics;
 *   position and density gradients are first summed (FP32 atomics) into the
 *   workspace's per-cell accumulator, which a second kernel on the same
 *   stream adds into g_sites / g_density and clears again, so the
 *   workspace is written: no other call may use it until the stream has
 *   passed this one.
 * g_T may be NULL (zero).  dist [R,3] (voro_render_fwd's output) and g_dist
 * [R] add L += sum_r g_dist[r] dist[r,0]; both NULL or both given.
 * params.skip_w must be 0.  Gradients reach site
 * positions through the crossing parameters of the bisector faces and, with
 * appearance 1, through the surface direction x - p_i (x moving with the
 * crossing that places it); tmax, early termination and max_steps pass none.
 */
voro_status voro_render_bwd(const voro_scene* scene, void* ws, size_t ws_bytes,
                            const float* o, const float* d, const float* tmax,
                            const int32_t* start_cell, int32_t R, const voro_params* params,
                            const float* rgb, const float* T, const float* g_rgb,
                            const float* g_T, const float* dist, const float* g_dist,
                            const int32_t* trace, int32_t trace_cap, float* g_sites,
                            float* g_density, float* g_texels, uint64_t* stats, void* stream);

/* ------------------------------------------------------------ cameras */

/*
 * Number of rays and pixels of V cameras (host-only).  Rays are ordered view
 * by view, pixels row-major, then samples.
 */
voro_status voro_camera_counts(const voro_camera* cams, int32_t V, int64_t* n_rays,
                               int64_t* n_pixels);

/*
 * Generate all rays of V <= VORO_MAX_VIEWS cameras (cams: host array).
 *   o, d [n_rays,3], tmax [n_rays] float device out.
 */
voro_status voro_gen_rays(const voro_camera* cams, int32_t V, float* o, float* d,
                          float* tmax, void* stream);

/*
 * Forward render of V views in one launch: rays are generated in the
 * kernel, waves take screen tiles of any view (params.schedule: from the grid
 * or from a persistent XCD-partitioned queue), the start cell of each ray is
 * the cell of its camera centre (found by a brute-force search inside this
 * call) or, for rolling-shutter rows and thin-lens samples, reached from it
 * by the nearest-site walk.
 *   rgb [n_pixels,3], T [n_pixels] float out: per pixel (thin lens: the mean
 *   over its spp samples).
 *   ray_rgbT [n_rays,4] float out: per-ray (rgb, T); required when a view
 *   has spp > 1 (the backward needs it), may be NULL otherwise.
 *   nsteps [n_rays] int32 out or NULL.
 *   trace [trace_cap][n_rays][2] int32 out or NULL: the exit of each ray's
 *   step k < trace_cap (Sec. 3.1: the bisector crossing that ends the
 *   segment in the k-th visited cell) at trace[k][ray] = {exit parameter t
 *   as the bit pattern of its FP32 value, next cell (-1: none)}; entries at
 *   and beyond a ray's step count are left untouched.  Caller-owned device
 *   memory of trace_cap * n_rays * 8 bytes, 8-byte aligned; trace_cap >= 1
 *   when trace is given (else VORO_EINVAL), ignored when it is NULL.  Handed
 *   to voro_render_views_bwd, it spares the adjoint the exit searches.
 * params.tile_w/tile_h/lanes_per_ray pick the tiling; img_w, max_record are
 * ignored.  Requires voro_prepare.
 */
voro_status voro_render_views_fwd(const voro_scene* scene, void* ws, size_t ws_bytes,
                                  const voro_camera* cams, int32_t V, const voro_params* params,
                                  float* rgb, float* T, float* ray_rgbT, int32_t* nsteps,
                                  int32_t* trace, int32_t trace_cap, uint64_t* stats,
                                  void* stream);

/*
 * Adjoint of voro_render_views_fwd (one launch; workgroups walk workgroup
 * tiles and merge gradient records in LDS before the atomics).  rgb/T (and ray_rgbT
 * when a view has spp > 1) are the saved forward outputs; g_rgb [n_pixels,3]
 * and g_T [n_pixels] (or NULL) the upstream gradients; a thin-lens pixel's
 * gradient is shared equally by its samples.  Accumulates (+=) like
 * voro_render_bwd.
 *   trace, trace_cap: NULL, or the exits voro_render_views_fwd stored for
 *   the same scene, cameras and walk parameters (same trace_cap): the
 *   adjoint then takes steps k < trace_cap from it and searches only the
 *   steps beyond; the gradients are those of the search.  A stored next
 *   cell outside [0, n_sites) ends that ray's walk (never read out of
 *   bounds); any other mismatch gives wrong gradients, as mismatched rgb/T
 *   would.  trace_cap >= 1 when trace is given (else VORO_EINVAL).
 */
voro_status voro_render_views_bwd(const voro_scene* scene, void* ws, size_t ws_bytes,
                                  const voro_camera* cams, int32_t V, const voro_params* params,
                                  const float* rgb, const float* T, const float* ray_rgbT,
                                  const int32_t* trace, int32_t trace_cap, const float* g_rgb,
                                  const float* g_T, float* g_sites, float* g_density,
                                  float* g_texels, uint64_t* stats, void* stream);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): voro_render_views_fwd
 * with its scratch - the tile-queue counters, the camera centres and their
 * cells, the nearest-site search's partial results - in a static device
 * array of the library (about 65 KB per GPU, held until the process ends)
 * instead of the workspace.  The workspace is only read: it must hold the
 * records voro_prepare wrote (voro_workspace_size bytes always suffice).
 * Outputs, arguments, validation and results are those of
 * voro_render_views_fwd without a trace.  V above VORO_MAX_VIEWS (the scratch's maximum) is
 * rejected with VORO_EINVAL.  Nothing is allocated: no hipMalloc, hipFree or
 * allocating library routine is called (the first call on a device looks
 * the array's device address up).  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (different streams, or threads)
 * race and must be serialised by the caller.
 */
voro_status voro_render_views_fwd_noalloc(const voro_scene* scene, const void* ws,
                                          size_t ws_bytes, const voro_camera* cams, int32_t V,
                                          const voro_params* params, float* rgb, float* T,
                                          float* ray_rgbT, int32_t* nsteps, uint64_t* stats,
                                          void* stream);

/* ------------------------------------------------- scene preprocessing */

/*
 * Bytes of device scratch voro_morton_reorder needs (host-only).
 */
voro_status voro_reorder_scratch_size(int32_t n_sites, int64_t n_edges, size_t* bytes);

/*
 * Reorder the cells of `in` along a 3D Morton (Z-order) curve of their
 * positions (Sec. 5.6: cells close in space get close addresses).  Writes
 * the permuted scene into the caller's arrays of `out` (same sizes and
 * texel type as `in`; the adjacency ids are renumbered and each row keeps
 * its cells' neighbours), perm [N] (new -> old) and inv_perm [N]
 * (old -> new).  Morton codes use 10 bits per axis over the sites'
 * bounding box; equal codes keep their original order.  `out`'s pointers
 * are written through (cast from const).  scratch: device, >=
 * voro_reorder_scratch_size bytes.
 */
voro_status voro_morton_reorder(const voro_scene* in, const voro_scene* out, int32_t* perm,
                                int32_t* inv_perm, void* scratch, size_t scratch_bytes,
                                void* stream);

/*
 * Convert `count` floats to IEEE binary16 (dtype VORO_TEX_F16) or bfloat16
 * (VORO_TEX_BF16), rounding to nearest even (Sec. 5.6 half-precision
 * attributes).  src, dst device; dst holds `count` 16-bit values.
 */
voro_status voro_cast_texels(const float* src, void* dst, int64_t count, int32_t dtype,
                             void* stream);

#ifdef __cplusplus
}
#endif

#endif /* VORO_H */
