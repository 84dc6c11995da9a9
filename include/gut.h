/*
 * gut.h -- C ABI of libgut, an MI355X (gfx950) rasterizer for 3D Gaussian
 * particles projected with the Unscented Transform (3DGUT, arXiv 2412.12507).
 *
 * The hot path is four calls, run in order on one HIP stream:
 *   gut_project     per (camera, particle): sigma points, 2D mean/covariance,
 *                   extent, tile rectangle, sort depth, SH colour
 *                   (Alg. 1 with Alg. 2, Eq. 6-10, Sec. 4.1)
 *   gut_bin         per-tile lists in depth order (Sec. 4.3), with the
 *                   tile culling of 3DGS / StopThePop (Sec. 4.1, 4.4)
 *   gut_render      per-tile front-to-back compositing (Eq. 5) with each
 *                   particle evaluated at its maximum response along the
 *                   pixel ray (Eq. 11, Sec. 4.2)
 *   gut_render_bwd  gradients w.r.t. means, scales, quaternions, opacities
 *                   and SH coefficients (Supp. B)
 * plus a continuous-batching serving loop (gut_serve_*).
 *
 * Conventions shared by every call:
 *  - Every array argument is a DEVICE pointer unless marked "host".  The
 *    caller allocates and owns every buffer; libgut allocates device memory
 *    only inside a gut_server (within its budget) and inside gut_bin for its
 *    tiny pinned read-back slot, and holds one static 64 MiB scratch array
 *    per GPU for gut_render_bwd_noalloc.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every call is asynchronous on it, except gut_bin, which waits once, for
 *    an event it records on the stream as soon as the visible-entry and pair
 *    counts exist (its later kernels are already queued behind that event).
 *  - Arrays are row-major, float32, contiguous.  Particle arrays are
 *    structure-of-arrays: means[n,3], scales[n,3], quats[n,4] (w,x,y,z; any
 *    non-zero quaternion, normalised inside), opacities[n], sh[n,K,3] with
 *    K = (sh_degree+1)^2.  The kernels take ACTIVATED parameters: scales > 0,
 *    opacities in (0,1).
 *  - Several cameras may be processed in one call.  Per-(camera, particle)
 *    arrays are laid out [n_cams, n, ...] (entry e = cam * n + i).  Per-pixel
 *    outputs are the cameras' images concatenated in order, each [H, W, ...].
 *    Tile ids are global: camera c's tiles start after all tiles of cameras
 *    0..c-1; gut_num_tiles gives the total.
 *  - Cameras use OpenCV axes (+x right, +y down, +z forward); pose (R, t) maps
 *    world to camera, x_c = R x_w + t.  Pixel (i, j) has its centre at
 *    (i + 1/2, j + 1/2).  A rolling-shutter camera exposes row r at time
 *    r/(H-1) between pose 0 and pose 1 (centre interpolated linearly,
 *    rotation spherically).
 *  - Errors: argument checks run before any launch and return GUT_E_INVALID
 *    (or GUT_E_UNSUPPORTED) without touching the GPU; a HIP failure returns
 *    GUT_E_HIP.  gut_last_error() gives a thread-local message for the last
 *    failure.  Nothing throws across the ABI.  NaN particle values are not
 *    checked.
 */
#ifndef GUT_H
#define GUT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GUT_OK = 0,
  GUT_E_INVALID = 1,     /* bad argument; nothing launched */
  GUT_E_CAPACITY = 2,    /* pair buffer too small; required size reported */
  GUT_E_HIP = 3,         /* a HIP runtime call failed */
  GUT_E_ADMISSION = 4,   /* serving: request can never fit the memory budget */
  GUT_E_UNSUPPORTED = 5, /* valid request outside what libgut supports */
  GUT_E_NOT_FOUND = 6    /* serving: unknown request id */
} gut_status;

typedef enum { GUT_PINHOLE = 0, GUT_FISHEYE_OPENCV = 1 } gut_model;
typedef enum { GUT_GLOBAL_SHUTTER = 0, GUT_ROLLING_TOP_TO_BOTTOM = 1 } gut_shutter;

/* Camera (host struct, passed by pointer to an array of n_cams).  Intrinsic D
 * and extrinsic W of Alg. 1.  model GUT_FISHEYE_OPENCV uses
 * theta_d = theta (1 + k1 theta^2 + k2 theta^4 + k3 theta^6 + k4 theta^8),
 * valid up to the first angle in (0, pi/2] where d theta_d/d theta = 0.
 * For a global shutter R1/t1 are ignored. */
typedef struct {
  int32_t model, shutter, width, height;
  double fx, fy, cx, cy, k[4];
  double R0[9], t0[3]; /* world->camera at exposure start (row-major) */
  double R1[9], t1[3]; /* world->camera at exposure end */
} gut_camera;

/* Particle set (Sec. 3): device pointers, borrowed for the duration of a call
 * (for the lifetime of a gut_server). */
typedef struct {
  int64_t n;
  int32_t sh_degree; /* 0..3 */
  int32_t reserved;
  const float* means;     /* [n,3]   */
  const float* scales;    /* [n,3]   */
  const float* quats;     /* [n,4]   */
  const float* opacities; /* [n]     */
  const float* sh;        /* [n,K,3] */
} gut_scene;

/* Method parameters.  gut_default_params fills: UT alpha=1, beta=2, kappa=0
 * (Sec. 4.4); alpha_min=1/255, alpha_max=0.99, t_min=1e-4, near_plane=0.2
 * (the 3DGS values the paper adopts); k_sigma_max=3 (extent cap); tile=16;
 * rs_iters=3 (rolling-shutter time iterations); bg = 0; kernel_degree=2.
 * kernel_degree n in [2, 8] selects the particle response
 * rho = exp(-lambda (omega^2)^(n/2)), the generalized Gaussian of degree n of
 * Supp. A, with lambda = 3^(2-n) / 2 so that every degree has the Gaussian's
 * response at canonical distance 3; n = 2 is the Gaussian exp(-omega^2 / 2)
 * of Eq. 11.  It applies to projection (the extent's cutoff distance),
 * rendering and the backward pass alike.
 * kbuffer k in [0, 16] (default 0): k > 0 selects "Ours (sorted)" of Sec. 4.3
 * in gut_render -- each pixel keeps its k farthest hits (distance along the
 * ray of tau_max) in a buffer and blends the nearest as the buffer overflows,
 * then the buffer nearest first (multi-layer alpha blending); n_contrib then
 * counts blended hits.  gut_render_bwd differentiates it in blend order.
 * It honours clip_depth (hybrid rendering, Sec. 6.2, renders primary rays
 * this way) and kernel_degree.  gut_serve_create returns GUT_E_UNSUPPORTED
 * for k > 0.
 * tile_cull (default 1): gut_bin keeps a tile of a particle's rectangle only
 * if the particle's extent ellipse (v - m)^T (k^2 Sigma')^-1 (v - m) <= 1
 * meets the tile's box -- the 2D conic drives the tiling and culling of 3DGS
 * and StopThePop (Sec. 4.1), which the method employs (Sec. 4.4); 0 keeps
 * every tile of the rectangle. */
typedef struct {
  float ut_alpha, ut_beta, ut_kappa;
  float alpha_min, alpha_max, t_min, near_plane, k_sigma_max;
  int32_t tile, rs_iters;
  float bg[3];
  int32_t kernel_degree;
  int32_t kbuffer;
  int32_t tile_cull;
} gut_params;

/* Outputs of gut_project (caller-allocated device arrays).
 *   rect   [C*n,4] int16  tile rectangle x0,y0,x1,y1 (inclusive, camera-local)
 *   tiles  [C*n]   uint32 tiles touched; 0 = culled
 *   depth  [C*n]   float  sort depth |mu - camera centre|
 *   rgb    [C*n,3] float  view-dependent colour max(0, 1/2 + SH)
 *   record [n,16]  float  render record: mu(3), opacity, M = S^-1 R^T (3x3,
 *                         rows padded to 4); written once per call
 *   mean2d [C*n,2] float  nullable: UT mean (Eq. 9); gut_bin needs it with tile_cull
 *   cov2d  [C*n,3] float  nullable: UT covariance xx, xy, yy (Eq. 10)
 *   extent [C*n,4] float  nullable (16-byte aligned): the extent ellipse
 *                         k^2 Sigma' (xx, xy, yy) and its cutoff k (Alg. 1
 *                         Extent); zeros for culled entries; gut_bin needs it
 *                         with tile_cull */
typedef struct {
  int16_t* rect;
  uint32_t* tiles;
  float* depth;
  float* rgb;
  float* record;
  float* mean2d;
  float* cov2d;
  float* extent;
} gut_projected;

void gut_default_params(gut_params* p);

/* Total tiles and pixels over n_cams cameras (host helpers; -1 on bad input). */
int64_t gut_num_tiles(const gut_camera* cams, int32_t n_cams, const gut_params* p);
int64_t gut_num_pixels(const gut_camera* cams, int32_t n_cams);

/* Alg. 1 / Alg. 2 for every (camera, particle).  A particle is culled
 * (tiles = 0) if its opacity is below alpha_min, any sigma point is invalid
 * for the camera, or its rectangle misses the image.  Requires n*n_cams <
 * 2^31 and n_cams <= 64. */
gut_status gut_project(const gut_scene* scene, const gut_camera* cams, int32_t n_cams,
                       const gut_params* p, const gut_projected* out, void* stream);

/* Workspace for gut_bin (bytes, 256-aligned base expected) for n particles
 * seen by the n_cams cameras (host array) and pair_capacity pairs: a count
 * matrix of ceil(n / 8192) rows by the cameras' total tile count (u32), 4 KiB,
 * and 16 bytes per pair.  0 on bad arguments. */
size_t gut_bin_workspace_bytes(int64_t n, const gut_camera* cams, int32_t n_cams, int64_t pair_capacity);

/* Global per-tile depth sort (Sec. 4.3): each tile's list holds the visible
 * entries whose rectangle covers it (and, with tile_cull, whose extent
 * ellipse meets it), ordered by (depth, entry id).  The lists are built by a
 * counting sort over tiles and a per-tile radix sort in LDS.
 *   tile_ranges [3T] uint32   out: [T,2] [start, end) of each tile in sorted_ids
 *                             (an empty list has start == end),
 *                             then [T] the render order: for each camera, its
 *                             camera-local tile indices with the longest lists
 *                             first (bucketed by floor(log2(length)); order
 *                             within a bucket unspecified), at the camera's
 *                             tile offset.  gut_render and gut_render_bwd take
 *                             tiles in this order to shorten the tail.
 *   sorted_ids  [pair_capacity] uint32 out: entry ids e = cam*n + i
 *   n_pairs     host int64*   out (nullable): number of pairs P
 * proj's rect (8-byte aligned), tiles and depth -- with tile_cull also
 * mean2d and extent -- are read as gut_project writes them (tiles[e] = the
 * area of rect[e], 0 when culled); tile_ranges must be 8-byte aligned.  The
 * workspace is gut_bin_workspace_bytes(n, cams, n_cams, pair_capacity).  If P >
 * pair_capacity nothing is written past the buffer, every tile's range is
 * empty, *n_pairs holds the required size and GUT_E_CAPACITY is returned. */
gut_status gut_bin(const gut_projected* proj, int64_t n, const gut_camera* cams, int32_t n_cams,
                   const gut_params* p, void* ws, size_t ws_bytes, int64_t pair_capacity,
                   uint32_t* tile_ranges, uint32_t* sorted_ids, int64_t* n_pairs, void* stream);

/* Eq. 5 front to back over each tile list with alpha = sigma * rho at tau_max
 * (Eq. 11); stops before a particle that would take T below t_min.
 *   clip_depth [P_px]  float   in, nullable: hybrid rendering (Sec. 6.2) --
 *                             each pixel's distance along its ray (from the
 *                             ray origin, world units) to the closest surface
 *                             intersection; a particle whose maximum-response
 *                             point lies farther is discarded for that pixel
 *                             (+inf: no clip).  NULL: no clipping.
 *   rgb       [P_px,3] float   out: C + T * bg
 *   T_final   [P_px]   float   out: final transmittance
 *   n_contrib [P_px]   uint32  out: list position + 1 of the last contributor
 *   n_eval    [P_px]   uint32  out, nullable: list entries evaluated
 * where P_px = gut_num_pixels(cams, n_cams). */
gut_status gut_render(const gut_projected* proj, int64_t n, const uint32_t* tile_ranges,
                      const uint32_t* sorted_ids, const gut_camera* cams, int32_t n_cams,
                      const gut_params* p, const float* clip_depth, float* rgb, float* T_final,
                      uint32_t* n_contrib, uint32_t* n_eval, void* stream);

/* Workspace for gut_render_bwd (bytes). */
size_t gut_render_bwd_workspace_bytes(int64_t n, int32_t n_cams);

/* Supp. B: gradients of a loss given dL/d(rgb) [P_px,3] and optionally
 * dL/d(T_final) [P_px] (nullable), recomputing the compositing front to back
 * from T_final and n_contrib.  clip_depth must be the array (or NULL) the
 * forward gut_render call used; the clip decision carries no gradient.  Gradients are w.r.t. the activated parameters
 * passed in `scene` and are OVERWRITTEN (summed over cameras):
 * g_means[n,3], g_scales[n,3], g_quats[n,4], g_opacities[n], g_sh[n,K,3].
 * No gradient flows through the sigma-point projection, the rectangles, the
 * sort order or the rolling-shutter exposure times (Sec. 4.1). */
gut_status gut_render_bwd(const gut_scene* scene, const gut_projected* proj,
                          const uint32_t* tile_ranges, const uint32_t* sorted_ids,
                          const gut_camera* cams, int32_t n_cams, const gut_params* p,
                          const float* clip_depth, const float* rgb, const float* T_final,
                          const uint32_t* n_contrib,
                          const float* d_rgb, const float* d_T, float* g_means, float* g_scales,
                          float* g_quats, float* g_opacities, float* g_sh, void* ws,
                          size_t ws_bytes, void* stream);

/* gut_render_bwd for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, results and errors as gut_render_bwd, without ws/ws_bytes:
 * the FP64 accumulators live in a static 64 MiB device array that the
 * library holds on each GPU it runs on until the process ends, so
 * gut_render_bwd_workspace_bytes(n, n_cams) must not exceed 64 MiB (about
 * 645k particles for one camera); larger calls return GUT_E_INVALID and
 * launch nothing.  It calls no allocating routine.  Every call on one GPU
 * shares that GPU's array (the accumulators are cleared at the start of each
 * call), so calls that overlap on one GPU -- on different streams or from
 * different host threads -- race and must be serialised by the caller. */
gut_status gut_render_bwd_noalloc(const gut_scene* scene, const gut_projected* proj,
                                  const uint32_t* tile_ranges, const uint32_t* sorted_ids,
                                  const gut_camera* cams, int32_t n_cams, const gut_params* p,
                                  const float* clip_depth, const float* rgb, const float* T_final,
                                  const uint32_t* n_contrib, const float* d_rgb,
                                  const float* d_T, float* g_means, float* g_scales,
                                  float* g_quats, float* g_opacities, float* g_sh, void* stream);

/* ---- Serving: continuous batching over a resident scene ----------------
 * A server keeps the scene resident, admits multi-camera requests while
 * device memory (mem_budget_bytes, one arena allocated at creation) and one
 * of max_slots execution slots are free, merges queued requests into one
 * batch per slot (at most max_batch_cams cameras), and runs each batch as
 * project -> bin -> one persistent render launch on the slot's own stream,
 * so batches overlap on the device.  Each request's images are written to the
 * caller's device buffers out_rgb[c] ([H_c, W_c, 3] float), which must stay
 * alive until the request completes.  Results are bitwise identical to
 * rendering the request alone. */
typedef struct gut_server gut_server;

typedef struct {
  double frames_per_s; /* cameras completed per second of wall time */
  double p50_ms, p99_ms, mean_ms, max_ms; /* completion - submission */
  double wall_s;
  int64_t submitted, completed, rejected, batches, cameras;
  int64_t peak_bytes; /* arena high-water mark */
} gut_serve_metrics;

gut_status gut_serve_create(const gut_scene* scene, const gut_params* p,
                            size_t mem_budget_bytes, int32_t max_slots, int32_t max_batch_cams,
                            gut_server** out);
/* Enqueue a request (cameras copied; out_rgb is a host array of n_cams device
 * pointers, copied).  GUT_E_ADMISSION if it can never fit the budget. */
gut_status gut_serve_submit(gut_server* s, const gut_camera* cams, int32_t n_cams,
                            float* const* out_rgb, uint64_t* request_id);
gut_status gut_serve_poll(gut_server* s, uint64_t id, int32_t* done);
gut_status gut_serve_wait(gut_server* s, uint64_t id);
/* Latency of a completed request in milliseconds. */
gut_status gut_serve_latency(gut_server* s, uint64_t id, double* ms);
gut_status gut_serve_stats(gut_server* s, gut_serve_metrics* out);
/* Reset the statistics window (latencies, counters, wall clock). */
gut_status gut_serve_reset_stats(gut_server* s);
gut_status gut_serve_destroy(gut_server* s);

const char* gut_status_string(gut_status st);
const char* gut_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GUT_H */
