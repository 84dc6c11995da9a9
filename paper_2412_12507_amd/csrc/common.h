// Internal definitions shared by the libgut HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstdio>

#include "gut.h"

namespace gut {

constexpr int kTile = 16;
constexpr int kTilePix = kTile * kTile;
constexpr int kMaxCams = 64;

// A camera prepared on the host in FP64.  The projection kernel reads the
// FP32 copies; the render kernels build per-tile ray frames from the FP64
// values so that pixel rays are exact to well below FP32 resolution.
struct DevCam {
  int model, shutter, W, H;
  int tiles_x, tiles_y, tile_base, pad0;
  long long pixel_base;
  // FP64
  double fx, fy, cx, cy;
  double k[4];
  double theta_lim, thetad_lim;
  double Q0[9];        // camera->world rotation at t = 0, row-major
  double c0[3], dc[3]; // camera centre at t = 0, and c1 - c0
  double axis[3];      // Q0^T Q1 = exp(angle [axis]x)  (camera-0 frame)
  double angle;
  double inv_hm1;      // 1/(H-1), 0 if H == 1
  // FP32
  float fxf, fyf, cxf, cyf;
  float kf[4];
  float theta_limf, inv_hm1f, anglef, pad1;
  float R0f[9];    // world->camera at t = 0
  float c0f[3];
  float deltaf[3]; // R0 (c1 - c0): centre motion in camera-0 coordinates
  float axisf[3];
  float dcf[3];    // c1 - c0 in world coordinates
};

// UT weights and spread, prepared on the host from (alpha, beta, kappa).
struct UTConst {
  float gamma;  // sqrt(3 + lambda)
  float wm0, wmi, wc0, wci;
};

struct Thresholds {
  float alpha_min, alpha_max, t_min, near_plane, k_sigma_max;
  float bg[3];
  int rs_iters;
  // Response of degree kdeg (2: the Gaussian).  With q = omega^2 log2(e) / 2
  // (the log2-unit exponent of the Gaussian), the degree-n exponent is
  // x = 2^(k_h log2 q + k_l) and sigma rho = 2^(lsig - x); the chain factor
  // of d alpha / d omega^2 relative to the Gaussian's is 2^((k_h - 1) log2 q + k_f).
  // k_lam and k_inv_n give the extent's cutoff (ln(sigma / alpha_min) / lambda)^(1/n).
  int kdeg;
  float k_h, k_inv_h, k_l, k_f, k_lam, k_inv_n;
};

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
const char* status_name(gut_status s);

#define GUT_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::gut::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),  \
                       __FILE__, __LINE__);                                    \
      return GUT_E_HIP;                                                        \
    }                                                                          \
  } while (0)

#define GUT_LAUNCH_CHECK()                                                     \
  do {                                                                         \
    hipError_t e_ = hipGetLastError();                                         \
    if (e_ != hipSuccess) {                                                    \
      ::gut::set_error("kernel launch failed: %s (%s:%d)",                     \
                       hipGetErrorString(e_), __FILE__, __LINE__);             \
      return GUT_E_HIP;                                                        \
    }                                                                          \
  } while (0)

// ---------------------------------------------------------------- host prep
gut_status make_devcam(const gut_camera& c, const gut_params& p, int tile_base,
                       long long pixel_base, DevCam* out);
gut_status check_params(const gut_params* p);
UTConst make_ut(const gut_params& p);
Thresholds make_thresholds(const gut_params& p);
gut_status check_scene(const gut_scene* s, bool need_sh);
gut_status prepare_cams(const gut_camera* cams, int n_cams, const gut_params& p,
                        DevCam* out, int64_t* total_tiles, int64_t* total_pixels);

gut_status fill_u32(uint32_t* p, int64_t m, uint32_t v, hipStream_t st);

// Internal stage launchers shared by the C entry points and the server.
gut_status project_launch(const gut_scene* scene, const DevCam* dc, int n_cams, const UTConst& ut,
                          const Thresholds& th, const gut_projected* out, bool write_record,
                          hipStream_t s);
gut_status render_batch_launch(const DevCam* d_cams, const DevCam* h_cams, int n_cams,
                               const Thresholds& th, int n, const uint32_t* ranges,
                               const uint32_t* order, const uint32_t* ids, const float* record,
                               const float* rgb, float* const* d_outs, unsigned* d_counters,
                               int* d_lists, int* h_lists, int n_blocks, hipStream_t s);
gut_status record_launch(const gut_scene* scene, float* record, hipStream_t s);
// Binning in two phases.  The count phase (bin_count_bytes(n, T) of
// workspace for n particles and T tiles over the cameras) queues the
// per-tile counts, the list starts, the render order and the pair total P,
// whose read-back bin_count_wait waits for; the sort phase (with
// bin_pair_bytes(cap) more) queues the pairs' scatter and the per-list
// sorts, which write nothing when P exceeds cap.
size_t bin_count_bytes(int64_t n, int64_t T);
size_t bin_pair_bytes(int64_t cap);
gut_status bin_count_launch(const gut_projected* proj, int n, const DevCam* dc, int n_cams, int64_t T,
                            bool cull, char* cws, uint32_t* tile_ranges, hipStream_t s);
// bin_count_wait also returns the number of lists of 4096 entries or more
// (n_long, when not null); the sort phase's parts can be queued separately:
// the scatter and the sorts of shorter lists, the long lists' sort, and the
// fallback sort of lists whose buckets came out too large, in that order.
gut_status bin_count_wait(uint64_t* P, uint32_t* n_long = nullptr);
constexpr int kSortLists = 1, kSortLong = 2, kSortFallback = 4, kSortAll = 7;
gut_status bin_sort_launch(const gut_projected* proj, int n, const DevCam* dc, int n_cams, int64_t T, bool cull,
                           char* cws, int64_t cap, char* pws, uint32_t* tile_ranges, uint32_t* sorted_ids,
                           hipStream_t s, int phases = kSortAll);

// ---------------------------------------------------------------- device math
__host__ __device__ inline float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ inline float dot3f(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline float3 cross3f(float3 a, float3 b) {
  return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
// The same with one rounding less per component (two instructions, not three).
__device__ inline float3 cross3f_fma(float3 a, float3 b) {
  return f3(fmaf(a.y, b.z, -a.z * b.y), fmaf(a.z, b.x, -a.x * b.z), fmaf(a.x, b.y, -a.y * b.x));
}

// FP64 3-vectors.  Products are summed with explicit fma: the code is built
// with contraction off (so that kernels sharing code round identically), and
// an explicit fma is both exact per call site and one instruction.
struct d3 { double x, y, z; };
__host__ __device__ inline d3 mk3(double x, double y, double z) { d3 r = {x, y, z}; return r; }
__host__ __device__ inline double dot(d3 a, d3 b) { return fma(a.x, b.x, fma(a.y, b.y, a.z * b.z)); }
__host__ __device__ inline d3 cross(d3 a, d3 b) {
  return mk3(fma(a.y, b.z, -a.z * b.y), fma(a.z, b.x, -a.x * b.z), fma(a.x, b.y, -a.y * b.x));
}
__host__ __device__ inline d3 add(d3 a, d3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
__host__ __device__ inline d3 sub(d3 a, d3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
__host__ __device__ inline d3 scl(d3 a, double s) { return mk3(a.x * s, a.y * s, a.z * s); }
// y + s x
__host__ __device__ inline d3 axpy(double s, d3 x, d3 y) {
  return mk3(fma(s, x.x, y.x), fma(s, x.y, y.y), fma(s, x.z, y.z));
}
__host__ __device__ inline d3 mv(const double* M, d3 v) {
  return mk3(fma(M[0], v.x, fma(M[1], v.y, M[2] * v.z)), fma(M[3], v.x, fma(M[4], v.y, M[5] * v.z)),
             fma(M[6], v.x, fma(M[7], v.y, M[8] * v.z)));
}

// Fisheye distortion polynomial theta_d(theta) (OpenCV fisheye model).
__host__ __device__ inline double thetad_poly(const double* k, double th) {
  double t2 = th * th;
  return th * fma(t2, fma(t2, fma(t2, fma(t2, k[3], k[2]), k[1]), k[0]), 1.0);
}
__host__ __device__ inline double thetad_deriv(const double* k, double th) {
  double t2 = th * th;
  return fma(t2, fma(t2, fma(t2, fma(t2, 9.0 * k[3], 7.0 * k[2]), 5.0 * k[1]), 3.0 * k[0]), 1.0);
}

// Rotate v by angle a about unit axis u (Rodrigues), FP64.
__host__ __device__ inline d3 rodrigues(d3 u, double a, d3 v) {
  double s = sin(a), c = cos(a);
  d3 uxv = cross(u, v);
  d3 uxuxv = cross(u, uxv);
  return add(v, add(scl(uxv, s), scl(uxuxv, 1.0 - c)));
}

// Camera-frame direction of image point (u, v) (a pixel centre or any point),
// FP64.  Fisheye: theta from theta_d by safeguarded Newton on [0, theta_lim];
// points beyond the image circle are clamped to it and reported invalid.
__device__ inline d3 unproject_dir(const DevCam& c, double u, double v, bool* valid) {
  double mx = (u - c.cx) / c.fx, my = (v - c.cy) / c.fy;
  if (c.model == GUT_PINHOLE) {
    *valid = true;
    return mk3(mx, my, 1.0);
  }
  double td = sqrt(mx * mx + my * my);
  *valid = td <= c.thetad_lim;
  double target = td < c.thetad_lim ? td : c.thetad_lim;
  double lo = 0.0, hi = c.theta_lim, th = target < hi ? target : hi;
  // beyond the circle the clamp is theta_lim itself (a double root of
  // theta_d(theta) - theta_d(theta_lim), where Newton would only crawl)
  if (!*valid) th = c.theta_lim;
  for (int it = 0; *valid && it < 60; it++) {  // Newton on [lo, hi], bisecting when it leaves
    double f = thetad_poly(c.k, th) - target;
    if (f == 0.0) break;
    if (f > 0) hi = th; else lo = th;
    double nt = th - f / thetad_deriv(c.k, th);
    if (!(nt >= lo && nt <= hi)) nt = 0.5 * (lo + hi);
    // 1e-14: far below what the FP32 tile coordinates hold, and above the
    // one-ulp oscillation a tighter test would never leave
    if (fabs(nt - th) <= 1e-14 * th || hi - lo <= 1e-14 * hi) { th = nt; break; }
    th = nt;
  }
  double st = sin(th), ct = cos(th);
  if (td > 0) return mk3(st * mx / td, st * my / td, ct);
  return mk3(0.0, 0.0, 1.0);
}

// World-space ray (origin, direction) of camera-frame direction dc exposed at
// time t: Q(t) = Q0 exp(t angle [axis]x), centre c0 + t (c1 - c0).
__device__ inline void ray_at(const DevCam& c, double t, d3 dc, d3* o, d3* d) {
  d3 r = dc;
  if (c.shutter == GUT_ROLLING_TOP_TO_BOTTOM && c.angle != 0.0)
    r = rodrigues(mk3(c.axis[0], c.axis[1], c.axis[2]), t * c.angle, dc);
  *d = mv(c.Q0, r);
  *o = mk3(c.c0[0] + t * c.dc[0], c.c0[1] + t * c.dc[1], c.c0[2] + t * c.dc[2]);
  if (c.shutter != GUT_ROLLING_TOP_TO_BOTTOM) *o = mk3(c.c0[0], c.c0[1], c.c0[2]);
}

__device__ inline double row_time(const DevCam& c, int row) {
  return c.shutter == GUT_ROLLING_TOP_TO_BOTTOM ? row * c.inv_hm1 : 0.0;
}

}  // namespace gut
