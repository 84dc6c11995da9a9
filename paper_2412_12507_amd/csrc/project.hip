// K1 -- per (camera, particle) projection with the Unscented Transform.
//
// Alg. 1 with Alg. 2 as Estimate2DGaussian: seven sigma points read off the
// factorisation Sigma = R S S^T R^T (Eq. 6), each projected exactly through
// the camera model g (pinhole or OpenCV fisheye; under a rolling shutter each
// point first finds the exposure time of the row it lands in), then the
// weighted mean and covariance (Eq. 7-10), an opacity-aware extent and the
// tile rectangle.  Also the sort depth and the view-dependent SH colour.
//
// One thread per particle for up to four cameras per launch: the SoA
// inputs are read once (coalesced across the wave) whatever the number of
// cameras; outputs are 28 B per (camera, particle), 24 B more with the mean
// and the extent ellipse that tile culling reads, plus a 64 B render record
// per particle written by the first launch.
#include "camera_dev.h"

namespace gut {

// Render record of one particle: mu, sigma and the rows of M = S^-1 R^T,
// formed in FP64 from the FP32 parameters and rounded once, so that the
// compositing kernels see M to half an ulp.
__device__ inline void write_record(float3 mu, float3 s, float4 q, float sig, float4* rec) {
  const double qw = q.x, qx = q.y, qy = q.z, qz = q.w;
  const double iq = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  const double w = qw * iq, x = qx * iq, y = qy * iq, z = qz * iq;
  const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                       2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                       2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
  const double is0 = 1.0 / s.x, is1 = 1.0 / s.y, is2 = 1.0 / s.z;
  rec[0] = make_float4(mu.x, mu.y, mu.z, sig);
  rec[1] = make_float4((float)(R[0] * is0), (float)(R[3] * is0), (float)(R[6] * is0), 0.0f);
  rec[2] = make_float4((float)(R[1] * is1), (float)(R[4] * is1), (float)(R[7] * is1), 0.0f);
  rec[3] = make_float4((float)(R[2] * is2), (float)(R[5] * is2), (float)(R[8] * is2), 0.0f);
}

// Cameras of one projection launch, passed by value (their FP32 fields are
// read from the kernel arguments with scalar loads).
constexpr int kProjCams = 4;
struct ProjCams {
  DevCam cam[kProjCams];
  int idx[kProjCams];  // the cameras' indices in the call (entry e = idx * n + i)
  int n;
};

// One thread per particle and every camera of the launch: the particle's
// parameters and SH coefficients are read once and stay in registers while
// the camera loop projects it (S9's one launch per stage).
template <int DEG>
__global__ void __launch_bounds__(256) project_kernel(
    int n, ProjCams pc, UTConst ut, Thresholds th, const float* __restrict__ means,
    const float* __restrict__ scales, const float* __restrict__ quats,
    const float* __restrict__ opac, const float* __restrict__ sh, int16_t* __restrict__ rect,
    uint32_t* __restrict__ tiles, float* __restrict__ depth, float* __restrict__ rgb,
    float* __restrict__ record, float* __restrict__ mean2d, float* __restrict__ cov2d,
    float* __restrict__ extent) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;

  float3 mu = f3(means[3 * i], means[3 * i + 1], means[3 * i + 2]);
  float3 s = f3(scales[3 * i], scales[3 * i + 1], scales[3 * i + 2]);
  float4 q = reinterpret_cast<const float4*>(quats)[i];
  float sig = opac[i];
  float R[9];
  quat_to_rot(q, R);
  if (record)  // render record (written by one launch per scene)
    write_record(mu, s, q, sig, reinterpret_cast<float4*>(record) + 4 * (long long)i);
  float b[3 * K];
  const bool live = sig >= th.alpha_min;
  if (live) {
    const float* src = sh + (long long)i * K * 3;
#pragma unroll
    for (int k = 0; k < 3 * K; k++) b[k] = src[k];
  }
  // the extent's cutoff: the distance k where sigma rho(k^2) = alpha_min (at
  // most k_sigma_max): sqrt(2 ln(sigma / alpha_min)) for the Gaussian, else
  // (ln(sigma / alpha_min) / lambda)^(1/n)
  float ks = 0.0f;
  if (live) {
    const float lnr = logf(sig / th.alpha_min);
    ks = th.kdeg == 2 ? sqrtf(2.0f * lnr) : powf(lnr / th.k_lam, th.k_inv_n);
    ks = fminf(th.k_sigma_max, ks);
  }

#pragma unroll 1
  for (int ci = 0; ci < pc.n; ci++) {
    const DevCam& cam = pc.cam[ci];
    const long long e = (long long)pc.idx[ci] * n + i;
    uint32_t ntiles = 0;
    short4 rc = make_short4(0, 0, 0, 0);
    float dep = 0.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    float2 vmean = make_float2(0.0f, 0.0f);
    float cxx = 0.0f, cxy = 0.0f, cyy = 0.0f;
    if (live) {
      // camera-0 coordinates of the mean, and of the three scaled axes
      const float* R0 = cam.R0f;
      float3 y0 = cam0_coords(cam, mu);
      float2 v[7];
      bool ok_all = true, ok;
      float t0 = solve_project(cam, y0, th, &v[0], &ok);
      ok_all &= ok;
      float sc3[3] = {s.x, s.y, s.z};
#pragma unroll
      for (int k = 0; k < 3; k++) {
        // column k of R S, scaled by sqrt(3 + lambda), in camera-0 coordinates
        float g = ut.gamma * sc3[k];
        float3 col = f3(R[k] * g, R[3 + k] * g, R[6 + k] * g);
        float3 dy = f3(R0[0] * col.x + R0[1] * col.y + R0[2] * col.z,
                       R0[3] * col.x + R0[4] * col.y + R0[5] * col.z,
                       R0[6] * col.x + R0[7] * col.y + R0[8] * col.z);
        solve_project(cam, f3(y0.x + dy.x, y0.y + dy.y, y0.z + dy.z), th, &v[1 + k], &ok);
        ok_all &= ok;
        solve_project(cam, f3(y0.x - dy.x, y0.y - dy.y, y0.z - dy.z), th, &v[4 + k], &ok);
        ok_all &= ok;
      }
      // Eq. 9-10
      float mx = ut.wm0 * v[0].x, my = ut.wm0 * v[0].y;
#pragma unroll
      for (int k = 1; k < 7; k++) { mx += ut.wmi * v[k].x; my += ut.wmi * v[k].y; }
#pragma unroll
      for (int k = 0; k < 7; k++) {
        float w = k == 0 ? ut.wc0 : ut.wci;
        float dx = v[k].x - mx, dyy = v[k].y - my;
        cxx += w * dx * dx;
        cxy += w * dx * dyy;
        cyy += w * dyy * dyy;
      }
      vmean = make_float2(mx, my);
      if (ok_all) {
        // Extent: the box of the ks-sigma ellipse
        float hx = ks * sqrtf(fmaxf(cxx, 0.0f)), hy = ks * sqrtf(fmaxf(cyy, 0.0f));
        const float inv_t = 1.0f / kTile;
        int x0 = max((int)floorf((mx - hx) * inv_t), 0);
        int y0i = max((int)floorf((my - hy) * inv_t), 0);
        int x1 = min((int)floorf((mx + hx) * inv_t), cam.tiles_x - 1);
        int y1 = min((int)floorf((my + hy) * inv_t), cam.tiles_y - 1);
        if (x0 <= x1 && y0i <= y1) {
          ntiles = (uint32_t)((x1 - x0 + 1) * (y1 - y0i + 1));
          rc = make_short4((short)x0, (short)y0i, (short)x1, (short)y1);
        }
      }
      if (ntiles) {
        // depth and colour from the camera centre at the mean point's exposure time
        float3 ctr = centre_at(cam, t0);
        float3 dv = f3(mu.x - ctr.x, mu.y - ctr.y, mu.z - ctr.z);
        dep = sqrtf(dot3f(dv, dv));
        float id = 1.0f / dep;
        float Y[K];
        sh_basis<DEG>(dv.x * id, dv.y * id, dv.z * id, Y);
        cr = 0.5f; cg = 0.5f; cb = 0.5f;
#pragma unroll
        for (int k = 0; k < K; k++) {
          cr += b[3 * k] * Y[k];
          cg += b[3 * k + 1] * Y[k];
          cb += b[3 * k + 2] * Y[k];
        }
        cr = fmaxf(cr, 0.0f); cg = fmaxf(cg, 0.0f); cb = fmaxf(cb, 0.0f);
      }
    }
    reinterpret_cast<short4*>(rect)[e] = rc;
    tiles[e] = ntiles;
    depth[e] = dep;
    rgb[3 * e] = cr;
    rgb[3 * e + 1] = cg;
    rgb[3 * e + 2] = cb;
    if (mean2d) reinterpret_cast<float2*>(mean2d)[e] = vmean;
    if (cov2d) { cov2d[3 * e] = cxx; cov2d[3 * e + 1] = cxy; cov2d[3 * e + 2] = cyy; }
    if (extent) {
      // the tile-culling ellipse (v - m)^T A^-1 (v - m) <= 1, A = ks^2 Sigma', of a visible entry
      const float k2 = ntiles ? ks * ks : 0.0f;
      reinterpret_cast<float4*>(extent)[e] = make_float4(k2 * cxx, k2 * cxy, k2 * cyy, ntiles ? ks : 0.0f);
    }
  }
}

// Render records only (mu, sigma, M = S^-1 R^T), for a resident scene.
__global__ void record_kernel(int n, const float* __restrict__ means,
                              const float* __restrict__ scales, const float* __restrict__ quats,
                              const float* __restrict__ opac, float* __restrict__ record) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  write_record(f3(means[3 * i], means[3 * i + 1], means[3 * i + 2]),
               f3(scales[3 * i], scales[3 * i + 1], scales[3 * i + 2]),
               reinterpret_cast<const float4*>(quats)[i], opac[i],
               reinterpret_cast<float4*>(record) + 4 * (long long)i);
}

gut_status record_launch(const gut_scene* scene, float* record, hipStream_t s) {
  const int n = (int)scene->n;
  if (n == 0) return GUT_OK;
  record_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, scene->means, scene->scales, scene->quats,
                                                scene->opacities, record);
  GUT_LAUNCH_CHECK();
  return GUT_OK;
}

gut_status project_launch(const gut_scene* scene, const DevCam* dc, int n_cams, const UTConst& ut,
                          const Thresholds& th, const gut_projected* out, bool write_record,
                          hipStream_t s) {
  const int n = (int)scene->n;
  if (n == 0) return GUT_OK;
  dim3 grid((n + 255) / 256), block(256);
  for (int c0 = 0; c0 < n_cams; c0 += kProjCams) {
    ProjCams pc;
    pc.n = n_cams - c0 < kProjCams ? n_cams - c0 : kProjCams;
    for (int j = 0; j < pc.n; j++) {
      pc.cam[j] = dc[c0 + j];
      pc.idx[j] = c0 + j;
    }
    float* rec = (write_record && c0 == 0) ? out->record : nullptr;
#define GUT_PROJ(D)                                                                            \
  project_kernel<D><<<grid, block, 0, s>>>(n, pc, ut, th, scene->means, scene->scales,         \
                                           scene->quats, scene->opacities, scene->sh, out->rect, \
                                           out->tiles, out->depth, out->rgb, rec, out->mean2d,   \
                                           out->cov2d, out->extent)
    switch (scene->sh_degree) {
      case 0: GUT_PROJ(0); break;
      case 1: GUT_PROJ(1); break;
      case 2: GUT_PROJ(2); break;
      default: GUT_PROJ(3); break;
    }
#undef GUT_PROJ
    GUT_LAUNCH_CHECK();
  }
  return GUT_OK;
}

}  // namespace gut

using namespace gut;

extern "C" gut_status gut_project(const gut_scene* scene, const gut_camera* cams, int32_t n_cams,
                                  const gut_params* p, const gut_projected* out, void* stream) {
  gut_status st = check_params(p);
  if (st != GUT_OK) return st;
  if ((st = check_scene(scene, true)) != GUT_OK) return st;
  if (scene->n == 0) {  // nothing to project; only the cameras are checked
    DevCam tmp[kMaxCams];
    return prepare_cams(cams, n_cams, *p, tmp, nullptr, nullptr);
  }
  if (!out || !out->rect || !out->tiles || !out->depth || !out->rgb || !out->record) {
    set_error("projected outputs rect, tiles, depth, rgb and record are required");
    return GUT_E_INVALID;
  }
  if (((uintptr_t)scene->quats & 15) || ((uintptr_t)out->record & 15) ||
      ((uintptr_t)out->rect & 7) || ((uintptr_t)out->mean2d & 7)) {
    set_error("quats and record must be 16-byte, rect and mean2d 8-byte aligned");
    return GUT_E_INVALID;
  }
  DevCam dc[kMaxCams];
  if ((st = prepare_cams(cams, n_cams, *p, dc, nullptr, nullptr)) != GUT_OK) return st;
  if (scene->n * (int64_t)n_cams >= (int64_t(1) << 31)) {
    set_error("n * n_cams must be below 2^31");
    return GUT_E_INVALID;
  }
  return project_launch(scene, dc, n_cams, make_ut(*p), make_thresholds(*p), out, true,
                        (hipStream_t)stream);
}
