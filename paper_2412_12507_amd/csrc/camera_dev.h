// FP32 device functions shared by the projection and backward kernels:
// quaternion rotation, camera model g (pinhole / OpenCV fisheye), the
// rolling-shutter exposure-time solve, and the real SH basis with its
// gradient.  Forward and backward call the same code, so their discrete
// decisions agree bit for bit.
#pragma once
#include "common.h"

namespace gut {

// Real spherical-harmonic constants (orthonormal, Condon-Shortley phase).
constexpr float kSH0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float kSH1 = 0.48860251190291992f;   // sqrt(3/(4 pi))
constexpr float kSH2a = 1.0925484305920792f;   // (1/2) sqrt(15/pi)
constexpr float kSH2b = 0.31539156525252005f;  // (1/4) sqrt(5/pi)
constexpr float kSH2c = 0.54627421529603959f;  // (1/4) sqrt(15/pi)
constexpr float kSH3a = 0.59004358992664352f;  // (1/4) sqrt(35/(2 pi))
constexpr float kSH3b = 2.8906114426405538f;   // (1/2) sqrt(105/pi)
constexpr float kSH3c = 0.45704579946446572f;  // (1/4) sqrt(21/(2 pi))
constexpr float kSH3d = 0.37317633259011546f;  // (1/4) sqrt(7/pi)
constexpr float kSH3e = 1.4453057213202769f;   // (1/4) sqrt(105/pi)

// Basis values Y_k(d) for unit d, k = l^2 + l + m.
template <int DEG>
__device__ inline void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = kSH0;
  if (DEG >= 1) {
    Y[1] = -kSH1 * y;
    Y[2] = kSH1 * z;
    Y[3] = -kSH1 * x;
  }
  if (DEG >= 2) {
    float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kSH2a * x * y;
    Y[5] = -kSH2a * y * z;
    Y[6] = kSH2b * (2.0f * zz - xx - yy);
    Y[7] = -kSH2a * x * z;
    Y[8] = kSH2c * (xx - yy);
    if (DEG >= 3) {
      Y[9] = -kSH3a * y * (3.0f * xx - yy);
      Y[10] = kSH3b * x * y * z;
      Y[11] = -kSH3c * y * (4.0f * zz - xx - yy);
      Y[12] = kSH3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
      Y[13] = -kSH3c * x * (4.0f * zz - xx - yy);
      Y[14] = kSH3e * z * (xx - yy);
      Y[15] = -kSH3a * x * (xx - 3.0f * yy);
    }
  }
}

__device__ inline void quat_to_rot(float4 q, float R[9]) {
  float inv = rsqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
  float w = q.x * inv, x = q.y * inv, y = q.z * inv, z = q.w * inv;
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z);       R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y);       R[7] = 2.f * (y * z + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
}

// Camera-frame position at exposure time t of a point whose camera-0
// coordinates are y0 = R0 (x - c0):  x_c = exp(-t angle [axis]x) (y0 - t R0 dc).
__device__ inline float3 cam_at(const DevCam& c, float3 y0, float t) {
  if (c.shutter != GUT_ROLLING_TOP_TO_BOTTOM) return y0;
  float3 y = f3(y0.x - t * c.deltaf[0], y0.y - t * c.deltaf[1], y0.z - t * c.deltaf[2]);
  if (c.anglef == 0.0f) return y;
  float s, oc;  // sin x and 1 - cos x, x = t angle
  const float x = t * c.anglef;
  if (fabsf(c.anglef) <= 0.5f) {
    // |x| <= 0.5 (t in [0, 1]): Taylor series of sin x to x^9 and of
    // 1 - cos x to x^10, truncation below 2e-11; 1 - cos x from its own
    // series also avoids the cancellation of 1 - cos x in FP32
    const float x2 = x * x;
    s = x * fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, 1.0f / 362880.0f, -1.0f / 5040.0f), 1.0f / 120.0f),
                          -1.0f / 6.0f), 1.0f);
    oc = x2 * fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, 1.0f / 3628800.0f, -1.0f / 40320.0f), 1.0f / 720.0f),
                            -1.0f / 24.0f), 0.5f);
  } else {
    float co;
    sincosf(x, &s, &co);
    oc = 1.0f - co;
  }
  float3 k = f3(c.axisf[0], c.axisf[1], c.axisf[2]);
  float3 kxy = cross3f(k, y);
  float3 kkxy = cross3f(k, kxy);
  return f3(y.x - s * kxy.x + oc * kkxy.x, y.y - s * kxy.y + oc * kkxy.y,
            y.z - s * kxy.z + oc * kkxy.z);
}

// g: camera-frame point -> pixel coordinates; returns validity.
__device__ inline bool project_cam(const DevCam& c, float3 p, float near_plane, float2* v) {
  // hardware reciprocal and reciprocal square root (about 1 ulp): the pixel
  // coordinates they feed carry far larger errors from the FP32 inputs
  if (c.model == GUT_PINHOLE) {
    float iz = __builtin_amdgcn_rcpf(p.z);
    v->x = c.fxf * p.x * iz + c.cxf;
    v->y = c.fyf * p.y * iz + c.cyf;
    return p.z > near_plane;
  }
  float r2 = p.x * p.x + p.y * p.y;
  // on the axis (r2 far below any pixel offset, and clear of denormals) the
  // projection is the principal point
  float ir = r2 > 1e-30f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
  float r = r2 * ir;
  float th = atan2f(r, p.z);
  float t2 = th * th;
  float td = th * (1.0f + t2 * (c.kf[0] + t2 * (c.kf[1] + t2 * (c.kf[2] + t2 * c.kf[3]))));
  float sc = td * ir;
  v->x = c.fxf * sc * p.x + c.cxf;
  v->y = c.fyf * sc * p.y + c.cyf;
  // |p| > near, compared squared
  return th <= c.theta_limf && fmaf(p.z, p.z, r2) > near_plane * near_plane;
}

// Exposure time of a point and its final projection (rolling shutter: the
// row the point lands in fixes its time; iterate from t = 1/2).
__device__ inline float solve_project(const DevCam& c, float3 y0, const Thresholds& th,
                                      float2* v, bool* valid) {
  float t = 0.0f;
  if (c.shutter == GUT_ROLLING_TOP_TO_BOTTOM) {
    t = 0.5f;
    for (int it = 0; it < th.rs_iters; it++) {
      float2 vv;
      bool ok = project_cam(c, cam_at(c, y0, t), th.near_plane, &vv);
      if (ok) t = fminf(fmaxf((vv.y - 0.5f) * c.inv_hm1f, 0.0f), 1.0f);
    }
  }
  *valid = project_cam(c, cam_at(c, y0, t), th.near_plane, v);
  return t;
}


// Cartesian gradient of each basis polynomial (tangential part is what
// matters: callers project onto the plane orthogonal to d).
template <int DEG>
__device__ inline void sh_basis_grad(float x, float y, float z, float3* g) {
  g[0] = f3(0.f, 0.f, 0.f);
  if (DEG >= 1) {
    g[1] = f3(0.f, -kSH1, 0.f);
    g[2] = f3(0.f, 0.f, kSH1);
    g[3] = f3(-kSH1, 0.f, 0.f);
  }
  if (DEG >= 2) {
    g[4] = f3(kSH2a * y, kSH2a * x, 0.f);
    g[5] = f3(0.f, -kSH2a * z, -kSH2a * y);
    g[6] = f3(-2.f * kSH2b * x, -2.f * kSH2b * y, 4.f * kSH2b * z);
    g[7] = f3(-kSH2a * z, 0.f, -kSH2a * x);
    g[8] = f3(2.f * kSH2c * x, -2.f * kSH2c * y, 0.f);
    if (DEG >= 3) {
      float xx = x * x, yy = y * y, zz = z * z;
      g[9] = f3(-6.f * kSH3a * x * y, -3.f * kSH3a * (xx - yy), 0.f);
      g[10] = f3(kSH3b * y * z, kSH3b * x * z, kSH3b * x * y);
      g[11] = f3(2.f * kSH3c * x * y, -kSH3c * (4.f * zz - xx - 3.f * yy), -8.f * kSH3c * y * z);
      g[12] = f3(-6.f * kSH3d * x * z, -6.f * kSH3d * y * z, kSH3d * (6.f * zz - 3.f * xx - 3.f * yy));
      g[13] = f3(-kSH3c * (4.f * zz - 3.f * xx - yy), 2.f * kSH3c * x * y, -8.f * kSH3c * x * z);
      g[14] = f3(2.f * kSH3e * x * z, -2.f * kSH3e * y * z, kSH3e * (xx - yy));
      g[15] = f3(-3.f * kSH3a * (xx - yy), 6.f * kSH3a * x * y, 0.f);
    }
  }
}

// Camera-0 coordinates y0 = R0 (x - c0) of a world point.
__device__ inline float3 cam0_coords(const DevCam& cam, float3 x) {
  float3 rel = f3(x.x - cam.c0f[0], x.y - cam.c0f[1], x.z - cam.c0f[2]);
  const float* R0 = cam.R0f;
  return f3(R0[0] * rel.x + R0[1] * rel.y + R0[2] * rel.z,
            R0[3] * rel.x + R0[4] * rel.y + R0[5] * rel.z,
            R0[6] * rel.x + R0[7] * rel.y + R0[8] * rel.z);
}

// Camera centre at exposure time t (FP32).
__device__ inline float3 centre_at(const DevCam& cam, float t) {
  if (cam.shutter != GUT_ROLLING_TOP_TO_BOTTOM) return f3(cam.c0f[0], cam.c0f[1], cam.c0f[2]);
  return f3(cam.c0f[0] + t * cam.dcf[0], cam.c0f[1] + t * cam.dcf[1], cam.c0f[2] + t * cam.dcf[2]);
}

}  // namespace gut
