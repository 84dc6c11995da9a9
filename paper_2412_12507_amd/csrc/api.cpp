// Host-side plumbing of libgut: argument checks, camera preparation in FP64,
// error reporting.  The per-stage entry points live beside their kernels.
#include <cstdarg>
#include <cstring>

#include "common.h"

namespace gut {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

const char* status_name(gut_status s) {
  switch (s) {
    case GUT_OK: return "GUT_OK";
    case GUT_E_INVALID: return "GUT_E_INVALID";
    case GUT_E_CAPACITY: return "GUT_E_CAPACITY";
    case GUT_E_HIP: return "GUT_E_HIP";
    case GUT_E_ADMISSION: return "GUT_E_ADMISSION";
    case GUT_E_UNSUPPORTED: return "GUT_E_UNSUPPORTED";
    case GUT_E_NOT_FOUND: return "GUT_E_NOT_FOUND";
  }
  return "GUT_E_UNKNOWN";
}

static bool finite_all(const double* v, int n) {
  for (int i = 0; i < n; i++)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// Fisheye validity limit: first angle in (0, pi/2] where d theta_d/d theta
// reaches zero (scan, then bisection), else pi/2.
static double host_theta_lim(const double* k) {
  const int steps = 4096;
  const double half_pi = 1.5707963267948966;
  double prev = 0.0;
  for (int i = 1; i <= steps; i++) {
    double th = half_pi * i / steps;
    if (thetad_deriv(k, th) <= 0.0) {
      double lo = prev, hi = th;
      for (int it = 0; it < 200; it++) {
        double mid = 0.5 * (lo + hi);
        if (thetad_deriv(k, mid) > 0.0) lo = mid; else hi = mid;
      }
      return lo;
    }
    prev = th;
  }
  return half_pi;
}

// Axis and angle of a rotation matrix (row-major), robust near 0 and pi.
static void rot_log(const double* R, double axis[3], double* angle) {
  double v[3] = {0.5 * (R[7] - R[5]), 0.5 * (R[2] - R[6]), 0.5 * (R[3] - R[1])};
  double s = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
  double a = std::atan2(s, c);
  *angle = a;
  if (a < 1e-300) { axis[0] = 0; axis[1] = 0; axis[2] = 1; *angle = 0.0; return; }
  if (s > 1e-6) {
    for (int i = 0; i < 3; i++) axis[i] = v[i] / s;
    return;
  }
  // angle close to pi: R + R^T = 2 cos(a) I + 2 (1 - cos(a)) u u^T
  double B[9];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) B[3 * i + j] = 0.5 * (R[3 * i + j] + R[3 * j + i]) - (i == j ? c : 0.0);
  int m = 0;
  for (int i = 1; i < 3; i++)
    if (B[4 * i] > B[4 * m]) m = i;
  double norm = std::sqrt(B[4 * m] > 0 ? B[4 * m] : 0.0);
  for (int i = 0; i < 3; i++) axis[i] = B[3 * m + i] / (norm > 0 ? norm : 1.0);
  double an = std::sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
  for (int i = 0; i < 3; i++) axis[i] /= an;
  if (axis[0] * v[0] + axis[1] * v[1] + axis[2] * v[2] < 0)
    for (int i = 0; i < 3; i++) axis[i] = -axis[i];
}

static bool orthonormal(const double* R) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double d = R[3 * i] * R[3 * j] + R[3 * i + 1] * R[3 * j + 1] + R[3 * i + 2] * R[3 * j + 2];
      if (std::fabs(d - (i == j ? 1.0 : 0.0)) > 1e-6) return false;
    }
  return true;
}

gut_status make_devcam(const gut_camera& c, const gut_params& p, int tile_base,
                       long long pixel_base, DevCam* o) {
  std::memset(o, 0, sizeof(*o));
  if (c.model != GUT_PINHOLE && c.model != GUT_FISHEYE_OPENCV) {
    set_error("camera model %d unknown", c.model);
    return GUT_E_INVALID;
  }
  if (c.shutter != GUT_GLOBAL_SHUTTER && c.shutter != GUT_ROLLING_TOP_TO_BOTTOM) {
    set_error("camera shutter %d unknown", c.shutter);
    return GUT_E_INVALID;
  }
  if (c.width <= 0 || c.height <= 0 || c.width > 65536 || c.height > 65536) {
    set_error("camera size %dx%d out of range", c.width, c.height);
    return GUT_E_INVALID;
  }
  double intr[8] = {c.fx, c.fy, c.cx, c.cy, c.k[0], c.k[1], c.k[2], c.k[3]};
  if (!finite_all(intr, 8) || !(c.fx > 0) || !(c.fy > 0)) {
    set_error("camera intrinsics must be finite with fx, fy > 0");
    return GUT_E_INVALID;
  }
  if (!finite_all(c.R0, 9) || !finite_all(c.t0, 3) || !orthonormal(c.R0)) {
    set_error("camera pose 0 must be finite with an orthonormal rotation");
    return GUT_E_INVALID;
  }
  const bool rolling = c.shutter == GUT_ROLLING_TOP_TO_BOTTOM;
  if (rolling && (!finite_all(c.R1, 9) || !finite_all(c.t1, 3) || !orthonormal(c.R1))) {
    set_error("camera pose 1 must be finite with an orthonormal rotation");
    return GUT_E_INVALID;
  }
  const int ts = p.tile;
  o->model = c.model;
  // a rolling shutter whose two poses are identical images exactly as a
  // global shutter: use the global-shutter kernels for it
  const bool still = rolling && std::memcmp(c.R0, c.R1, sizeof(c.R0)) == 0 &&
                     std::memcmp(c.t0, c.t1, sizeof(c.t0)) == 0;
  o->shutter = still ? GUT_GLOBAL_SHUTTER : c.shutter;
  o->W = c.width;
  o->H = c.height;
  o->tiles_x = (c.width + ts - 1) / ts;
  o->tiles_y = (c.height + ts - 1) / ts;
  o->tile_base = tile_base;
  o->pixel_base = pixel_base;
  o->fx = c.fx; o->fy = c.fy; o->cx = c.cx; o->cy = c.cy;
  for (int i = 0; i < 4; i++) o->k[i] = c.k[i];
  if (c.model == GUT_FISHEYE_OPENCV) {
    o->theta_lim = host_theta_lim(c.k);
    if (!(o->theta_lim > 1e-6)) {
      set_error("fisheye distortion leaves no valid field of view");
      return GUT_E_INVALID;
    }
  } else {
    o->theta_lim = 1.5707963267948966;
  }
  o->thetad_lim = thetad_poly(c.k, o->theta_lim);
  for (int r = 0; r < 3; r++)
    for (int k = 0; k < 3; k++) o->Q0[3 * r + k] = c.R0[3 * k + r];
  double c0[3], c1[3];
  for (int i = 0; i < 3; i++) {
    c0[i] = -(c.R0[i] * c.t0[0] + c.R0[3 + i] * c.t0[1] + c.R0[6 + i] * c.t0[2]);
    c1[i] = rolling ? -(c.R1[i] * c.t1[0] + c.R1[3 + i] * c.t1[1] + c.R1[6 + i] * c.t1[2]) : c0[i];
  }
  for (int i = 0; i < 3; i++) { o->c0[i] = c0[i]; o->dc[i] = c1[i] - c0[i]; }
  o->axis[0] = 0; o->axis[1] = 0; o->axis[2] = 1; o->angle = 0.0;
  if (rolling && std::memcmp(c.R0, c.R1, sizeof(c.R0)) != 0) {
    double Rrel[9];  // Q0^T Q1 = R0 R1^T
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++)
        Rrel[3 * i + j] = c.R0[3 * i] * c.R1[3 * j] + c.R0[3 * i + 1] * c.R1[3 * j + 1] +
                          c.R0[3 * i + 2] * c.R1[3 * j + 2];
    rot_log(Rrel, o->axis, &o->angle);
  }
  o->inv_hm1 = c.height > 1 ? 1.0 / (c.height - 1) : 0.0;
  o->fxf = (float)c.fx; o->fyf = (float)c.fy; o->cxf = (float)c.cx; o->cyf = (float)c.cy;
  for (int i = 0; i < 4; i++) o->kf[i] = (float)c.k[i];
  o->theta_limf = (float)o->theta_lim;
  o->inv_hm1f = (float)o->inv_hm1;
  o->anglef = (float)o->angle;
  for (int i = 0; i < 9; i++) o->R0f[i] = (float)c.R0[i];
  for (int i = 0; i < 3; i++) {
    o->c0f[i] = (float)c0[i];
    o->deltaf[i] = (float)(c.R0[3 * i] * o->dc[0] + c.R0[3 * i + 1] * o->dc[1] + c.R0[3 * i + 2] * o->dc[2]);
    o->axisf[i] = (float)o->axis[i];
    o->dcf[i] = (float)o->dc[i];
  }
  return GUT_OK;
}

gut_status check_params(const gut_params* p) {
  if (!p) { set_error("params is NULL"); return GUT_E_INVALID; }
  double a = p->ut_alpha, kap = p->ut_kappa;
  if (!std::isfinite(a) || !std::isfinite(p->ut_beta) || !std::isfinite(kap) ||
      !(a * a * (3.0 + kap) > 0.0)) {
    set_error("UT parameters must be finite with alpha^2 (3 + kappa) > 0");
    return GUT_E_INVALID;
  }
  if (!(p->alpha_min > 0) || !(p->alpha_max > p->alpha_min) || !(p->alpha_max <= 1.0f) ||
      !(p->t_min > 0) || !(p->t_min < 1) || !(p->near_plane >= 0) || !(p->k_sigma_max > 0) ||
      !std::isfinite(p->bg[0] + p->bg[1] + p->bg[2])) {
    set_error("thresholds out of range");
    return GUT_E_INVALID;
  }
  if (p->tile != kTile) {
    set_error("tile size %d unsupported (libgut renders 16x16 tiles)", p->tile);
    return GUT_E_UNSUPPORTED;
  }
  if (p->rs_iters < 0 || p->rs_iters > 64) {
    set_error("rs_iters must be in [0, 64]");
    return GUT_E_INVALID;
  }
  if (p->kernel_degree < 2 || p->kernel_degree > 8) {
    set_error("kernel_degree must be in [2, 8]");
    return GUT_E_INVALID;
  }
  if (p->kbuffer < 0 || p->kbuffer > 16) {
    set_error("kbuffer must be in [0, 16]");
    return GUT_E_INVALID;
  }
  if (p->tile_cull != 0 && p->tile_cull != 1) {
    set_error("tile_cull must be 0 or 1");
    return GUT_E_INVALID;
  }
  return GUT_OK;
}

UTConst make_ut(const gut_params& p) {
  double a = p.ut_alpha, b = p.ut_beta, kap = p.ut_kappa;
  double lam = a * a * (3.0 + kap) - 3.0;  // Alg. 2: lambda = alpha^2 (3 + kappa) - 3
  UTConst u;
  u.gamma = (float)std::sqrt(3.0 + lam);
  u.wm0 = (float)(lam / (3.0 + lam));
  u.wmi = (float)(1.0 / (2.0 * (3.0 + lam)));
  u.wc0 = (float)(lam / (3.0 + lam) + (1.0 - a * a + b));
  u.wci = u.wmi;
  return u;
}

Thresholds make_thresholds(const gut_params& p) {
  Thresholds t;
  t.alpha_min = p.alpha_min;
  t.alpha_max = p.alpha_max;
  t.t_min = p.t_min;
  t.near_plane = p.near_plane;
  t.k_sigma_max = p.k_sigma_max;
  for (int i = 0; i < 3; i++) t.bg[i] = p.bg[i];
  t.rs_iters = p.rs_iters;
  // generalized Gaussian of degree n (Supp. A): rho = exp(-lambda (omega^2)^(n/2))
  // with lambda = 3^(2-n) / 2, the response of the Gaussian at distance 3
  const int n = p.kernel_degree;
  const double h = 0.5 * n, lam = 0.5 * std::pow(3.0, 2.0 - n);
  const double log2e = 1.4426950408889634, l2ln2 = std::log2(2.0 * 0.6931471805599453);
  t.kdeg = n;
  t.k_h = (float)h;
  t.k_inv_h = (float)(1.0 / h);
  t.k_l = (float)(std::log2(lam * log2e) + h * l2ln2);
  t.k_f = (float)(std::log2(2.0 * lam * h) + (h - 1.0) * l2ln2);
  t.k_lam = (float)lam;
  t.k_inv_n = (float)(1.0 / n);
  return t;
}

gut_status check_scene(const gut_scene* s, bool need_sh) {
  if (!s) { set_error("scene is NULL"); return GUT_E_INVALID; }
  if (s->n < 0 || s->n >= (int64_t(1) << 31)) { set_error("scene size %lld out of range", (long long)s->n); return GUT_E_INVALID; }
  if (s->sh_degree < 0 || s->sh_degree > 3) { set_error("sh_degree %d unsupported", s->sh_degree); return GUT_E_INVALID; }
  if (s->n > 0 && (!s->means || !s->scales || !s->quats || !s->opacities || (need_sh && !s->sh))) {
    set_error("scene arrays must not be NULL");
    return GUT_E_INVALID;
  }
  return GUT_OK;
}

gut_status prepare_cams(const gut_camera* cams, int n_cams, const gut_params& p, DevCam* out,
                        int64_t* total_tiles, int64_t* total_pixels) {
  if (!cams || n_cams <= 0 || n_cams > kMaxCams) {
    set_error("n_cams must be in [1, %d] with a camera array", kMaxCams);
    return GUT_E_INVALID;
  }
  int64_t tiles = 0, pix = 0;
  for (int c = 0; c < n_cams; c++) {
    gut_status st = make_devcam(cams[c], p, (int)tiles, (long long)pix, &out[c]);
    if (st != GUT_OK) return st;
    tiles += (int64_t)out[c].tiles_x * out[c].tiles_y;
    pix += (int64_t)cams[c].width * cams[c].height;
    if (tiles >= (int64_t(1) << 30)) { set_error("too many tiles"); return GUT_E_INVALID; }
  }
  if (total_tiles) *total_tiles = tiles;
  if (total_pixels) *total_pixels = pix;
  return GUT_OK;
}

}  // namespace gut

using namespace gut;

extern "C" {

void gut_default_params(gut_params* p) {
  if (!p) return;
  p->ut_alpha = 1.0f;
  p->ut_beta = 2.0f;
  p->ut_kappa = 0.0f;
  p->alpha_min = 1.0f / 255.0f;
  p->alpha_max = 0.99f;
  p->t_min = 1e-4f;
  p->near_plane = 0.2f;
  p->k_sigma_max = 3.0f;
  p->tile = kTile;
  p->rs_iters = 3;
  p->bg[0] = p->bg[1] = p->bg[2] = 0.0f;
  p->kernel_degree = 2;
  p->kbuffer = 0;
  p->tile_cull = 1;
}

int64_t gut_num_tiles(const gut_camera* cams, int32_t n_cams, const gut_params* p) {
  if (check_params(p) != GUT_OK || !cams || n_cams <= 0) return -1;
  int64_t t = 0;
  for (int c = 0; c < n_cams; c++) {
    if (cams[c].width <= 0 || cams[c].height <= 0) return -1;
    t += (int64_t)((cams[c].width + p->tile - 1) / p->tile) * ((cams[c].height + p->tile - 1) / p->tile);
  }
  return t;
}

int64_t gut_num_pixels(const gut_camera* cams, int32_t n_cams) {
  if (!cams || n_cams <= 0) return -1;
  int64_t t = 0;
  for (int c = 0; c < n_cams; c++) {
    if (cams[c].width <= 0 || cams[c].height <= 0) return -1;
    t += (int64_t)cams[c].width * cams[c].height;
  }
  return t;
}

const char* gut_status_string(gut_status st) { return status_name(st); }
const char* gut_last_error(void) { return g_err; }

}  // extern "C"
