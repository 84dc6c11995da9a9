/*
 * oracle.c -- plain FP64 CPU reference of the 3DGUT rasterizer hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for a reader checking it
 * against the paper by eye: straightforward loops, double precision, one
 * function per step of the method, no code shared with the GPU path.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------- */
/* Small vector helpers                                                       */
/* ------------------------------------------------------------------------- */

static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static void matvec(const double M[9], const double v[3], double out[3]) {
  for (int r = 0; r < 3; r++) out[r] = M[3 * r] * v[0] + M[3 * r + 1] * v[1] + M[3 * r + 2] * v[2];
}
static void matTvec(const double M[9], const double v[3], double out[3]) {
  for (int c = 0; c < 3; c++) out[c] = M[c] * v[0] + M[3 + c] * v[1] + M[6 + c] * v[2];
}
static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* ------------------------------------------------------------------------- */
/* Rotation from a quaternion (w, x, y, z); Sec. 3 stores R as a quaternion.  */
/* ------------------------------------------------------------------------- */

void ora_quat_to_rot(const double q_in[4], double R[9]) {
  double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
  double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void rot_to_quat(const double m[9], double q[4]) {
  double tr = m[0] + m[4] + m[8], S;
  if (tr > 0) {
    S = sqrt(tr + 1.0) * 2;
    q[0] = 0.25 * S; q[1] = (m[7] - m[5]) / S; q[2] = (m[2] - m[6]) / S; q[3] = (m[3] - m[1]) / S;
  } else if (m[0] > m[4] && m[0] > m[8]) {
    S = sqrt(1.0 + m[0] - m[4] - m[8]) * 2;
    q[0] = (m[7] - m[5]) / S; q[1] = 0.25 * S; q[2] = (m[1] + m[3]) / S; q[3] = (m[2] + m[6]) / S;
  } else if (m[4] > m[8]) {
    S = sqrt(1.0 + m[4] - m[0] - m[8]) * 2;
    q[0] = (m[2] - m[6]) / S; q[1] = (m[1] + m[3]) / S; q[2] = 0.25 * S; q[3] = (m[5] + m[7]) / S;
  } else {
    S = sqrt(1.0 + m[8] - m[0] - m[4]) * 2;
    q[0] = (m[3] - m[1]) / S; q[1] = (m[2] + m[6]) / S; q[2] = (m[5] + m[7]) / S; q[3] = 0.25 * S;
  }
}

/* ------------------------------------------------------------------------- */
/* Camera: poses, projection g(x), pixel rays                                 */
/* ------------------------------------------------------------------------- */

/* Per-camera constants, computed once per call: camera centres, the two
 * camera-to-world rotations as quaternions and the fisheye validity limit. */
typedef struct {
  const ora_camera* c;
  double c0[3], c1[3], q0[4], q1[4];
  double theta_lim, thetad_lim;
} camctx;

static double fisheye_thetad(const double k[4], double th) {
  double t2 = th * th;
  return th * (1 + t2 * (k[0] + t2 * (k[1] + t2 * (k[2] + t2 * k[3]))));
}
static double fisheye_dthetad(const double k[4], double th) {
  double t2 = th * th;
  return 1 + t2 * (3 * k[0] + t2 * (5 * k[1] + t2 * (7 * k[2] + t2 * 9 * k[3])));
}

/* Validity limit of the fisheye model (reading R6): the first angle in
 * (0, pi/2] where d theta_d / d theta reaches 0, else pi/2. */
double ora_theta_lim(const double k[4]) {
  const int steps = 4096;
  double prev = 0.0;
  for (int i = 1; i <= steps; i++) {
    double th = 0.5 * M_PI * i / steps;
    if (fisheye_dthetad(k, th) <= 0) {
      double lo = prev, hi = th;
      for (int it = 0; it < 200; it++) {
        double mid = 0.5 * (lo + hi);
        if (fisheye_dthetad(k, mid) > 0) lo = mid; else hi = mid;
      }
      return lo;
    }
    prev = th;
  }
  return 0.5 * M_PI;
}

static void camctx_init(camctx* X, const ora_camera* c) {
  double Q0[9], Q1[9];
  X->c = c;
  matTvec(c->R0, c->t0, X->c0);
  matTvec(c->R1, c->t1, X->c1);
  for (int i = 0; i < 3; i++) { X->c0[i] = -X->c0[i]; X->c1[i] = -X->c1[i]; }
  for (int r = 0; r < 3; r++)
    for (int k = 0; k < 3; k++) { Q0[3 * r + k] = c->R0[3 * k + r]; Q1[3 * r + k] = c->R1[3 * k + r]; }
  rot_to_quat(Q0, X->q0);
  rot_to_quat(Q1, X->q1);
  X->theta_lim = c->model == ORA_FISHEYE ? ora_theta_lim(c->k) : 0.5 * M_PI;
  X->thetad_lim = fisheye_thetad(c->k, X->theta_lim);
}

/* Camera pose at exposure time t.  Global shutter: the start pose.  Rolling
 * shutter (reading R7): camera centre interpolated linearly, camera-to-world
 * rotation by spherical linear interpolation of the two quaternions. */
static void pose_ctx(const camctx* X, double t, double Rwc[9], double centre[3]) {
  const ora_camera* c = X->c;
  if (c->shutter == ORA_GLOBAL) {
    memcpy(Rwc, c->R0, 9 * sizeof(double));
    memcpy(centre, X->c0, 3 * sizeof(double));
    return;
  }
  double q0[4], q1[4], q[4], Q[9];
  memcpy(q0, X->q0, sizeof(q0));
  memcpy(q1, X->q1, sizeof(q1));
  double cosom = q0[0] * q1[0] + q0[1] * q1[1] + q0[2] * q1[2] + q0[3] * q1[3];
  if (cosom < 0) { cosom = -cosom; for (int i = 0; i < 4; i++) q1[i] = -q1[i]; }
  if (cosom > 1.0 - 1e-15) {
    for (int i = 0; i < 4; i++) q[i] = (1 - t) * q0[i] + t * q1[i];
  } else {
    double om = acos(cosom), so = sin(om);
    double a = sin((1 - t) * om) / so, b = sin(t * om) / so;
    for (int i = 0; i < 4; i++) q[i] = a * q0[i] + b * q1[i];
  }
  ora_quat_to_rot(q, Q);
  for (int r = 0; r < 3; r++)
    for (int k = 0; k < 3; k++) Rwc[3 * r + k] = Q[3 * k + r];
  for (int i = 0; i < 3; i++) centre[i] = (1 - t) * X->c0[i] + t * X->c1[i];
}

void ora_pose(const ora_camera* c, double t, double Rwc[9], double centre[3]) {
  camctx X;
  camctx_init(&X, c);
  pose_ctx(&X, t, Rwc, centre);
}

/* g(x): world point -> pixel coordinates at exposure time t (readings R3-R5,
 * R8).  Pinhole: valid in front of the near plane.  Fisheye: valid up to the
 * validity angle and beyond the near distance. */
static int project_ctx(const camctx* X, const ora_params* p, double t, const double x[3],
                       double v[2], double* margin) {
  const ora_camera* c = X->c;
  double Rwc[9], cen[3], rel[3], xc[3];
  pose_ctx(X, t, Rwc, cen);
  for (int i = 0; i < 3; i++) rel[i] = x[i] - cen[i];
  matvec(Rwc, rel, xc);
  if (c->model == ORA_PINHOLE) {
    *margin = xc[2] - p->near_plane;
    if (xc[2] != 0.0) {
      v[0] = c->fx * xc[0] / xc[2] + c->cx;
      v[1] = c->fy * xc[1] / xc[2] + c->cy;
    } else {
      v[0] = v[1] = 0.0;
    }
    return xc[2] > p->near_plane;
  }
  double r = sqrt(xc[0] * xc[0] + xc[1] * xc[1]);
  double th = atan2(r, xc[2]);
  double rho = sqrt(dot3(xc, xc));
  double m1 = X->theta_lim - th, m2 = rho - p->near_plane;
  *margin = m1 < m2 ? m1 : m2;
  double td = fisheye_thetad(c->k, th);
  if (r > 0) {
    v[0] = c->fx * td * xc[0] / r + c->cx;
    v[1] = c->fy * td * xc[1] / r + c->cy;
  } else {
    v[0] = c->cx;
    v[1] = c->cy;
  }
  return th <= X->theta_lim && rho > p->near_plane;
}

int ora_project_point(const ora_camera* c, const ora_params* p, double t, const double x[3],
                      double v[2], double* margin) {
  camctx X;
  camctx_init(&X, c);
  return project_ctx(&X, p, t, x, v, margin);
}

/* Exposure time of a point under a rolling shutter (reading R7): the row the
 * point lands in fixes its time; iterate t <- clamp((v_y - 1/2)/(H - 1), 0, 1)
 * from t = 1/2, keeping t when a projection is invalid, then project at the
 * final t.  Global shutter: t = 0. */
static int solve_time_ctx(const camctx* X, const ora_params* p, int iters, const double x[3],
                          double* t_out, double v[2], double* margin) {
  const ora_camera* c = X->c;
  double t = 0.0, mmin = INFINITY, m;
  if (c->shutter == ORA_ROLLING) {
    t = 0.5;
    double denom = c->height > 1 ? (double)(c->height - 1) : 1.0;
    for (int it = 0; it < iters; it++) {
      double vv[2];
      int ok = project_ctx(X, p, t, x, vv, &m);
      if (m < mmin) mmin = m;
      if (ok) t = c->height > 1 ? clampd((vv[1] - 0.5) / denom, 0.0, 1.0) : 0.0;
    }
  }
  int ok = project_ctx(X, p, t, x, v, &m);
  if (m < mmin) mmin = m;
  *margin = mmin;
  *t_out = t;
  return ok;
}

int ora_solve_time(const ora_camera* c, const ora_params* p, int iters, const double x[3],
                   double* t_out, double v[2], double* margin) {
  camctx X;
  camctx_init(&X, c);
  return solve_time_ctx(&X, p, iters, x, t_out, v, margin);
}

/* Monte-Carlo reference projection (Supp. C, Gaussian projection quality):
 * each world point goes through the camera as a sigma point does, with its
 * rolling-shutter exposure time solved by `iters` fixed-point iterations. */
void ora_project_samples(const ora_camera* c, const ora_params* p, int iters, int64_t m,
                         const double* x, double* v, int32_t* ok) {
  camctx X;
  camctx_init(&X, c);
  for (int64_t j = 0; j < m; j++) {
    double t, margin;
    ok[j] = solve_time_ctx(&X, p, iters, &x[3 * j], &t, &v[2 * j], &margin);
  }
}

/* EWA projection (Eq. 3): the mean projected at exposure time t, and the
 * covariance J Sigma J^T with J the Jacobian of the camera's projection of a
 * world point at that fixed time (the first-order Taylor term, here taken by
 * central differences of step h in each world axis, so it includes the lens
 * distortion but not the rolling shutter).  Returns 0 if any projection is
 * invalid. */
int ora_ewa(const ora_camera* c, const ora_params* p, double t, const double mu[3],
            const double quat[4], const double scale[3], double h, double mean2d[2],
            double cov2d[3]) {
  camctx X;
  camctx_init(&X, c);
  double margin, J[2][3];
  if (!project_ctx(&X, p, t, mu, mean2d, &margin)) return 0;
  for (int k = 0; k < 3; k++) {
    double xp[3] = {mu[0], mu[1], mu[2]}, xm[3] = {mu[0], mu[1], mu[2]}, vp[2], vm[2];
    xp[k] += h;
    xm[k] -= h;
    if (!project_ctx(&X, p, t, xp, vp, &margin) || !project_ctx(&X, p, t, xm, vm, &margin)) return 0;
    J[0][k] = (vp[0] - vm[0]) / (2 * h);
    J[1][k] = (vp[1] - vm[1]) / (2 * h);
  }
  /* Sigma = R diag(s^2) R^T (Eq. 2) */
  double R[9], S[9];
  ora_quat_to_rot(quat, R);
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      double acc = 0;
      for (int k = 0; k < 3; k++) acc += R[3 * a + k] * scale[k] * scale[k] * R[3 * b + k];
      S[3 * a + b] = acc;
    }
  double JS[2][3];
  for (int r = 0; r < 2; r++)
    for (int b = 0; b < 3; b++) {
      double acc = 0;
      for (int k = 0; k < 3; k++) acc += J[r][k] * S[3 * k + b];
      JS[r][b] = acc;
    }
  double C[2][2];
  for (int r = 0; r < 2; r++)
    for (int q = 0; q < 2; q++) {
      double acc = 0;
      for (int k = 0; k < 3; k++) acc += JS[r][k] * J[q][k];
      C[r][q] = acc;
    }
  cov2d[0] = C[0][0];
  cov2d[1] = C[0][1];
  cov2d[2] = C[1][1];
  return 1;
}

/* Ray through pixel-centre coordinates (u, v): origin and direction in world
 * space.  Rolling shutter: the pose of row floor(v) at t = row/(H-1).
 * Fisheye: theta from theta_d by bisection on [0, theta_lim]; pixels outside
 * the image circle theta_d(theta_lim) have no ray (returns 0, but o and d are
 * still filled with the ray at the circle for the ambiguity check). */
static int pixel_ray_ctx(const camctx* X, double u, double v, double o[3], double d[3],
                         double* margin) {
  const ora_camera* c = X->c;
  double t = 0.0;
  if (c->shutter == ORA_ROLLING && c->height > 1) t = floor(v) / (double)(c->height - 1);
  double dc[3];
  int ok = 1;
  *margin = INFINITY;
  if (c->model == ORA_PINHOLE) {
    dc[0] = (u - c->cx) / c->fx;
    dc[1] = (v - c->cy) / c->fy;
    dc[2] = 1.0;
  } else {
    double mx = (u - c->cx) / c->fx, my = (v - c->cy) / c->fy;
    double td = sqrt(mx * mx + my * my);
    *margin = X->thetad_lim - td;
    ok = td <= X->thetad_lim;
    double target = td < X->thetad_lim ? td : X->thetad_lim;
    double lo = 0.0, hi = X->theta_lim;
    for (int it = 0; it < 100; it++) {
      double mid = 0.5 * (lo + hi);
      if (fisheye_thetad(c->k, mid) < target) lo = mid; else hi = mid;
    }
    double th = 0.5 * (lo + hi);
    if (td > 0) {
      dc[0] = sin(th) * mx / td;
      dc[1] = sin(th) * my / td;
    } else {
      dc[0] = dc[1] = 0.0;
    }
    dc[2] = cos(th);
  }
  double Rwc[9];
  pose_ctx(X, t, Rwc, o);
  matTvec(Rwc, dc, d);
  return ok;
}

int ora_pixel_ray(const ora_camera* c, double u, double v, double o[3], double d[3],
                  double* margin) {
  camctx X;
  camctx_init(&X, c);
  return pixel_ray_ctx(&X, u, v, o, d, margin);
}

/* ------------------------------------------------------------------------- */
/* Real spherical harmonics (radiance phi_beta(d), Sec. 3), from Legendre     */
/* polynomials: Y_l^m = N_lm Q_l^|m|(z) * {1, sqrt2 Re (x+iy)^m, sqrt2 Im ...}, */
/* Q_l^m = (-1)^m d^m P_l / dz^m, N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).    */
/* ------------------------------------------------------------------------- */

static double factorial(int n) { double f = 1; for (int i = 2; i <= n; i++) f *= i; return f; }

static void legendre_poly(int l, double c[8]) {
  double pm[8] = {1}, p[8] = {0, 1};
  if (l == 0) { memset(c, 0, 8 * sizeof(double)); c[0] = 1; return; }
  for (int n = 1; n < l; n++) { /* (n+1) P_{n+1} = (2n+1) z P_n - n P_{n-1} */
    double nx[8] = {0};
    for (int j = 0; j < 7; j++) nx[j + 1] += (2 * n + 1) * p[j] / (n + 1);
    for (int j = 0; j < 8; j++) nx[j] -= n * pm[j] / (n + 1);
    memcpy(pm, p, sizeof(p));
    memcpy(p, nx, sizeof(p));
  }
  memcpy(c, p, 8 * sizeof(double));
}

static void sh_term(int l, int m, const double d[3], double* Y, double g[3]) {
  int a = m < 0 ? -m : m;
  double c[8];
  legendre_poly(l, c);
  for (int r = 0; r < a; r++) /* differentiate a times */
    for (int j = 0; j < 7; j++) c[j] = c[j + 1] * (j + 1);
  double sgn = (a % 2) ? -1.0 : 1.0;
  double Q = 0, dQ = 0, zp = 1;
  for (int j = 0; j < 8; j++) { Q += c[j] * zp; zp *= d[2]; }
  zp = 1;
  for (int j = 1; j < 8; j++) { dQ += j * c[j] * zp; zp *= d[2]; }
  Q *= sgn;
  dQ *= sgn;
  double N = sqrt((2 * l + 1) / (4 * M_PI) * factorial(l - a) / factorial(l + a));
  /* (x + i y)^a and a (x + i y)^(a-1) */
  double re = 1, im = 0, re1 = 0, im1 = 0;
  for (int k = 0; k < a; k++) {
    re1 = re; im1 = im;
    double nr = re * d[0] - im * d[1], ni = re * d[1] + im * d[0];
    re = nr; im = ni;
  }
  /* re1 + i im1 = (x+iy)^(a-1) */
  double trig, tx, ty;
  if (m == 0) { trig = 1; tx = ty = 0; }
  else if (m > 0) { trig = sqrt(2.0) * re; tx = sqrt(2.0) * a * re1; ty = -sqrt(2.0) * a * im1; }
  else { trig = sqrt(2.0) * im; tx = sqrt(2.0) * a * im1; ty = sqrt(2.0) * a * re1; }
  *Y = N * Q * trig;
  if (g) {
    g[0] = N * Q * tx;
    g[1] = N * Q * ty;
    g[2] = N * dQ * trig;
  }
}

void ora_sh_basis(int degree, const double dir[3], double* Y) {
  for (int l = 0; l <= degree; l++)
    for (int m = -l; m <= l; m++) sh_term(l, m, dir, &Y[l * l + l + m], NULL);
}
void ora_sh_basis_grad(int degree, const double dir[3], double* dY) {
  for (int l = 0; l <= degree; l++)
    for (int m = -l; m <= l; m++) {
      double y;
      sh_term(l, m, dir, &y, &dY[3 * (l * l + l + m)]);
    }
}

/* ------------------------------------------------------------------------- */
/* Unscented transform (Eq. 6-10, Alg. 2)                                     */
/* ------------------------------------------------------------------------- */

void ora_ut_weights(double a, double b, double kappa, double* lambda, double wm[7], double wc[7]) {
  double lam = a * a * (3 + kappa) - 3; /* lambda = alpha^2 (3 + kappa) - 3 */
  *lambda = lam;
  wm[0] = lam / (3 + lam);
  wc[0] = lam / (3 + lam) + (1 - a * a + b);
  for (int i = 1; i < 7; i++) wm[i] = wc[i] = 1.0 / (2 * (3 + lam));
}

/* Sigma points x_0 = mu, x_{i}, x_{i+3} = mu +/- sqrt((3+lambda) Sigma)_[i],
 * with the square root read off the factorisation Sigma = R S S^T R^T:
 * column i of R S (reading R1). */
static void sigma_points(const double mu[3], const double R[9], const double s[3], double lam,
                         double X[7][3]) {
  double g = sqrt(3 + lam);
  for (int j = 0; j < 3; j++) X[0][j] = mu[j];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double col = R[3 * j + i] * s[i];
      X[1 + i][j] = mu[j] + g * col;
      X[4 + i][j] = mu[j] - g * col;
    }
}

static void ut_moments(double V[7][2], const double wm[7], const double wc[7], double mean[2],
                       double cov[3]) {
  mean[0] = mean[1] = 0;
  for (int i = 0; i < 7; i++) { mean[0] += wm[i] * V[i][0]; mean[1] += wm[i] * V[i][1]; }
  cov[0] = cov[1] = cov[2] = 0;
  for (int i = 0; i < 7; i++) {
    double dx = V[i][0] - mean[0], dy = V[i][1] - mean[1];
    cov[0] += wc[i] * dx * dx;
    cov[1] += wc[i] * dx * dy;
    cov[2] += wc[i] * dy * dy;
  }
}

void ora_ut_affine(const double mu[3], const double quat[4], const double scale[3],
                   const ora_params* p, const double A[6], const double b[2], double mean2d[2],
                   double cov2d[3]) {
  double R[9], X[7][3], V[7][2], lam, wm[7], wc[7];
  ora_quat_to_rot(quat, R);
  ora_ut_weights(p->ut_alpha, p->ut_beta, p->ut_kappa, &lam, wm, wc);
  sigma_points(mu, R, scale, lam, X);
  for (int i = 0; i < 7; i++)
    for (int r = 0; r < 2; r++) V[i][r] = A[3 * r] * X[i][0] + A[3 * r + 1] * X[i][1] + A[3 * r + 2] * X[i][2] + b[r];
  ut_moments(V, wm, wc, mean2d, cov2d);
}

/* ------------------------------------------------------------------------- */
/* Project (Alg. 1 with Alg. 2 as Estimate2DGaussian)                         */
/* ------------------------------------------------------------------------- */

static void sh_color(int degree, const double* beta /* [K,3] */, const double dir[3], double raw[3]) {
  double Y[16];
  int K = (degree + 1) * (degree + 1);
  ora_sh_basis(degree, dir, Y);
  for (int ch = 0; ch < 3; ch++) {
    double acc = 0.5;
    for (int k = 0; k < K; k++) acc += beta[3 * k + ch] * Y[k];
    raw[ch] = acc;
  }
}

static int tiles_x(const ora_camera* c, const ora_params* p) { return (c->width + p->tile - 1) / p->tile; }
static int tiles_y(const ora_camera* c, const ora_params* p) { return (c->height + p->tile - 1) / p->tile; }

/* Particle response at squared canonical distance w2 = omega^2 (Supp. A):
 * rho = exp(-lambda (w2)^(n/2)), the generalized Gaussian of degree n.  The
 * scale lambda is chosen so that rho at distance r = 3 equals the reference
 * Gaussian's exp(-r^2 / 2); that reading gives lambda = r^(2-n) / 2, so that
 * degree 2 is exactly the Gaussian exp(-omega^2 / 2) of Eq. 11. */
static double kernel_lambda(int n) { return 0.5 * pow(3.0, 2.0 - n); }

static double response(const ora_params* p, double w2) {
  const int n = p->kernel_degree;
  if (n == 2) return exp(-0.5 * w2);
  return exp(-kernel_lambda(n) * pow(w2, 0.5 * n));
}

/* d rho / d omega^2 = -lambda (n/2) (omega^2)^(n/2 - 1) rho */
static double response_dw2(const ora_params* p, double w2) {
  const int n = p->kernel_degree;
  if (n == 2) return -0.5 * exp(-0.5 * w2);
  return -kernel_lambda(n) * 0.5 * n * pow(w2, 0.5 * n - 1.0) * response(p, w2);
}

/* The canonical distance at which sigma rho falls to alpha_min:
 * lambda k^n = ln(sigma / alpha_min). */
static double cutoff_distance(const ora_params* p, double sig) {
  const int n = p->kernel_degree;
  if (n == 2) return sqrt(2.0 * log(sig / p->alpha_min));
  return pow(log(sig / p->alpha_min) / kernel_lambda(n), 1.0 / n);
}

int ora_project(const ora_scene* s, const ora_camera* c, const ora_params* p, ora_proj* out) {
  const int K = (s->sh_degree + 1) * (s->sh_degree + 1);
  const int tx = tiles_x(c, p), ty = tiles_y(c, p);
  double lam, wm[7], wc[7];
  camctx CX;
  camctx_init(&CX, c);
  ora_ut_weights(p->ut_alpha, p->ut_beta, p->ut_kappa, &lam, wm, wc);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < s->n; i++) {
    const double* mu = &s->means[3 * i];
    double sig = s->opacities[i];
    int cull = 0;
    memset(&out->mean2d[2 * i], 0, 2 * sizeof(double));
    memset(&out->cov2d[3 * i], 0, 3 * sizeof(double));
    memset(&out->edge[4 * i], 0, 4 * sizeof(double));
    for (int j = 0; j < 4; j++) out->rect[4 * i + j] = 0;
    out->tiles[i] = 0;
    out->depth[i] = 0;
    out->tstar[i] = 0;
    out->valid_margin[i] = INFINITY;
    out->kext[i] = 0;
    for (int j = 0; j < 3; j++) out->rgb[3 * i + j] = out->rgb_raw[3 * i + j] = 0;
    if (sig < p->alpha_min) { out->cull[i] = 1; continue; } /* can never reach alpha_min */

    double R[9], X[7][3], V[7][2], T7[7], mmin = INFINITY;
    int all_ok = 1;
    ora_quat_to_rot(&s->quats[4 * i], R);
    sigma_points(mu, R, &s->scales[3 * i], lam, X);
    for (int k = 0; k < 7; k++) {
      double m;
      int ok = solve_time_ctx(&CX, p, p->rs_iters, X[k], &T7[k], V[k], &m);
      all_ok &= ok;
      if (m < mmin) mmin = m;
    }
    out->valid_margin[i] = mmin;
    out->tstar[i] = T7[0];
    double mean[2], cov[3];
    ut_moments(V, wm, wc, mean, cov);
    out->mean2d[2 * i] = mean[0]; out->mean2d[2 * i + 1] = mean[1];
    out->cov2d[3 * i] = cov[0]; out->cov2d[3 * i + 1] = cov[1]; out->cov2d[3 * i + 2] = cov[2];
    if (!all_ok) cull = 2;

    /* Extent(Sigma', sigma) (reading R10): the k-sigma box with k the
     * distance at which sigma * rho(k^2) reaches alpha_min, capped at 3. */
    double ks = cutoff_distance(p, sig);
    if (ks > p->k_sigma_max) ks = p->k_sigma_max;
    out->kext[i] = ks;
    double hx = ks * sqrt(cov[0] > 0 ? cov[0] : 0), hy = ks * sqrt(cov[2] > 0 ? cov[2] : 0);
    double* e = &out->edge[4 * i];
    e[0] = mean[0] - hx; e[1] = mean[1] - hy; e[2] = mean[0] + hx; e[3] = mean[1] + hy;
    /* ComputeRectangle: tiles [floor((v-h)/tile), floor((v+h)/tile)] clipped. */
    int x0 = (int)floor(e[0] / p->tile), y0 = (int)floor(e[1] / p->tile);
    int x1 = (int)floor(e[2] / p->tile), y1 = (int)floor(e[3] / p->tile);
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > tx - 1) x1 = tx - 1;
    if (y1 > ty - 1) y1 = ty - 1;
    if (cull == 0 && (x0 > x1 || y0 > y1)) cull = 3;
    int* r = &out->rect[4 * i];
    r[0] = x0; r[1] = y0; r[2] = x1; r[3] = y1;
    out->tiles[i] = cull == 0 ? (x1 - x0 + 1) * (y1 - y0 + 1) : 0;

    /* Sort depth (reading R11) and view-dependent colour (reading R13) from
     * the camera centre at the mean point's exposure time. */
    double Rwc[9], cen[3], dv[3];
    pose_ctx(&CX, T7[0], Rwc, cen);
    for (int j = 0; j < 3; j++) dv[j] = mu[j] - cen[j];
    double dist = sqrt(dot3(dv, dv));
    out->depth[i] = dist;
    for (int j = 0; j < 3; j++) dv[j] /= dist;
    double raw[3];
    sh_color(s->sh_degree, &s->sh[(int64_t)3 * K * i], dv, raw);
    for (int j = 0; j < 3; j++) {
      out->rgb_raw[3 * i + j] = raw[j];
      out->rgb[3 * i + j] = raw[j] > 0 ? raw[j] : 0;
    }
    out->cull[i] = cull;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Bin: per-tile lists ordered by (depth, particle id) (Sec. 4.3)             */
/* ------------------------------------------------------------------------- */

typedef struct { double depth; int32_t id; int32_t flags; } bin_entry;

static int cmp_entry(const void* a, const void* b) {
  const bin_entry* x = (const bin_entry*)a;
  const bin_entry* y = (const bin_entry*)b;
  if (x->depth < y->depth) return -1;
  if (x->depth > y->depth) return 1;
  return (x->id > y->id) - (x->id < y->id);
}

static int floordiv(double v, int t) { return (int)floor(v / t); }

/* Rectangles of particle i: primary (exact), maximal and minimal (edges moved
 * by +/- amb->edge pixels).  Returns 0 if the particle cannot be in any list. */
static int particle_rects(const ora_proj* pr, int64_t i, const ora_camera* c, const ora_params* p,
                          const ora_amb* amb, int prim[4], int mx[4], int mn[4], int* undecided) {
  int cull = pr->cull[i];
  if (cull == 1) return 0;
  int valid_undecided = fabs(pr->valid_margin[i]) < amb->valid;
  if (cull == 2 && !valid_undecided) return 0;
  const double* e = &pr->edge[4 * i];
  const int tx = tiles_x(c, p), ty = tiles_y(c, p);
  double d = amb->edge;
  int lim[4] = {0, 0, tx - 1, ty - 1};
  for (int j = 0; j < 4; j++) {
    prim[j] = floordiv(e[j], p->tile);
    int lo = floordiv(e[j] - d, p->tile), hi = floordiv(e[j] + d, p->tile);
    mx[j] = j < 2 ? lo : hi;
    mn[j] = j < 2 ? hi : lo;
  }
  for (int j = 0; j < 2; j++) {
    if (prim[j] < lim[j]) prim[j] = lim[j];
    if (mx[j] < lim[j]) mx[j] = lim[j];
    if (mn[j] < lim[j]) mn[j] = lim[j];
  }
  for (int j = 2; j < 4; j++) {
    if (prim[j] > lim[j]) prim[j] = lim[j];
    if (mx[j] > lim[j]) mx[j] = lim[j];
    if (mn[j] > lim[j]) mn[j] = lim[j];
  }
  if (cull != 0) prim[0] = 1, prim[2] = 0; /* culled: primary rect is empty */
  *undecided = valid_undecided;
  return mx[0] <= mx[2] && mx[1] <= mx[3];
}

int ora_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
}

double ora_ellipse_box_qmin(const double m[2], const double A[3], double x0, double y0,
                            double x1, double y1) {
  const double det = A[0] * A[2] - A[1] * A[1];
  if (!(det > 0)) return 0.0; /* degenerate ellipse: no culling */
  if (m[0] >= x0 && m[0] <= x1 && m[1] >= y0 && m[1] <= y1) return 0.0;
  /* Q = A^-1; outside the box the minimum of the convex form lies on its
   * boundary: the smallest of the four edges' clamped one-dimensional minima */
  const double Qxx = A[2] / det, Qxy = -A[1] / det, Qyy = A[0] / det;
  double best = INFINITY;
  for (int e = 0; e < 2; e++) { /* vertical edges x = x0, x1 */
    const double dx = (e ? x1 : x0) - m[0];
    double y = m[1] - Qxy * dx / Qyy;
    if (y < y0) y = y0;
    if (y > y1) y = y1;
    const double dy = y - m[1];
    const double q = Qxx * dx * dx + 2.0 * Qxy * dx * dy + Qyy * dy * dy;
    if (q < best) best = q;
  }
  for (int e = 0; e < 2; e++) { /* horizontal edges y = y0, y1 */
    const double dy = (e ? y1 : y0) - m[1];
    double x = m[0] - Qxy * dy / Qxx;
    if (x < x0) x = x0;
    if (x > x1) x = x1;
    const double dx = x - m[0];
    const double q = Qxx * dx * dx + 2.0 * Qxy * dx * dy + Qyy * dy * dy;
    if (q < best) best = q;
  }
  return best;
}

/* Membership of tile (x, y) in particle i's list.  The rectangle part is
 * decided (inp) or undecided (und_rect) from the extent's edges; with tile
 * culling the tile must also meet the extent ellipse (Sec. 4.1: the 2D conic
 * feeds the tiling and culling of 3DGS and StopThePop), i.e. the minimum over
 * the tile's closed box of (v-m)^T (k^2 Sigma')^-1 (v-m) is at most 1.  That
 * decision is undecided within the margin the FP32 ellipse can move: if its
 * boundary moves by at most `edge` pixels (the same bound as the rectangle's
 * edges; the error comes from the projected sigma points, in every direction
 * alike) and its matrix entries carry a relative rounding `conic`, the
 * decision can flip only for
 *   |sqrt(q_min) - 1| <= edge / sqrt(lambda_min) + conic trace / (2 lambda_min),
 * lambda_min being the smaller eigenvalue of k^2 Sigma' (the ellipse grown by
 * `edge` pixels lies inside q <= (1 + edge / sqrt(lambda_min))^2, the one
 * shrunk by it contains q <= (1 - edge / sqrt(lambda_min))^2).  Returns bit0
 * primary member, bit1 undecided. */
static int tile_membership(const ora_proj* pr, int64_t i, const ora_params* p, const ora_amb* amb,
                           int x, int y, int inp, int und_rect) {
  int ein = 1, eund = 0;
  if (p->tile_cull) {
    const double k2 = pr->kext[i] * pr->kext[i];
    const double A[3] = {k2 * pr->cov2d[3 * i], k2 * pr->cov2d[3 * i + 1], k2 * pr->cov2d[3 * i + 2]};
    const double tr = A[0] + A[2], det = A[0] * A[2] - A[1] * A[1];
    const double disc = sqrt(0.25 * (A[0] - A[2]) * (A[0] - A[2]) + A[1] * A[1]);
    const double lmax = 0.5 * tr + disc, lmin = lmax > 0 ? det / lmax : 0.0;
    if (!(lmin > 0)) {
      eund = 1; /* degenerate in FP64: kept here, the FP32 side may cull */
    } else {
      const double t = p->tile;
      const double q = ora_ellipse_box_qmin(&pr->mean2d[2 * i], A, x * t, y * t, (x + 1) * t, (y + 1) * t);
      const double margin = amb->edge / sqrt(lmin) + 0.5 * amb->conic * tr / lmin;
      ein = q <= 1.0;
      eund = fabs(sqrt(q) - 1.0) <= margin;
    }
  }
  const int member = inp && ein;
  const int undec = (und_rect || eund) && (inp || und_rect) && (ein || eund);
  return (member ? 1 : 0) | (undec ? 2 : 0);
}

int64_t ora_bin(int64_t n, const ora_proj* pr, const ora_camera* c, const ora_params* p,
                const ora_amb* amb, int64_t* tile_start, int32_t* ids, int32_t* flags) {
  const int tx = tiles_x(c, p), ty = tiles_y(c, p);
  const int64_t T = (int64_t)tx * ty;
  int64_t* cnt = (int64_t*)calloc(T + 1, sizeof(int64_t));
  for (int64_t i = 0; i < n; i++) {
    int pm[4], mx[4], mn[4], und;
    if (!particle_rects(pr, i, c, p, amb, pm, mx, mn, &und)) continue;
    for (int y = mx[1]; y <= mx[3]; y++)
      for (int x = mx[0]; x <= mx[2]; x++) {
        int inp = x >= pm[0] && x <= pm[2] && y >= pm[1] && y <= pm[3];
        int inmin = x >= mn[0] && x <= mn[2] && y >= mn[1] && y <= mn[3];
        if (tile_membership(pr, i, p, amb, x, y, inp, und || !inmin)) cnt[(int64_t)y * tx + x]++;
      }
  }
  int64_t total = 0;
  for (int64_t t = 0; t < T; t++) total += cnt[t];
  if (!ids) { free(cnt); return total; }
  tile_start[0] = 0;
  for (int64_t t = 0; t < T; t++) tile_start[t + 1] = tile_start[t] + cnt[t];
  bin_entry* ent = (bin_entry*)malloc((total > 0 ? total : 1) * sizeof(bin_entry));
  memset(cnt, 0, (T + 1) * sizeof(int64_t));
  for (int64_t i = 0; i < n; i++) {
    int pm[4], mx[4], mn[4], und;
    if (!particle_rects(pr, i, c, p, amb, pm, mx, mn, &und)) continue;
    for (int y = mx[1]; y <= mx[3]; y++)
      for (int x = mx[0]; x <= mx[2]; x++) {
        int inp = x >= pm[0] && x <= pm[2] && y >= pm[1] && y <= pm[3];
        int inmin = x >= mn[0] && x <= mn[2] && y >= mn[1] && y <= mn[3];
        const int fl = tile_membership(pr, i, p, amb, x, y, inp, und || !inmin);
        if (!fl) continue;
        int64_t t = (int64_t)y * tx + x;
        bin_entry* b = &ent[tile_start[t] + cnt[t]++];
        b->depth = pr->depth[i];
        b->id = (int32_t)i;
        b->flags = fl;
      }
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < T; t++)
    qsort(&ent[tile_start[t]], (size_t)(tile_start[t + 1] - tile_start[t]), sizeof(bin_entry), cmp_entry);
  for (int64_t k = 0; k < total; k++) { ids[k] = ent[k].id; flags[k] = ent[k].flags; }
  free(ent);
  free(cnt);
  return total;
}

/* ------------------------------------------------------------------------- */
/* Particle response on a ray: Eq. 11 and alpha = sigma * rho (Eq. 5)         */
/* ------------------------------------------------------------------------- */

typedef struct {
  double mu[3], M[9], sigma; /* M = S^-1 R^T */
} particle_geo;

static void make_geo(const ora_scene* s, int64_t i, particle_geo* g) {
  double R[9];
  ora_quat_to_rot(&s->quats[4 * i], R);
  for (int k = 0; k < 3; k++) {
    g->mu[k] = s->means[3 * i + k];
    for (int j = 0; j < 3; j++) g->M[3 * k + j] = R[3 * j + k] / s->scales[3 * i + k];
  }
  g->sigma = s->opacities[i];
}

/* o_g = S^-1 R^T (o - mu), d_g = S^-1 R^T d; tau_max = -o_g.d_g / d_g.d_g;
 * omega^2 = |o_g x d_g|^2 / |d_g|^2 (the squared canonical distance of the
 * maximum-response point, formed without cancellation). */
static void eval_geo(const particle_geo* g, const double o[3], const double d[3], double og[3],
                     double dg[3], double* odot, double* om2) {
  double rel[3] = {o[0] - g->mu[0], o[1] - g->mu[1], o[2] - g->mu[2]}, cr[3];
  matvec(g->M, rel, og);
  matvec(g->M, d, dg);
  *odot = dot3(og, dg);
  cross3(og, dg, cr);
  *om2 = dot3(cr, cr) / dot3(dg, dg);
}

int ora_particle_alpha(const double mu[3], const double quat[4], const double scale[3],
                       double opacity, const double o[3], const double d[3], int32_t kernel_degree,
                       double* tau_max, double* omega2, double* alpha_raw) {
  ora_params kp;
  kp.kernel_degree = kernel_degree;
  double R[9];
  particle_geo g;
  ora_quat_to_rot(quat, R);
  for (int k = 0; k < 3; k++) {
    g.mu[k] = mu[k];
    for (int j = 0; j < 3; j++) g.M[3 * k + j] = R[3 * j + k] / scale[k];
  }
  g.sigma = opacity;
  double og[3], dg[3], odot, om2;
  eval_geo(&g, o, d, og, dg, &odot, &om2);
  *tau_max = -odot / dot3(dg, dg);
  *omega2 = om2;
  *alpha_raw = opacity * response(&kp, om2);
  return odot < 0;
}

/* ------------------------------------------------------------------------- */
/* Render: front-to-back Eq. 5 over the tile list, response at tau_max        */
/* ------------------------------------------------------------------------- */

enum { PT_NONE = 0, PT_TOGGLE, PT_ALPHA, PT_STOP, PT_TAU, PT_SWAP, PT_CLIP, PT_ORDER };
typedef struct { int type; int64_t pos, pos2; } perturb;
typedef struct { double rgb[3], T; int nc, ne; } pix_result;

typedef struct {
  const ora_scene* s;
  const ora_proj* pr;
  const ora_params* p;
  const particle_geo* geo;
  const ora_amb* amb;
} render_ctx;

#define MAXCAND 64

/* Hybrid rendering (Sec. 6.2): the rasterizer discards a hit whose
 * maximum-response point tau_max lies beyond the ray's closest surface
 * intersection, clipv (distance along the ray from its origin; INFINITY:
 * none). */
static double hit_distance(double odot, const double dg[3], const double d[3]) {
  return -odot / dot3(dg, dg) * sqrt(dot3(d, d));
}

static void add_cand(perturb* cand, int* ncand, perturb c) {
  if (!cand || *ncand >= MAXCAND) return;
  for (int i = 0; i < *ncand; i++)
    if (cand[i].type == c.type && cand[i].pos == c.pos && cand[i].pos2 == c.pos2) return;
  cand[(*ncand)++] = c;
}

/* "Ours (sorted)" (Sec. 4.3): multi-layer alpha blending with a per-ray
 * buffer of the k farthest hits seen so far.  A hit is a list entry with
 * tau_max > 0, not clipped and alpha >= alpha_min, placed at its
 * maximum-response distance along the ray.  While the buffer has room, a hit
 * is inserted in distance order (after nearer ones, before equal or farther
 * ones).  Once it is full, the nearer of the new hit and the buffer's nearest
 * is blended into the pixel front to back; if that was the buffered one, the
 * new hit takes a place in the buffer.  Blending stops before a hit that
 * would take T below t_min (the blended part's transmittance has vanished);
 * at the end of the list the buffer is blended nearest first under the same
 * rule.  n_contrib counts blended hits. */
typedef struct { double dist, a; int64_t q; int32_t id; } hit_rec;
#define ORA_MAXK 256

/* x strictly nearer than y; PT_ORDER flips the order of one pair. */
static int nearer(const render_ctx* X, const hit_rec* x, const hit_rec* y, perturb pt, perturb* cand,
                  int* ncand) {
  int r = x->dist < y->dist;
  if (fabs(x->dist - y->dist) <= X->amb->order * fmax(x->dist, y->dist))
    add_cand(cand, ncand, (perturb){PT_ORDER, x->q < y->q ? x->q : y->q, x->q < y->q ? y->q : x->q});
  if (pt.type == PT_ORDER && ((pt.pos == x->q && pt.pos2 == y->q) || (pt.pos == y->q && pt.pos2 == x->q)))
    r = !r;
  return r;
}

/* Eq. 5 for one hit; returns 1 (and adds nothing) if it would take T below t_min. */
static int blend_hit(const render_ctx* X, const hit_rec* h, double* T, double C[3], int* nc, perturb pt,
                     perturb* cand, int* ncand) {
  const ora_params* p = X->p;
  const double Tn = *T * (1.0 - h->a);
  if (fabs(Tn / p->t_min - 1.0) < X->amb->trans) add_cand(cand, ncand, (perturb){PT_STOP, h->q, 0});
  int stop = Tn < p->t_min;
  if (pt.type == PT_STOP && pt.pos == h->q) stop = !stop;
  if (stop) return 1;
  const double* c = &X->pr->rgb[3 * h->id];
  for (int ch = 0; ch < 3; ch++) C[ch] += h->a * *T * c[ch];
  *T = Tn;
  (*nc)++;
  return 0;
}

static void render_pixel_kbuffer(const render_ctx* X, const int32_t* ids, const int32_t* flags,
                                 int64_t L, const double o[3], const double d[3], double clipv,
                                 perturb pt, pix_result* res, perturb* cand, int* ncand) {
  const ora_params* p = X->p;
  const int k = p->kbuffer < ORA_MAXK ? p->kbuffer : ORA_MAXK;
  hit_rec buf[ORA_MAXK];
  int n = 0, nc = 0, member_pos = 0, ne = -1, stopped = 0;
  double T = 1.0, C[3] = {0, 0, 0};
  for (int64_t pos = 0; pos < L && !stopped; pos++) {
    int64_t q = pos;
    if (pt.type == PT_SWAP && pos == pt.pos) q = pos + 1;
    else if (pt.type == PT_SWAP && pos == pt.pos + 1) q = pos - 1;
    int member = flags[q] & 1;
    if (pt.type == PT_TOGGLE && pt.pos == q) member = !member;
    if (flags[q] & 2) add_cand(cand, ncand, (perturb){PT_TOGGLE, q, 0});
    if (pos + 1 < L && (flags[q] & 1) && (flags[q + 1] & 1)) {
      double d0 = X->pr->depth[ids[q]], d1 = X->pr->depth[ids[q + 1]];
      if (fabs(d1 - d0) <= X->amb->depth * d0) add_cand(cand, ncand, (perturb){PT_SWAP, pos, 0});
    }
    if (!member) continue;
    member_pos++;
    const particle_geo* g = &X->geo[ids[q]];
    double og[3], dg[3], odot, om2;
    eval_geo(g, o, d, og, dg, &odot, &om2);
    if (fabs(odot) < X->amb->tau * sqrt(dot3(og, og) * dot3(dg, dg)))
      add_cand(cand, ncand, (perturb){PT_TAU, q, 0});
    int skip = odot >= 0;
    if (pt.type == PT_TAU && pt.pos == q) skip = !skip;
    if (skip) continue;
    const double dist = hit_distance(odot, dg, d);
    if (isfinite(clipv)) {
      if (fabs(dist - clipv) <= X->amb->clip * clipv) add_cand(cand, ncand, (perturb){PT_CLIP, q, 0});
      int behind = dist > clipv;
      if (pt.type == PT_CLIP && pt.pos == q) behind = !behind;
      if (behind) continue;
    }
    double a = g->sigma * response(p, om2);
    if (a > p->alpha_max) a = p->alpha_max;
    if (fabs(a - p->alpha_min) < X->amb->alpha) add_cand(cand, ncand, (perturb){PT_ALPHA, q, 0});
    int below = a < p->alpha_min;
    if (pt.type == PT_ALPHA && pt.pos == q) below = !below;
    if (below) continue;
    hit_rec h = {dist, a, q, ids[q]};
    if (n == k) {
      /* full: blend the nearer of the new hit and the buffer's nearest */
      if (!nearer(X, &buf[0], &h, pt, cand, ncand)) {
        if (blend_hit(X, &h, &T, C, &nc, pt, cand, ncand)) { stopped = 1; ne = member_pos; }
        continue;
      }
      if (blend_hit(X, &buf[0], &T, C, &nc, pt, cand, ncand)) { stopped = 1; ne = member_pos; continue; }
      for (int j = 1; j < n; j++) buf[j - 1] = buf[j];
      n--;
    }
    /* insert after the hits nearer than h */
    int at = 0;
    while (at < n && nearer(X, &buf[at], &h, pt, cand, ncand)) at++;
    for (int j = n; j > at; j--) buf[j] = buf[j - 1];
    buf[at] = h;
    n++;
  }
  if (ne < 0) ne = member_pos;
  for (int j = 0; j < n && !stopped; j++)
    if (blend_hit(X, &buf[j], &T, C, &nc, pt, cand, ncand)) stopped = 1;
  for (int ch = 0; ch < 3; ch++) res->rgb[ch] = C[ch] + T * p->bg[ch];
  res->T = T;
  res->nc = nc;
  res->ne = ne;
}

static void render_pixel(const render_ctx* X, const int32_t* ids, const int32_t* flags, int64_t L,
                         const double o[3], const double d[3], double clipv, perturb pt,
                         pix_result* res, perturb* cand, int* ncand) {
  const ora_params* p = X->p;
  if (X->p->kbuffer > 0) {
    render_pixel_kbuffer(X, ids, flags, L, o, d, clipv, pt, res, cand, ncand);
    return;
  }
  double T = 1.0, C[3] = {0, 0, 0};
  int member_pos = 0, nc = 0, ne = -1;
  for (int64_t pos = 0; pos < L; pos++) {
    int64_t q = pos;
    if (pt.type == PT_SWAP && pos == pt.pos) q = pos + 1;
    else if (pt.type == PT_SWAP && pos == pt.pos + 1) q = pos - 1;
    int member = flags[q] & 1;
    if (pt.type == PT_TOGGLE && pt.pos == q) member = !member;
    if (cand && (flags[q] & 2) && *ncand < MAXCAND) cand[(*ncand)++] = (perturb){PT_TOGGLE, q};
    if (cand && pos + 1 < L && (flags[q] & 1) && (flags[q + 1] & 1) && *ncand < MAXCAND) {
      double d0 = X->pr->depth[ids[q]], d1 = X->pr->depth[ids[q + 1]];
      if (fabs(d1 - d0) <= X->amb->depth * d0) cand[(*ncand)++] = (perturb){PT_SWAP, pos};
    }
    if (!member) continue;
    member_pos++;
    const particle_geo* g = &X->geo[ids[q]];
    double og[3], dg[3], odot, om2;
    eval_geo(g, o, d, og, dg, &odot, &om2);
    if (cand && *ncand < MAXCAND &&
        fabs(odot) < X->amb->tau * sqrt(dot3(og, og) * dot3(dg, dg)))
      cand[(*ncand)++] = (perturb){PT_TAU, q};
    int skip = odot >= 0; /* tau_max <= 0: the maximum lies behind the origin (reading R15) */
    if (pt.type == PT_TAU && pt.pos == q) skip = !skip;
    if (skip) continue;
    if (isfinite(clipv)) {
      const double dist = hit_distance(odot, dg, d);
      if (cand && *ncand < MAXCAND && fabs(dist - clipv) <= X->amb->clip * clipv)
        cand[(*ncand)++] = (perturb){PT_CLIP, q};
      int behind = dist > clipv;
      if (pt.type == PT_CLIP && pt.pos == q) behind = !behind;
      if (behind) continue;
    }
    double a = g->sigma * response(p, om2);
    if (a > p->alpha_max) a = p->alpha_max;
    if (cand && *ncand < MAXCAND && fabs(a - p->alpha_min) < X->amb->alpha)
      cand[(*ncand)++] = (perturb){PT_ALPHA, q};
    int below = a < p->alpha_min;
    if (pt.type == PT_ALPHA && pt.pos == q) below = !below;
    if (below) continue;
    double Tn = T * (1.0 - a);
    if (cand && *ncand < MAXCAND && fabs(Tn / p->t_min - 1.0) < X->amb->trans)
      cand[(*ncand)++] = (perturb){PT_STOP, q};
    int stop = Tn < p->t_min; /* stop before adding (reading R16) */
    if (pt.type == PT_STOP && pt.pos == q) stop = !stop;
    if (stop) { ne = member_pos; break; }
    const double* c = &X->pr->rgb[3 * ids[q]];
    for (int ch = 0; ch < 3; ch++) C[ch] += a * T * c[ch];
    T = Tn;
    nc = member_pos;
  }
  if (ne < 0) ne = member_pos;
  for (int ch = 0; ch < 3; ch++) res->rgb[ch] = C[ch] + T * p->bg[ch];
  res->T = T;
  res->nc = nc;
  res->ne = ne;
}

static particle_geo* build_geo(const ora_scene* s, const ora_proj* pr) {
  particle_geo* geo = (particle_geo*)malloc((s->n > 0 ? s->n : 1) * sizeof(particle_geo));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < s->n; i++)
    if (pr->cull[i] != 1) make_geo(s, i, &geo[i]);
  return geo;
}

static int cmp_depth_id(const void* a, const void* b) { return cmp_entry(a, b); }

int ora_render(const ora_scene* s, const ora_proj* pr, const ora_camera* c, const ora_params* p,
               const ora_amb* amb, const int64_t* tile_start, const int32_t* ids,
               const int32_t* flags, const int32_t* tile_list, int32_t n_tiles,
               int32_t brute_force, const double* clip, ora_image* out) {
  const int tx = tiles_x(c, p), ts = p->tile;
  particle_geo* geo = build_geo(s, pr);
  render_ctx X = {s, pr, p, geo, amb};
  camctx CX;
  camctx_init(&CX, c);
  int32_t *bf_ids = NULL, *bf_flags = NULL;
  int64_t bf_n = 0;
  if (brute_force) { /* every visible particle, ordered by (depth, id), for every pixel */
    bin_entry* e = (bin_entry*)malloc((s->n > 0 ? s->n : 1) * sizeof(bin_entry));
    for (int64_t i = 0; i < s->n; i++)
      if (pr->cull[i] == 0) { e[bf_n].depth = pr->depth[i]; e[bf_n].id = (int32_t)i; e[bf_n].flags = 1; bf_n++; }
    qsort(e, (size_t)bf_n, sizeof(bin_entry), cmp_depth_id);
    bf_ids = (int32_t*)malloc((bf_n > 0 ? bf_n : 1) * sizeof(int32_t));
    bf_flags = (int32_t*)malloc((bf_n > 0 ? bf_n : 1) * sizeof(int32_t));
    for (int64_t k = 0; k < bf_n; k++) { bf_ids[k] = e[k].id; bf_flags[k] = 1; }
    free(e);
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t slot = 0; slot < n_tiles; slot++) {
    int32_t t = tile_list[slot];
    int tyi = t / tx, txi = t % tx;
    const int32_t* lid = brute_force ? bf_ids : &ids[tile_start[t]];
    const int32_t* lfl = brute_force ? bf_flags : &flags[tile_start[t]];
    int64_t L = brute_force ? bf_n : tile_start[t + 1] - tile_start[t];
    perturb cand[MAXCAND];
    for (int ly = 0; ly < ts; ly++)
      for (int lx = 0; lx < ts; lx++) {
        int64_t pix = (int64_t)slot * ts * ts + ly * ts + lx;
        int px = txi * ts + lx, py = tyi * ts + ly;
        pix_result r = {{p->bg[0], p->bg[1], p->bg[2]}, 1.0, 0, 0};
        int ncand = 0, nalt = 0;
        int inside = px < c->width && py < c->height;
        double o[3], d[3], pm = INFINITY;
        const double clipv = clip && px < c->width && py < c->height ? clip[(int64_t)py * c->width + px]
                                                                     : INFINITY;
        if (inside) {
          inside = pixel_ray_ctx(&CX, px + 0.5, py + 0.5, o, d, &pm);
          if (inside)
            render_pixel(&X, lid, lfl, L, o, d, clipv, (perturb){PT_NONE, 0}, &r, cand, &ncand);
        }
        out->inside[pix] = inside;
        for (int ch = 0; ch < 3; ch++) out->rgb[3 * pix + ch] = r.rgb[ch];
        out->T[pix] = r.T;
        out->n_contrib[pix] = r.nc;
        out->n_eval[pix] = r.ne;
        if (!out->n_alt) continue;
        int namb = ncand;
        /* Alternatives: the image-circle decision, then each undecided decision flipped alone. */
        if (px < c->width && py < c->height && fabs(pm) < amb->pixel) {
          namb++;
          pix_result a = {{p->bg[0], p->bg[1], p->bg[2]}, 1.0, 0, 0};
          if (!inside) render_pixel(&X, lid, lfl, L, o, d, clipv, (perturb){PT_NONE, 0}, &a, NULL, NULL);
          int64_t k = pix * ORA_MAXALT + nalt;
          for (int ch = 0; ch < 3; ch++) out->alt_rgb[3 * k + ch] = a.rgb[ch];
          out->alt_T[k] = a.T; out->alt_nc[k] = a.nc; out->alt_ne[k] = a.ne;
          nalt++;
        }
        for (int q = 0; q < ncand && inside; q++) {
          pix_result a;
          render_pixel(&X, lid, lfl, L, o, d, clipv, cand[q], &a, NULL, NULL);
          double diff = fabs(a.T - r.T);
          for (int ch = 0; ch < 3; ch++) diff = fmax(diff, fabs(a.rgb[ch] - r.rgb[ch]));
          int same_int = a.nc == r.nc && a.ne == r.ne;
          if (diff <= amb->diff && same_int) continue;
          if (nalt >= ORA_MAXALT) { namb += 1000; continue; } /* flag overflow */
          int64_t k = pix * ORA_MAXALT + nalt;
          for (int ch = 0; ch < 3; ch++) out->alt_rgb[3 * k + ch] = a.rgb[ch];
          out->alt_T[k] = a.T; out->alt_nc[k] = a.nc; out->alt_ne[k] = a.ne;
          nalt++;
        }
        out->n_alt[pix] = nalt;
        if (out->n_amb) out->n_amb[pix] = namb;
      }
  }
  free(geo);
  free(bf_ids);
  free(bf_flags);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Backward (Supp. B)                                                         */
/* ------------------------------------------------------------------------- */

typedef struct { int32_t id; double a, Tb, om2; int clamped; double og[3], dg[3]; } contrib_rec;

/* Per-particle chain from dL/d(mu, M, sigma, rgb) to the activated
 * parameters: M = S^-1 R^T gives dL/ds and dL/dR; R(q/|q|) gives dL/dq; the
 * colour's SH evaluation gives dL/dbeta and dL/dmu through the direction. */
static void finish_particle(const ora_scene* s, const ora_proj* pr, const camctx* CX,
                            int64_t i, const double gM[9], const double grgb[3],
                            double* g_means, double* g_scales, double* g_quats, double* g_sh) {
  const int K = (s->sh_degree + 1) * (s->sh_degree + 1);
  double R[9];
  const double* q = &s->quats[4 * i];
  const double* sc = &s->scales[3 * i];
  ora_quat_to_rot(q, R);
  double gR[9] = {0};
  for (int k = 0; k < 3; k++) {
    double acc = 0;
    for (int j = 0; j < 3; j++) {
      acc += gM[3 * k + j] * (-R[3 * j + k] / (sc[k] * sc[k])); /* dM_kj/ds_k */
      gR[3 * j + k] += gM[3 * k + j] / sc[k];                  /* dM_kj/dR_jk */
    }
    g_scales[3 * i + k] += acc;
  }
  double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
  const double* G = gR;
  double gq[4];
  gq[0] = 2 * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
  gq[1] = 2 * (y * G[1] + z * G[2] + y * G[3] - 2 * x * G[4] - w * G[5] + z * G[6] + w * G[7] - 2 * x * G[8]);
  gq[2] = 2 * (-2 * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] - 2 * y * G[8]);
  gq[3] = 2 * (-2 * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2 * z * G[4] + y * G[5] + x * G[6] + y * G[7]);
  double qh[4] = {w, x, y, z}, pd = 0;
  for (int k = 0; k < 4; k++) pd += qh[k] * gq[k];
  for (int k = 0; k < 4; k++) g_quats[4 * i + k] += (gq[k] - qh[k] * pd) / qn;

  /* colour: rgb = max(0, 1/2 + sum beta Y(d)), d = (mu - o*)/|mu - o*| */
  double Rwc[9], cen[3], dv[3];
  pose_ctx(CX, pr->tstar[i], Rwc, cen);
  for (int j = 0; j < 3; j++) dv[j] = s->means[3 * i + j] - cen[j];
  double dist = sqrt(dot3(dv, dv));
  for (int j = 0; j < 3; j++) dv[j] /= dist;
  double Y[16], dY[48], gd[3] = {0, 0, 0};
  ora_sh_basis(s->sh_degree, dv, Y);
  ora_sh_basis_grad(s->sh_degree, dv, dY);
  for (int ch = 0; ch < 3; ch++) {
    if (!(pr->rgb_raw[3 * i + ch] > 0)) continue;
    for (int k = 0; k < K; k++) {
      g_sh[((int64_t)K * i + k) * 3 + ch] += grgb[ch] * Y[k];
      for (int j = 0; j < 3; j++) gd[j] += grgb[ch] * s->sh[((int64_t)K * i + k) * 3 + ch] * dY[3 * k + j];
    }
  }
  double pdd = dot3(gd, dv);
  for (int j = 0; j < 3; j++) g_means[3 * i + j] += (gd[j] - dv[j] * pdd) / dist;
}

/* The k-buffer's blend sequence of one pixel (Sec. 4.3, as in
 * render_pixel_kbuffer): the contributors in the order they are blended, each
 * with the transmittance before it.  Returns their number (at most L). */
typedef struct { contrib_rec r; double dist; } kbuf_item;
static int64_t kbuffer_sequence(const ora_params* p, const particle_geo* geo, const int32_t* lid,
                                const int32_t* lfl, int64_t L, const double o[3], const double d[3],
                                double clipv, contrib_rec* rec) {
  const int k = p->kbuffer < ORA_MAXK ? p->kbuffer : ORA_MAXK;
  kbuf_item buf[ORA_MAXK];
  int n = 0;
  int64_t m = 0;
  double T = 1.0;
  int stopped = 0;
  /* Eq. 5 for one hit: appended with T before it, unless it would take T below t_min */
#define KB_BLEND(it)                                              \
  do {                                                            \
    const double Tn_ = T * (1.0 - (it).r.a);                      \
    if (Tn_ < p->t_min) { stopped = 1; break; }                   \
    rec[m] = (it).r;                                              \
    rec[m].Tb = T;                                                \
    m++;                                                          \
    T = Tn_;                                                      \
  } while (0)
  for (int64_t pos = 0; pos < L && !stopped; pos++) {
    if (!(lfl[pos] & 1)) continue;
    const particle_geo* g = &geo[lid[pos]];
    kbuf_item h;
    double odot, om2;
    eval_geo(g, o, d, h.r.og, h.r.dg, &odot, &om2);
    if (odot >= 0) continue;
    h.dist = hit_distance(odot, h.r.dg, d);
    if (h.dist > clipv) continue;
    double a = g->sigma * response(p, om2);
    h.r.clamped = a > p->alpha_max;
    if (h.r.clamped) a = p->alpha_max;
    if (a < p->alpha_min) continue;
    h.r.id = lid[pos];
    h.r.a = a;
    h.r.om2 = om2;
    if (n == k) {
      if (!(buf[0].dist < h.dist)) { KB_BLEND(h); continue; }
      KB_BLEND(buf[0]);
      if (stopped) continue;
      for (int j = 1; j < n; j++) buf[j - 1] = buf[j];
      n--;
    }
    int at = 0;
    while (at < n && buf[at].dist < h.dist) at++;
    for (int j = n; j > at; j--) buf[j] = buf[j - 1];
    buf[at] = h;
    n++;
  }
  for (int j = 0; j < n && !stopped; j++) KB_BLEND(buf[j]);
#undef KB_BLEND
  return m;
}

int ora_backward(const ora_scene* s, const ora_proj* pr, const ora_camera* c, const ora_params* p,
                 const int64_t* tile_start, const int32_t* ids, const int32_t* flags,
                 const double* clip, const double* dL_drgb, const double* dL_dT, double* g_means,
                 double* g_scales, double* g_quats, double* g_opac, double* g_sh) {
  const int tx = tiles_x(c, p), ty = tiles_y(c, p), ts = p->tile;
  const int K = (s->sh_degree + 1) * (s->sh_degree + 1);
  const int64_t n = s->n;
  particle_geo* geo = build_geo(s, pr);
  camctx CX;
  camctx_init(&CX, c);
  double* gM = (double*)calloc((size_t)(n > 0 ? n : 1) * 9, sizeof(double));
  double* grgb = (double*)calloc((size_t)(n > 0 ? n : 1) * 3, sizeof(double));
  memset(g_means, 0, n * 3 * sizeof(double));
  memset(g_scales, 0, n * 3 * sizeof(double));
  memset(g_quats, 0, n * 4 * sizeof(double));
  memset(g_opac, 0, n * sizeof(double));
  memset(g_sh, 0, n * K * 3 * sizeof(double));
#pragma omp parallel
  {
    int64_t cap = 1024;
    contrib_rec* rec = (contrib_rec*)malloc(cap * sizeof(contrib_rec));
#pragma omp for schedule(dynamic, 1)
    for (int64_t t = 0; t < (int64_t)tx * ty; t++) {
      int tyi = (int)(t / tx), txi = (int)(t % tx);
      int64_t L = tile_start[t + 1] - tile_start[t];
      const int32_t* lid = &ids[tile_start[t]];
      const int32_t* lfl = &flags[tile_start[t]];
      if (L > cap) { cap = L; rec = (contrib_rec*)realloc(rec, cap * sizeof(contrib_rec)); }
      for (int ly = 0; ly < ts; ly++)
        for (int lx = 0; lx < ts; lx++) {
          int px = txi * ts + lx, py = tyi * ts + ly;
          if (px >= c->width || py >= c->height) continue;
          int64_t pix = (int64_t)py * c->width + px;
          const double* gC = &dL_drgb[3 * pix];
          double gT = dL_dT ? dL_dT[pix] : 0.0;
          /* a pixel whose loss weights are all zero contributes nothing */
          if (gC[0] == 0.0 && gC[1] == 0.0 && gC[2] == 0.0 && gT == 0.0) continue;
          double o[3], d[3], pm;
          if (!pixel_ray_ctx(&CX, px + 0.5, py + 0.5, o, d, &pm)) continue;
          /* forward pass, keeping each contributor (Eq. 5) in blend order */
          double T = 1.0;
          int m = 0;
          if (p->kbuffer > 0) {
            m = (int)kbuffer_sequence(p, geo, lid, lfl, L, o, d, clip ? clip[pix] : INFINITY, rec);
            if (m > 0) T = rec[m - 1].Tb * (1.0 - rec[m - 1].a);
          }
          for (int64_t pos = 0; pos < L && p->kbuffer <= 0; pos++) {
            if (!(lfl[pos] & 1)) continue;
            const particle_geo* g = &geo[lid[pos]];
            double og[3], dg[3], odot, om2;
            eval_geo(g, o, d, og, dg, &odot, &om2);
            if (odot >= 0) continue;
            if (clip && hit_distance(odot, dg, d) > clip[pix]) continue;
            double a = g->sigma * response(p, om2);
            int clamped = a > p->alpha_max;
            if (clamped) a = p->alpha_max;
            if (a < p->alpha_min) continue;
            double Tn = T * (1.0 - a);
            if (Tn < p->t_min) break;
            contrib_rec* r = &rec[m++];
            r->id = lid[pos]; r->a = a; r->Tb = T; r->om2 = om2; r->clamped = clamped;
            memcpy(r->og, og, sizeof(og));
            memcpy(r->dg, dg, sizeof(dg));
            T = Tn;
          }
          const double TN = T;
          /* backward sweep: S_after accumulates sum_{j>i} c_j alpha_j T_j */
          double Sa[3] = {0, 0, 0};
          for (int k = m - 1; k >= 0; k--) {
            contrib_rec* r = &rec[k];
            const double* col = &pr->rgb[3 * r->id];
            double gA = 0;
            for (int ch = 0; ch < 3; ch++) {
              gA += gC[ch] * (col[ch] * r->Tb - (Sa[ch] + TN * p->bg[ch]) / (1.0 - r->a));
#pragma omp atomic
              grgb[3 * r->id + ch] += r->a * r->Tb * gC[ch];
            }
            gA -= gT * TN / (1.0 - r->a);
            for (int ch = 0; ch < 3; ch++) Sa[ch] += col[ch] * r->a * r->Tb;
            if (r->clamped) continue; /* alpha = alpha_max: no dependence (reading R14) */
            const particle_geo* g = &geo[r->id];
            double e = response(p, r->om2);
#pragma omp atomic
            g_opac[r->id] += gA * e;
            /* d alpha / d omega^2 = sigma d rho / d omega^2 (-1/2 sigma e^{-omega^2/2}
             * for the Gaussian, Supp. B) */
            double gom2 = gA * g->sigma * response_dw2(p, r->om2);
            /* d omega^2 / d o_g = 2 o_g + 2 tau_g d_g/|d_g| ; d omega^2 / d d_g = 2 tau (o_g + tau d_g) */
            double dd = dot3(r->dg, r->dg);
            double tau = -dot3(r->og, r->dg) / dd;
            double pv[3], gog[3], gdg[3];
            for (int j = 0; j < 3; j++) pv[j] = r->og[j] + tau * r->dg[j];
            for (int j = 0; j < 3; j++) { gog[j] = gom2 * 2 * pv[j]; gdg[j] = gom2 * 2 * tau * pv[j]; }
            /* d o_g / d mu = -S^-1 R^T */
            double gmu[3];
            matTvec(g->M, gog, gmu);
            double rel[3] = {o[0] - g->mu[0], o[1] - g->mu[1], o[2] - g->mu[2]};
            for (int j = 0; j < 3; j++) {
#pragma omp atomic
              g_means[3 * r->id + j] -= gmu[j];
            }
            for (int a_ = 0; a_ < 3; a_++)
              for (int b_ = 0; b_ < 3; b_++) {
                double v = gog[a_] * rel[b_] + gdg[a_] * d[b_];
#pragma omp atomic
                gM[9 * (int64_t)r->id + 3 * a_ + b_] += v;
              }
          }
        }
    }
    free(rec);
  }
  for (int64_t i = 0; i < n; i++) {
    if (pr->cull[i] == 1) continue;
    finish_particle(s, pr, &CX, i, &gM[9 * i], &grgb[3 * i], g_means, g_scales, g_quats, g_sh);
  }
  free(gM);
  free(grgb);
  free(geo);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Frozen-decision loss for finite differences (reading R21)                  */
/* ------------------------------------------------------------------------- */

int64_t ora_record(const ora_scene* s, const ora_proj* pr, const ora_camera* c, const ora_params* p,
                   const int64_t* tile_start, const int32_t* ids, const int32_t* flags,
                   const double* clip, int64_t* pix_start, int32_t* contrib, int32_t* clamped) {
  const int tx = tiles_x(c, p), ts = p->tile;
  particle_geo* geo = build_geo(s, pr);
  camctx CX;
  camctx_init(&CX, c);
  const int64_t npx = (int64_t)c->width * c->height;
  int64_t total = 0, cap = 0;
  contrib_rec* rec = NULL;
  for (int64_t pix = 0; pix < npx; pix++) {
    int px = (int)(pix % c->width), py = (int)(pix / c->width);
    int64_t t = (int64_t)(py / ts) * tx + px / ts;
    double o[3], d[3], pm;
    if (contrib) pix_start[pix] = total;
    if (!pixel_ray_ctx(&CX, px + 0.5, py + 0.5, o, d, &pm)) continue;
    if (p->kbuffer > 0) {  /* the contributors in blend order */
      const int64_t L = tile_start[t + 1] - tile_start[t];
      if (L > cap) { cap = L; rec = (contrib_rec*)realloc(rec, (size_t)cap * sizeof(contrib_rec)); }
      const int64_t m = kbuffer_sequence(p, geo, &ids[tile_start[t]], &flags[tile_start[t]], L, o, d,
                                         clip ? clip[pix] : INFINITY, rec);
      for (int64_t j = 0; j < m; j++, total++)
        if (contrib) { contrib[total] = rec[j].id; clamped[total] = rec[j].clamped; }
      continue;
    }
    double T = 1.0;
    for (int64_t pos = tile_start[t]; pos < tile_start[t + 1]; pos++) {
      if (!(flags[pos] & 1)) continue;
      const particle_geo* g = &geo[ids[pos]];
      double og[3], dg[3], odot, om2;
      eval_geo(g, o, d, og, dg, &odot, &om2);
      if (odot >= 0) continue;
      if (clip && hit_distance(odot, dg, d) > clip[pix]) continue;
      double a = g->sigma * response(p, om2);
      int cl = a > p->alpha_max;
      if (cl) a = p->alpha_max;
      if (a < p->alpha_min) continue;
      double Tn = T * (1.0 - a);
      if (Tn < p->t_min) break;
      if (contrib) { contrib[total] = ids[pos]; clamped[total] = cl; }
      total++;
      T = Tn;
    }
  }
  if (contrib) pix_start[npx] = total;
  free(rec);
  free(geo);
  return total;
}

double ora_loss_frozen(const ora_scene* s, const ora_proj* pr, const ora_camera* c,
                       const ora_params* p, const int64_t* pix_start, const int32_t* contrib,
                       const int32_t* clamped, const double* wC, const double* wT) {
  const int K = (s->sh_degree + 1) * (s->sh_degree + 1);
  const int64_t npx = (int64_t)c->width * c->height;
  double* rgb = (double*)malloc((size_t)(s->n > 0 ? s->n : 1) * 3 * sizeof(double));
  particle_geo* geo = (particle_geo*)malloc((size_t)(s->n > 0 ? s->n : 1) * sizeof(particle_geo));
  camctx CX;
  camctx_init(&CX, c);
  for (int64_t i = 0; i < s->n; i++) {
    make_geo(s, i, &geo[i]);
    double Rwc[9], cen[3], dv[3], raw[3];
    pose_ctx(&CX, pr->tstar[i], Rwc, cen);
    for (int j = 0; j < 3; j++) dv[j] = s->means[3 * i + j] - cen[j];
    double dist = sqrt(dot3(dv, dv));
    for (int j = 0; j < 3; j++) dv[j] /= dist;
    sh_color(s->sh_degree, &s->sh[(int64_t)3 * K * i], dv, raw);
    for (int j = 0; j < 3; j++) rgb[3 * i + j] = pr->rgb_raw[3 * i + j] > 0 ? raw[j] : 0.0;
  }
  double L = 0;
  for (int64_t pix = 0; pix < npx; pix++) {
    int px = (int)(pix % c->width), py = (int)(pix / c->width);
    double o[3], d[3], pm;
    double T = 1.0, C[3] = {0, 0, 0};
    if (pixel_ray_ctx(&CX, px + 0.5, py + 0.5, o, d, &pm)) {
      for (int64_t k = pix_start[pix]; k < pix_start[pix + 1]; k++) {
        const particle_geo* g = &geo[contrib[k]];
        double og[3], dg[3], odot, om2;
        eval_geo(g, o, d, og, dg, &odot, &om2);
        double a = clamped[k] ? p->alpha_max : g->sigma * response(p, om2);
        for (int ch = 0; ch < 3; ch++) C[ch] += a * T * rgb[3 * contrib[k] + ch];
        T *= (1.0 - a);
      }
    } else {
      continue;
    }
    for (int ch = 0; ch < 3; ch++) L += wC[3 * pix + ch] * (C[ch] + T * p->bg[ch]);
    if (wT) L += wT[pix] * T;
  }
  free(rgb);
  free(geo);
  return L;
}
