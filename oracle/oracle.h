/*
 * oracle.h -- plain FP64 CPU reference of the 3DGUT rasterizer hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP path.
 *
 * Every function follows the paper (arXiv 2412.12507) step by step in double
 * precision, with no blocking, fusion or reordering beyond what the equations
 * state:
 *   - particle response and covariance factorisation: Eq. 1-2 (Sec. 3);
 *   - unscented transform: Eq. 6-10 and Alg. 2 (Sec. 4.1, Supp. E);
 *   - extent, rectangle, tiling: Alg. 1 (Supp. E);
 *   - volume rendering: Eq. 5 (Sec. 3);
 *   - maximum-response evaluation: Eq. 11 (Sec. 4.2);
 *   - global per-tile depth sort: Sec. 4.3;
 *   - backward pass: Supp. B.
 * Where the paper is silent the readings listed in the design notes apply and
 * are named at the point of use (camera frame and pixel centres, fisheye
 * validity limit, rolling-shutter timing, extent rule, sort depth, SH
 * direction, thresholds).
 *
 * Parity unpinned: the extent rule, the sort depth, the tie-break, the SH
 * evaluation direction and the rolling-shutter timing rule are readings the
 * paper does not fix; they are pinned only by agreement between this oracle
 * and the GPU path.
 */
#ifndef GUT_ORACLE_H
#define GUT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_PINHOLE = 0, ORA_FISHEYE = 1 };
enum { ORA_GLOBAL = 0, ORA_ROLLING = 1 };

typedef struct {
  int32_t model, shutter, width, height;
  double fx, fy, cx, cy, k[4];
  double R0[9], t0[3]; /* world->camera at exposure start, row-major */
  double R1[9], t1[3]; /* world->camera at exposure end             */
} ora_camera;

typedef struct {
  double ut_alpha, ut_beta, ut_kappa;
  double alpha_min, alpha_max, t_min, near_plane, k_sigma_max;
  int32_t tile, rs_iters;
  double bg[3];
  int32_t kernel_degree; /* n of the generalized Gaussian response (Supp. A); 2 = Gaussian */
  int32_t kbuffer;       /* 0: tile-order compositing; k > 0: per-ray k-buffer (MLAB, Sec. 4.3) */
  int32_t tile_cull;     /* 1: a rectangle tile joins a list only if the extent ellipse meets it
                            (the 3DGS / StopThePop tile culling of Sec. 4.1 and 4.4); 0: every
                            tile of the rectangle */
} ora_params;

typedef struct {
  int64_t n;
  int32_t sh_degree;
  const double *means, *scales, *quats, *opacities, *sh; /* [n,3] [n,3] [n,4] [n] [n,K,3] */
} ora_scene;

/* Per-particle projection record (Alg. 1 outputs plus bookkeeping). */
typedef struct {
  int32_t* cull;        /* [n] 0 visible, 1 opacity < alpha_min, 2 invalid sigma point, 3 empty rect */
  double* mean2d;       /* [n,2] */
  double* cov2d;        /* [n,3] xx, xy, yy */
  int32_t* rect;        /* [n,4] tile x0, y0, x1, y1 (inclusive) */
  int32_t* tiles;       /* [n] tiles touched */
  double* depth;        /* [n] */
  double* rgb;          /* [n,3] clamped at 0 */
  double* rgb_raw;      /* [n,3] before the clamp */
  double* tstar;        /* [n] exposure time of the mean point (0 for a global shutter) */
  double* edge;         /* [n,4] v_x - h_x, v_y - h_y, v_x + h_x, v_y + h_y in pixels */
  double* valid_margin; /* [n] smallest validity margin over all sigma-point projections */
  double* kext;         /* [n] the extent's cutoff k (the ellipse is (v-m)^T Sigma'^-1 (v-m) <= k^2) */
} ora_proj;

/* Ambiguity thresholds: decisions whose margin falls below these are treated
 * as undecided between FP32 and FP64 and yield alternative results. */
typedef struct {
  double alpha;  /* |alpha - alpha_min|                        */
  double trans;  /* |T'/T_min - 1|                             */
  double tau;    /* |o_g . d_g| / (|o_g| |d_g|)                 */
  double depth;  /* |d_i - d_j| / d_i for neighbours in a list */
  double edge;   /* pixels between a rectangle edge and a tile boundary */
  double valid;  /* validity margin of a sigma point          */
  double pixel;  /* fisheye image-circle margin (radians)     */
  double diff;   /* an alternative is kept only if it differs by more than this */
  double clip;   /* |hit distance - clip distance| (relative) */
  double order;  /* |distance difference| of two hits in a k-buffer (relative) */
  double conic;  /* relative rounding of the extent ellipse's matrix entries (tile culling) */
} ora_amb;

#define ORA_MAXALT 8

/* Per-pixel render outputs for a list of tiles (pixel = tile slot * tile^2 + local index). */
typedef struct {
  double* rgb;          /* [np,3] */
  double* T;            /* [np]   */
  int32_t* n_contrib;   /* [np]   list position + 1 of the last contributor */
  int32_t* n_eval;      /* [np]   list entries evaluated up to the stop */
  int32_t* inside;      /* [np]   1 if the pixel exists and has a valid ray */
  int32_t* n_alt;       /* [np]   number of alternatives kept (nullable) */
  double* alt_rgb;      /* [np,ORA_MAXALT,3] (nullable with n_alt) */
  double* alt_T;        /* [np,ORA_MAXALT]   */
  int32_t* alt_nc;      /* [np,ORA_MAXALT]   */
  int32_t* alt_ne;      /* [np,ORA_MAXALT]   */
  int32_t* n_amb;       /* [np] ambiguous decisions seen (including dropped ones) */
} ora_image;

/* ---- primitives exposed for the pins ---- */
double ora_theta_lim(const double k[4]);
void ora_ut_weights(double a, double b, double kappa, double* lambda, double wm[7], double wc[7]);
/* UT through an affine map v = A x + b (A 2x3 row-major). */
void ora_ut_affine(const double mu[3], const double quat[4], const double scale[3],
                   const ora_params* p, const double A[6], const double b[2],
                   double mean2d[2], double cov2d[3]);
void ora_quat_to_rot(const double q[4], double R[9]);
/* world->camera rotation and camera centre at exposure time t in [0,1]. */
void ora_pose(const ora_camera* c, double t, double Rwc[9], double centre[3]);
/* Project a world point at time t: returns 1 if valid; v = pixel coords. */
int ora_project_point(const ora_camera* c, const ora_params* p, double t, const double x[3],
                      double v[2], double* margin);
/* Solve the rolling-shutter exposure time of a point (Sec. 4.1, reading R7). */
int ora_solve_time(const ora_camera* c, const ora_params* p, int iters, const double x[3],
                   double* t, double v[2], double* margin);
/* Monte-Carlo reference projection (Supp. C): m world points x[m,3] through
 * the camera, each with its rolling-shutter time solved by `iters`
 * iterations; v[m,2] pixel positions, ok[m] validity. */
void ora_project_samples(const ora_camera* c, const ora_params* p, int iters, int64_t m,
                         const double* x, double* v, int32_t* ok);
/* EWA projection (Eq. 3) at exposure time t: mean and covariance J Sigma J^T
 * with J the camera's Jacobian at mu by central differences of step h.
 * Returns 0 if a projection is invalid. */
int ora_ewa(const ora_camera* c, const ora_params* p, double t, const double mu[3],
            const double quat[4], const double scale[3], double h, double mean2d[2],
            double cov2d[3]);
/* Ray of pixel centre (u, v) (row from v): returns 1 if valid. */
int ora_pixel_ray(const ora_camera* c, double u, double v, double o[3], double d[3],
                  double* margin);
void ora_sh_basis(int degree, const double dir[3], double* Y /* [(deg+1)^2] */);
void ora_sh_basis_grad(int degree, const double dir[3], double* dY /* [(deg+1)^2,3] */);
/* alpha of one particle on one ray (Eq. 11 + Eq. 5's alpha) with the response of
 * degree kernel_degree (Supp. A; 2 = Gaussian); returns 0 if tau <= 0. */
int ora_particle_alpha(const double mu[3], const double quat[4], const double scale[3],
                       double opacity, const double o[3], const double d[3], int32_t kernel_degree,
                       double* tau_max, double* omega2, double* alpha_raw);

/* Tile culling of one extent ellipse (mean m, matrix A = k^2 Sigma', xx xy yy):
 * the minimum of (v-m)^T A^-1 (v-m) over the closed box [x0,x1] x [y0,y1]
 * (0 when m lies inside); the box meets the ellipse iff it is <= 1. */
double ora_ellipse_box_qmin(const double m[2], const double A[3], double x0, double y0,
                            double x1, double y1);

/* OpenMP threads of the calls below: n > 0 sets them; returns the count in use. */
int ora_set_threads(int n);

/* ---- pipeline ---- */
int ora_project(const ora_scene* s, const ora_camera* c, const ora_params* p, ora_proj* out);
/* Tile lists sorted by (depth, id).  flags bit0: member of the primary list;
 * bit1: membership undecided (rect edge, validity or, with tile culling, the
 * ellipse test within the margin).
 * Call with ids == NULL to get the entry count. */
int64_t ora_bin(int64_t n, const ora_proj* pr, const ora_camera* c, const ora_params* p,
                const ora_amb* amb, int64_t* tile_start /* [T+1] */, int32_t* ids,
                int32_t* flags);
int ora_render(const ora_scene* s, const ora_proj* pr, const ora_camera* c,
               const ora_params* p, const ora_amb* amb, const int64_t* tile_start,
               const int32_t* ids, const int32_t* flags, const int32_t* tile_list,
               int32_t n_tiles, int32_t brute_force,
               const double* clip /* [H*W] nullable: hybrid-rendering clip distances, Sec. 6.2 */,
               ora_image* out);
/* Backward (Supp. B): gradients w.r.t. the activated parameters. */
int ora_backward(const ora_scene* s, const ora_proj* pr, const ora_camera* c,
                 const ora_params* p, const int64_t* tile_start, const int32_t* ids,
                 const int32_t* flags, const double* clip /* [H*W] nullable */,
                 const double* dL_drgb /* [H,W,3] */,
                 const double* dL_dT /* [H,W] nullable */, double* g_means, double* g_scales,
                 double* g_quats, double* g_opac, double* g_sh);
/* Frozen-decision loss for finite differences: record contributors once,
 * then evaluate L = sum wC*C + wT*T with every discrete decision held. */
int64_t ora_record(const ora_scene* s, const ora_proj* pr, const ora_camera* c,
                   const ora_params* p, const int64_t* tile_start, const int32_t* ids,
                   const int32_t* flags, const double* clip /* [H*W] nullable */,
                   int64_t* pix_start /* [H*W+1] */,
                   int32_t* contrib /* nullable for count */, int32_t* clamped);
double ora_loss_frozen(const ora_scene* s, const ora_proj* pr, const ora_camera* c,
                       const ora_params* p, const int64_t* pix_start, const int32_t* contrib,
                       const int32_t* clamped, const double* wC, const double* wT);

#ifdef __cplusplus
}
#endif
#endif
