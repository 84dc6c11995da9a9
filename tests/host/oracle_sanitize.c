/* Drives every entry point of the FP64 oracle on small scenes so that a
 * build under AddressSanitizer and UndefinedBehaviorSanitizer checks its
 * memory accesses and arithmetic (tests/test_serve_core_host.py builds and
 * runs it).  Not a parity test: the values are only checked to be finite.
 * Inputs come from a small linear congruential generator. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static unsigned long long g_state = 88172645463325252ull;
static double urand(void) { /* [0, 1) */
  g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}
static double nrand(void) { /* approximately normal: sum of uniforms */
  double s = 0;
  for (int i = 0; i < 12; i++) s += urand();
  return s - 6.0;
}

#define FAIL(...) do { fprintf(stderr, __VA_ARGS__); fprintf(stderr, "\n"); exit(1); } while (0)

static void finite_or_die(const double* v, int64_t m, const char* what) {
  for (int64_t i = 0; i < m; i++)
    if (!isfinite(v[i])) FAIL("%s[%lld] is not finite", what, (long long)i);
}

static void camera(ora_camera* c, int model, int rolling, int w, int h) {
  memset(c, 0, sizeof(*c));
  c->model = model;
  c->shutter = rolling ? ORA_ROLLING : ORA_GLOBAL;
  c->width = w;
  c->height = h;
  c->fx = c->fy = model == ORA_PINHOLE ? 0.9 * w : w / 3.14159265358979;
  c->cx = 0.5 * w;
  c->cy = 0.5 * h;
  if (model == ORA_FISHEYE) { c->k[0] = 0.03; c->k[1] = -0.02; c->k[2] = 0.01; c->k[3] = -0.004; }
  double ca = cos(0.1), sa = sin(0.1);
  double I[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, Ry[9] = {ca, 0, sa, 0, 1, 0, -sa, 0, ca};
  memcpy(c->R0, I, sizeof(I));
  memcpy(c->R1, rolling ? Ry : I, sizeof(I));
  c->t0[2] = 3.0;
  c->t1[0] = rolling ? 0.3 : 0.0;
  c->t1[2] = 3.0;
}

static void params(ora_params* p, int degree, int kbuf) {
  memset(p, 0, sizeof(*p));
  p->ut_alpha = 1; p->ut_beta = 2; p->ut_kappa = 0;
  p->alpha_min = 1.0 / 255; p->alpha_max = 0.99; p->t_min = 1e-4; p->near_plane = 0.2;
  p->k_sigma_max = 3; p->tile = 16; p->rs_iters = 3;
  p->kernel_degree = degree;
  p->kbuffer = kbuf;
  p->tile_cull = degree == 2;  /* both tile rules */
}

static void run(const ora_camera* c, const ora_params* p, int n, int deg, int use_clip) {
  const int K = (deg + 1) * (deg + 1);
  double* mu = malloc(sizeof(double) * 3 * n);
  double* sc = malloc(sizeof(double) * 3 * n);
  double* q = malloc(sizeof(double) * 4 * n);
  double* op = malloc(sizeof(double) * n);
  double* sh = malloc(sizeof(double) * 3 * K * n);
  for (int i = 0; i < n; i++) {
    for (int j = 0; j < 3; j++) { mu[3 * i + j] = 2 * urand() - 1; sc[3 * i + j] = exp(-2.5 + 0.5 * nrand()); }
    for (int j = 0; j < 4; j++) q[4 * i + j] = nrand();
    op[i] = 1 / (1 + exp(-nrand()));
    for (int k = 0; k < 3 * K; k++) sh[3 * K * i + k] = k < 3 ? 2 * urand() - 1 : 0.05 * nrand();
  }
  ora_scene s = {n, deg, mu, sc, q, op, sh};
  ora_proj pr;
  pr.cull = malloc(sizeof(int32_t) * n);
  pr.mean2d = malloc(sizeof(double) * 2 * n);
  pr.cov2d = malloc(sizeof(double) * 3 * n);
  pr.rect = malloc(sizeof(int32_t) * 4 * n);
  pr.tiles = malloc(sizeof(int32_t) * n);
  pr.depth = malloc(sizeof(double) * n);
  pr.rgb = malloc(sizeof(double) * 3 * n);
  pr.rgb_raw = malloc(sizeof(double) * 3 * n);
  pr.tstar = malloc(sizeof(double) * n);
  pr.edge = malloc(sizeof(double) * 4 * n);
  pr.valid_margin = malloc(sizeof(double) * n);
  pr.kext = malloc(sizeof(double) * n);
  if (ora_project(&s, c, p, &pr) != 0) FAIL("ora_project failed");
  ora_amb amb = {1e-6, 1e-4, 1e-5, 1e-6, 2e-3, 1e-5, 1e-9, 1e-7, 1e-5, 1e-5, 1e-6};
  const int tx = (c->width + 15) / 16, ty = (c->height + 15) / 16, T = tx * ty;
  int64_t* ts = malloc(sizeof(int64_t) * (T + 1));
  int64_t P = ora_bin(n, &pr, c, p, &amb, ts, NULL, NULL);
  int32_t* ids = malloc(sizeof(int32_t) * (P > 0 ? P : 1));
  int32_t* fl = malloc(sizeof(int32_t) * (P > 0 ? P : 1));
  if (ora_bin(n, &pr, c, p, &amb, ts, ids, fl) != P) FAIL("ora_bin count changed");
  const int H = c->height, W = c->width, np = T * 256;
  double* clip = NULL;
  if (use_clip) {
    clip = malloc(sizeof(double) * H * W);
    for (int k = 0; k < H * W; k++) clip[k] = k % 10 == 0 ? INFINITY : 2.0 + 2.0 * urand();
  }
  int32_t* tl = malloc(sizeof(int32_t) * T);
  for (int t = 0; t < T; t++) tl[t] = t;
  ora_image im;
  im.rgb = malloc(sizeof(double) * 3 * np);
  im.T = malloc(sizeof(double) * np);
  im.n_contrib = malloc(sizeof(int32_t) * np);
  im.n_eval = malloc(sizeof(int32_t) * np);
  im.inside = malloc(sizeof(int32_t) * np);
  im.n_alt = malloc(sizeof(int32_t) * np);
  im.alt_rgb = malloc(sizeof(double) * 3 * ORA_MAXALT * np);
  im.alt_T = malloc(sizeof(double) * ORA_MAXALT * np);
  im.alt_nc = malloc(sizeof(int32_t) * ORA_MAXALT * np);
  im.alt_ne = malloc(sizeof(int32_t) * ORA_MAXALT * np);
  im.n_amb = malloc(sizeof(int32_t) * np);
  for (int bf = 0; bf < 2; bf++) {
    if (ora_render(&s, &pr, c, p, &amb, ts, ids, fl, tl, T, bf, clip, &im) != 0) FAIL("ora_render failed");
    finite_or_die(im.rgb, 3 * (int64_t)np, "rgb");
    finite_or_die(im.T, np, "T");
  }
  double* wC = malloc(sizeof(double) * 3 * H * W);
  double* wT = malloc(sizeof(double) * H * W);
  for (int k = 0; k < 3 * H * W; k++) wC[k] = nrand();
  for (int k = 0; k < H * W; k++) wT[k] = nrand();
  double* g = calloc((size_t)n * (3 + 3 + 4 + 1 + 3 * K), sizeof(double));
  if (ora_backward(&s, &pr, c, p, ts, ids, fl, clip, wC, wT, g, g + 3 * n, g + 6 * n, g + 10 * n,
                   g + 11 * n) != 0)
    FAIL("ora_backward failed");
  finite_or_die(g, (int64_t)n * (11 + 3 * K), "gradients");
  int64_t* ps = malloc(sizeof(int64_t) * (H * W + 1));
  int64_t m = ora_record(&s, &pr, c, p, ts, ids, fl, clip, ps, NULL, NULL);
  int32_t* con = malloc(sizeof(int32_t) * (m > 0 ? m : 1));
  int32_t* cl = malloc(sizeof(int32_t) * (m > 0 ? m : 1));
  if (ora_record(&s, &pr, c, p, ts, ids, fl, clip, ps, con, cl) != m) FAIL("ora_record count changed");
  double L = ora_loss_frozen(&s, &pr, c, p, ps, con, cl, wC, wT);
  if (!isfinite(L)) FAIL("frozen loss not finite");
  /* primitives */
  double v[2], mg, t, o[3], d[3], lam, wm[7], wc[7], A[6] = {1, 0.2, 0.1, 0, 1, -0.3}, b[2] = {1, 2};
  double m2[2], c2[3], R[9], Rw[9], cen[3], Y[16], dY[48], tau, om2, ar;
  ora_ut_weights(1, 2, 0, &lam, wm, wc);
  ora_ut_affine(mu, q, sc, p, A, b, m2, c2);
  ora_quat_to_rot(q, R);
  ora_pose(c, 0.5, Rw, cen);
  (void)ora_project_point(c, p, 0.3, mu, v, &mg);
  (void)ora_solve_time(c, p, 3, mu, &t, v, &mg);
  (void)ora_pixel_ray(c, 0.5 * W, 0.5 * H, o, d, &mg);
  ora_sh_basis(3, d, Y);
  ora_sh_basis_grad(3, d, dY);
  (void)ora_particle_alpha(mu, q, sc, op[0], o, d, p->kernel_degree, &tau, &om2, &ar);
  (void)ora_ewa(c, p, 0.0, mu, q, sc, 1e-6, m2, c2);
  const double em[2] = {3.0, -2.0}, eA[3] = {40.0, 25.0, 20.0};
  (void)ora_ellipse_box_qmin(em, eA, 0, 0, 16, 16);
  double xs[30];
  double vs[20];
  int32_t ok[10];
  for (int k = 0; k < 30; k++) xs[k] = nrand();
  ora_project_samples(c, p, 20, 10, xs, vs, ok);
  (void)ora_theta_lim(c->k);
  free(mu); free(sc); free(q); free(op); free(sh);
  free(pr.cull); free(pr.mean2d); free(pr.cov2d); free(pr.rect); free(pr.tiles); free(pr.depth);
  free(pr.rgb); free(pr.rgb_raw); free(pr.tstar); free(pr.edge); free(pr.valid_margin);
  free(pr.kext);
  free(ts); free(ids); free(fl); free(clip); free(tl);
  free(im.rgb); free(im.T); free(im.n_contrib); free(im.n_eval); free(im.inside); free(im.n_alt);
  free(im.alt_rgb); free(im.alt_T); free(im.alt_nc); free(im.alt_ne); free(im.n_amb);
  free(wC); free(wT); free(g); free(ps); free(con); free(cl);
}

int main(void) {
  ora_camera c;
  ora_params p;
  int cases = 0;
  for (int model = 0; model < 2; model++)
    for (int rolling = 0; rolling < 2; rolling++)
      for (int variant = 0; variant < 3; variant++) {
        camera(&c, model, rolling, 72 + 7 * variant, 40 + 5 * variant);
        params(&p, variant == 1 ? 4 : 2, variant == 2 ? 4 : 0);
        run(&c, &p, 120, variant == 0 ? 0 : 3, variant != 0);
        cases++;
      }
  printf("oracle sanitize ok (%d cases)\n", cases);
  return 0;
}
