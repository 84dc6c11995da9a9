// Per-tile evaluation of the 3D particle response (Eq. 11) shared by the
// forward and backward compositing kernels.
//
// Conditioning.  A particle's response along a pixel ray depends on
// omega^2 = |o_g x d_g|^2 / |d_g|^2 with o_g = S^-1 R^T (o - mu) and
// d_g = S^-1 R^T d.  For a small particle far from the camera, o_g is long
// (distance / scale, up to ~1e4) and nearly parallel to d_g, so forming the
// cross product from FP32 rays loses most of its bits.  Instead each tile gets
// an FP64 frame (origin o_T, unit anchor direction n, tangent basis e1, e2)
// and every pixel ray is written EXACTLY as a direction proportional to
// n + u e1 + v e2 (u, v small, so FP32 holds them to ~1e-10), plus, under a
// rolling shutter, an origin o_T + dt (c1 - c0).  Per (tile, particle) pair
// the kernel forms in FP64, once,
//   d_g(n), d_g(e1), d_g(e2), w = o_g x d_g(n), A = o_g x d_g(e1),
//   B = o_g x d_g(e2)   (and the dt terms m x ...,  m = S^-1 R^T (c1 - c0))
// and stores them as FP32; per pixel the cross product is the short sum
// w + u A + v B whose terms are of the size of the result, so FP32 keeps
// ~1e-6 relative accuracy for every particle.  This costs fewer FP32 ops per
// evaluation than transforming each ray into the particle frame.
//
// The same inline functions, with explicit fmaf and contraction disabled at
// compile time, are used by forward and backward so that every discrete
// decision (tau_max > 0, alpha >= alpha_min, clamping) is identical in both.
#pragma once
#include "common.h"

namespace gut {

// FP64 tile frame kept in LDS: origin, anchor direction, tangent basis, time.
struct TileFrameD {
  double o[3], n[3], e1[3], e2[3], tT;
};

__device__ inline void tile_frame(const DevCam& cam, int tx, int ty, TileFrameD* F) {
  double ua = fmin(tx * (double)kTile + 0.5 * kTile, (double)cam.W);
  double va = fmin(ty * (double)kTile + 0.5 * kTile, (double)cam.H);
  int ra = min(ty * kTile + kTile / 2, cam.H - 1);
  double tT = row_time(cam, ra);
  bool ok;
  d3 dca = unproject_dir(cam, ua, va, &ok);
  d3 o, d;
  ray_at(cam, tT, dca, &o, &d);
  d = scl(d, 1.0 / sqrt(dot(d, d)));
  d3 ref = fabs(d.x) <= fabs(d.y) && fabs(d.x) <= fabs(d.z) ? mk3(1, 0, 0)
           : (fabs(d.y) <= fabs(d.z) ? mk3(0, 1, 0) : mk3(0, 0, 1));
  d3 e1 = cross(d, ref);
  e1 = scl(e1, 1.0 / sqrt(dot(e1, e1)));
  d3 e2 = cross(d, e1);
  F->o[0] = o.x; F->o[1] = o.y; F->o[2] = o.z;
  F->n[0] = d.x; F->n[1] = d.y; F->n[2] = d.z;
  F->e1[0] = e1.x; F->e1[1] = e1.y; F->e1[2] = e1.z;
  F->e2[0] = e2.x; F->e2[1] = e2.y; F->e2[2] = e2.z;
  F->tT = tT;
}

// Pixel ray in tile coordinates: direction ~ n + u e1 + v e2, origin o_T + dt (c1 - c0).
__device__ inline bool pixel_ray(const DevCam& cam, const TileFrameD& F, int px, int py, float* u,
                                 float* v, float* dt) {
  double tr = row_time(cam, py);
  bool valid;
  d3 dc = unproject_dir(cam, px + 0.5, py + 0.5, &valid);
  d3 o, d;
  ray_at(cam, tr, dc, &o, &d);
  double dn = d.x * F.n[0] + d.y * F.n[1] + d.z * F.n[2];
  if (!(dn > 0.0)) return false;
  double idn = 1.0 / dn;
  *u = (float)((d.x * F.e1[0] + d.y * F.e1[1] + d.z * F.e1[2]) * idn);
  *v = (float)((d.x * F.e2[0] + d.y * F.e2[1] + d.z * F.e2[2]) * idn);
  *dt = (float)(tr - F.tT);
  return valid;
}

template <bool RS>
struct Slots {
  static constexpr int N = RS ? 10 : 7;
};

// Per-pair terms, FP64 -> FP32 slots:
//   0: d_g(n).xyz, sigma (negated: sign test needed per pixel; 0: never)
//   1: d_g(e1).xyz, r    2: d_g(e2).xyz, g    3: w.xyz, b
//   4: A.xyz, s          5: B.xyz, ta          6: tb, -, -, -
//   RS: 7: (m x d_g(n)).xyz, m.d_g(n)  8: (m x d_g(e1)).xyz, m.d_g(e1)
//       9: (m x d_g(e2)).xyz, m.d_g(e2)
// where s, ta, tb are o_g . d_g(.) for the tau_max > 0 test.
template <bool RS>
__device__ inline void pair_setup(const float4* __restrict__ record, const float* __restrict__ rgb,
                                  long long e, int i, const TileFrameD& F, const DevCam& cam,
                                  float umax, float vmax, float dtmax, float4* out) {
  float4 r0 = record[4 * (long long)i], r1 = record[4 * (long long)i + 1];
  float4 r2 = record[4 * (long long)i + 2], r3 = record[4 * (long long)i + 3];
  const double M[9] = {r1.x, r1.y, r1.z, r2.x, r2.y, r2.z, r3.x, r3.y, r3.z};
  d3 rel = mk3(F.o[0] - (double)r0.x, F.o[1] - (double)r0.y, F.o[2] - (double)r0.z);
  d3 og = mv(M, rel);
  d3 dn = mv(M, mk3(F.n[0], F.n[1], F.n[2]));
  d3 da = mv(M, mk3(F.e1[0], F.e1[1], F.e1[2]));
  d3 db = mv(M, mk3(F.e2[0], F.e2[1], F.e2[2]));
  d3 w = cross(og, dn), A = cross(og, da), B = cross(og, db);
  double s = dot(og, dn), ta = dot(og, da), tb = dot(og, db);
  double spread = umax * fabs(ta) + vmax * fabs(tb);
  d3 w2 = mk3(0, 0, 0), A2 = w2, B2 = w2;
  double s2 = 0, ta2 = 0, tb2 = 0;
  if (RS) {
    d3 m = mv(M, mk3(cam.dc[0], cam.dc[1], cam.dc[2]));
    w2 = cross(m, dn); A2 = cross(m, da); B2 = cross(m, db);
    s2 = dot(m, dn); ta2 = dot(m, da); tb2 = dot(m, db);
    spread += dtmax * (fabs(s2) + umax * fabs(ta2) + vmax * fabs(tb2));
  }
  float sig = r0.w;
  if (s + spread < 0.0) {
    // o_g . d_g < 0 (tau_max > 0) for every ray of the tile
  } else if (s - spread >= 0.0) {
    sig = 0.0f;  // tau_max <= 0 for every ray: never contributes
  } else {
    sig = -sig;  // mixed: decide per pixel
  }
  const float* c = rgb + 3 * e;
  out[0] = make_float4((float)dn.x, (float)dn.y, (float)dn.z, sig);
  out[1] = make_float4((float)da.x, (float)da.y, (float)da.z, c[0]);
  out[2] = make_float4((float)db.x, (float)db.y, (float)db.z, c[1]);
  out[3] = make_float4((float)w.x, (float)w.y, (float)w.z, c[2]);
  out[4] = make_float4((float)A.x, (float)A.y, (float)A.z, (float)s);
  out[5] = make_float4((float)B.x, (float)B.y, (float)B.z, (float)ta);
  out[6] = make_float4((float)tb, 0.0f, 0.0f, 0.0f);
  if (RS) {
    out[7] = make_float4((float)w2.x, (float)w2.y, (float)w2.z, (float)s2);
    out[8] = make_float4((float)A2.x, (float)A2.y, (float)A2.z, (float)ta2);
    out[9] = make_float4((float)B2.x, (float)B2.y, (float)B2.z, (float)tb2);
  }
}

struct Eval {
  float a;      // alpha after the alpha_max clamp (0 when the pair is skipped)
  float ex;     // exp(-omega^2 / 2)
  bool ok;      // tau_max > 0 and alpha >= alpha_min
  bool clamped; // sigma * ex > alpha_max
  float3 dg, cr;
  float idd;    // 1 / |d_g|^2
};

// One pair's terms, loaded from LDS once and shared by the pixels a thread owns.
template <bool RS>
struct PairRegs {
  float4 p0, p1, p2, p3, p4, p5;
  float4 p7, p8, p9;
  bool mixed;  // sign of o_g . d_g varies across the tile (wave-uniform)
};

template <bool RS>
__device__ __forceinline__ void load_pair(const float4* P, PairRegs<RS>& r) {
  r.p0 = P[0]; r.p1 = P[1]; r.p2 = P[2]; r.p3 = P[3]; r.p4 = P[4]; r.p5 = P[5];
  if (RS) { r.p7 = P[7]; r.p8 = P[8]; r.p9 = P[9]; }
  // every lane reads the same pair: move the flag to a scalar register
  r.mixed = __builtin_amdgcn_readfirstlane(__float_as_int(r.p0.w)) < 0;
}

// alpha of one pair on one pixel ray (Eq. 11 and alpha = sigma rho), with no
// divergent branches; o->ok is false if tau_max <= 0 or alpha < alpha_min.
template <bool RS>
__device__ __forceinline__ void eval_pair(const PairRegs<RS>& r, const float4* P, float u, float v,
                                          float dt, float amin, float amax, Eval* o) {
  float3 dg = f3(fmaf(v, r.p2.x, fmaf(u, r.p1.x, r.p0.x)), fmaf(v, r.p2.y, fmaf(u, r.p1.y, r.p0.y)),
                 fmaf(v, r.p2.z, fmaf(u, r.p1.z, r.p0.z)));
  float3 cr = f3(fmaf(v, r.p5.x, fmaf(u, r.p4.x, r.p3.x)), fmaf(v, r.p5.y, fmaf(u, r.p4.y, r.p3.y)),
                 fmaf(v, r.p5.z, fmaf(u, r.p4.z, r.p3.z)));
  if (RS) {
    float3 m = f3(fmaf(v, r.p9.x, fmaf(u, r.p8.x, r.p7.x)), fmaf(v, r.p9.y, fmaf(u, r.p8.y, r.p7.y)),
                  fmaf(v, r.p9.z, fmaf(u, r.p8.z, r.p7.z)));
    cr = f3(fmaf(dt, m.x, cr.x), fmaf(dt, m.y, cr.y), fmaf(dt, m.z, cr.z));
  }
  bool ok = true;
  if (r.mixed) {  // rare, and uniform across the wave
    float sg = fmaf(v, P[6].x, fmaf(u, r.p5.w, r.p4.w));
    if (RS) sg = fmaf(dt, fmaf(v, r.p9.w, fmaf(u, r.p8.w, r.p7.w)), sg);
    ok = sg < 0.0f;
  }
  const float sig = fabsf(r.p0.w);
  float dd = fmaf(dg.z, dg.z, fmaf(dg.y, dg.y, dg.x * dg.x));
  float cc = fmaf(cr.z, cr.z, fmaf(cr.y, cr.y, cr.x * cr.x));
  float idd = __builtin_amdgcn_rcpf(dd);
  // exp(-omega^2/2) = 2^(-omega^2 log2(e) / 2)
  float ex = __builtin_amdgcn_exp2f((cc * idd) * -0.72134752044448170f);
  float araw = sig * ex;
  float a = fminf(araw, amax);
  ok = ok && (a >= amin);
  o->a = ok ? a : 0.0f;
  o->ex = ex;
  o->ok = ok;
  o->clamped = araw > amax;
  o->dg = dg;
  o->cr = cr;
  o->idd = idd;
}

// Block-wide maxima of |u|, |v|, |dt| over the tile's valid pixels (NP per thread).
template <int NP>
__device__ inline void tile_bounds(const float* u, const float* v, const float* dt,
                                   const bool* valid, float* red, float* umax, float* vmax,
                                   float* dtmax) {
  float a = 0.0f, b = 0.0f, c = 0.0f;
#pragma unroll
  for (int k = 0; k < NP; k++) {
    if (valid[k]) {
      a = fmaxf(a, fabsf(u[k]));
      b = fmaxf(b, fabsf(v[k]));
      c = fmaxf(c, fabsf(dt[k]));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a = fmaxf(a, __shfl_xor(a, o, 64));
    b = fmaxf(b, __shfl_xor(b, o, 64));
    c = fmaxf(c, __shfl_xor(c, o, 64));
  }
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) { red[3 * w] = a; red[3 * w + 1] = b; red[3 * w + 2] = c; }
  __syncthreads();
  float A = 0, B = 0, Cc = 0;
  for (int k = 0; k < nw; k++) {
    A = fmaxf(A, red[3 * k]);
    B = fmaxf(B, red[3 * k + 1]);
    Cc = fmaxf(Cc, red[3 * k + 2]);
  }
  // a little slack so the FP64 sign classification covers FP32 rounding of u, v
  *umax = A * 1.0001f + 1e-7f;
  *vmax = B * 1.0001f + 1e-7f;
  *dtmax = Cc * 1.0001f + 1e-7f;
}

// Tile visited by block b: blocks are dealt round-robin to the 8 XCDs, so
// give each XCD a contiguous run of tiles (neighbouring tiles share most of
// their particles, and each XCD has its own L2).
__device__ inline int xcd_tile(int b, int n) {
  const int nx = 8;
  int x = b % nx, j = b / nx;
  int q = n / nx, r = n % nx;
  int start = x * q + min(x, r);
  return start + j;
}

}  // namespace gut
