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
  float umax, vmax, dtmax, l2amin;  // compositing: the tile's |u|, |v|, |dt| bounds and log2(alpha_min)
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
  double dn = dot(d, mk3(F.n[0], F.n[1], F.n[2]));
  if (!(dn > 0.0)) return false;
  double idn = 1.0 / dn;
  *u = (float)(dot(d, mk3(F.e1[0], F.e1[1], F.e1[2])) * idn);
  *v = (float)(dot(d, mk3(F.e2[0], F.e2[1], F.e2[2])) * idn);
  *dt = (float)(tr - F.tT);
  return valid;
}

// log2(e) / 2: omega^2 / 2 in natural units is omega^2 * kHalfLog2e in log2 units.
constexpr double kHalfLog2e = 0.72134752044448170368;

// Pair slots (float4 each) kept in LDS for one (tile, particle) pair.
//
// Global shutter.  The two quadratic forms of a pixel's (u, v) that decide
// the response are factored in FP64 (QR of the affine maps (u, v) -> vector)
// into sums of squares,
//   |o_g x d_g|^2 log2(e)/2 = (f1 + r11 u + r12 v)^2 + (f2 + r22 v)^2 + f3
//   |d_g|^2                 = (g1 + h11 u + h12 v)^2 + (g2 + h22 v)^2 + g3
// so a pixel needs 10 FMAs for both and no term cancels beyond what the
// affine maps themselves carry.
//   0: f1 r11 r12 Kp    1: f2 r22 f3 lsig    2: g1 h11 h12 mixed
//   3: g2 h22 g3 -      4: colour r g (FP64)  5: s ta tb -
//   6: colour b (FP64), -
// and, for the backward only, the vectors for the closest point p:
//   7: d_g(n).xyz w.x   8: d_g(e1).xyz w.y   9: d_g(e2).xyz w.z
//  10: A.xyz B.x       11: B.y B.z - -
// Rolling shutter.  The origin moves with the row, so the cross product is
// bilinear in (u, v) and dt and is formed from its vectors per pixel:
//   0: d_g(n).xyz mixed  1: d_g(e1).xyz lsig  2: d_g(e2).xyz Kp
//   3: w.xyz ta          4: A.xyz tb          5: B.xyz s
//   6: colour r g (FP64) 7: (m x d_g(n)).xyz m.d_g(n)
//   8: (m x d_g(e1)).xyz m.d_g(e1)               9: (m x d_g(e2)).xyz m.d_g(e2)
//  10: colour b (FP64), -
// (colours are kept in FP64 because the compositing accumulates in FP64)
// Here w = o_g x d_g(n), A = o_g x d_g(e1), B = o_g x d_g(e2),
// s, ta, tb = o_g . d_g(.) (the tau_max > 0 test, needed per pixel only when
// its sign varies over the tile: mixed = -1), lsig = log2(sigma) and
// Kp = log2(sigma / alpha_min) (-1: never contributes), so that
//   alpha = min(2^(lsig - omega'^2), alpha_max),  alpha >= alpha_min <=> omega'^2 <= Kp
// with omega'^2 = omega^2 log2(e) / 2.
// Bit of pair_setup's result set when the sign of o_g . d_g varies over the
// tile (the per-pixel tau_max > 0 test is needed); the low bits are per wave.
constexpr unsigned kMixedBit = 1u << 8;

template <bool RS, bool BWD>
struct Slots {
  static constexpr int N = RS ? 11 : (BWD ? 12 : 7);
};

// 1 / sqrt(x) for a normal x > 0: the hardware estimate (relative error
// below 2^-22) and one Newton step, ~1e-13 relative: the factorisation below
// needs ~1e-7.
__device__ __forceinline__ double rsq64(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  return fma(0.5 * r, fma(-x * r, r, 1.0), r);
}

// QR of the affine map (u, v) -> c0 + u c1 + v c2 (FP64 Gram-Schmidt; one
// pass keeps the form to ~1e-7 of the alpha_min decision scale, below the
// FP32 rounding the coefficients then take): |c0 + u c1 + v c2|^2 =
// (q[0] + q[1] u + q[2] v)^2 + (q[3] + q[4] v)^2 + q[5].
__device__ inline void affine_qr(d3 c0, d3 c1, d3 c2, double q[6]) {
  // (a norm below 1e-300 counts as zero: the estimate is not made for denormals)
  const double n11 = dot(c1, c1), i11 = n11 > 1e-300 ? rsq64(n11) : 0.0;
  const double r11 = n11 * i11;
  const d3 a1 = scl(c1, i11);
  const double r12 = dot(c2, a1);
  const d3 b = axpy(-r12, a1, c2);
  const double n22 = dot(b, b), i22 = n22 > 1e-300 ? rsq64(n22) : 0.0;
  const double r22 = n22 * i22;
  const d3 a2 = scl(b, i22);
  const double f1 = dot(c0, a1), f2 = dot(c0, a2);
  const d3 rem = axpy(-f2, a2, axpy(-f1, a1, c0));
  q[0] = f1; q[1] = r11; q[2] = r12; q[3] = f2; q[4] = r22; q[5] = dot(rem, rem);
}

// Per-wave culling.  With d_g = D x, D = [d_g(n) d_g(e1) d_g(e2)],
// x = (1, u, v), the pixels where omega^2 <= K' form {x : x^T N x <= 0} with
// N_ij = (o_g x D_i).(o_g x D_j) - K' D_i.D_j  (Lagrange's identity on
// |o_g|^2 |d_g|^2 - (o_g.d_g)^2 - K' |d_g|^2), i.e. an ellipse in (u, v)
// that is tested exactly against each wave's pixel box.  K' carries a 1e-3
// relative margin (and, under a rolling shutter, the distance the ray origin
// moves within the tile, which bounds how far the line moves), so a culled
// pair fails the per-pixel FP32 test for every pixel of the wave (that
// test's own rounding is ~1e-6 relative) and culling changes no result.
// Forward and backward cull identically.
struct WaveBoxes {
  float u0[4], u1[4], v0[4], v1[4];
  float cmax[4];  // largest clip distance of the wave's pixels (hybrid rendering)
};

// Does the ellipse qmin + [du dv] [[N11 N12] [N12 N22]] [du dv]^T <= 0
// (qmin < 0, matrix positive definite; coordinates relative to its centre)
// meet the box [a0, a1] x [b0, b1]?  The quadratic is convex, so its minimum
// over the box is at the centre if the centre is inside, else on an edge,
// where it is a 1D quadratic minimised in closed form and clamped.
__device__ inline bool ellipse_meets_box(double qmin, double N11, double N12, double N22,
                                         double iN11, double iN22, double a0, double a1,
                                         double b0, double b1) {
  if (a0 <= 0.0 && a1 >= 0.0 && b0 <= 0.0 && b1 >= 0.0) return true;
  const double slack = -1e-6 * qmin;
  // edge with one offset x fixed; the other offset y ranges over [lo, hi]
  auto edge = [&](double x, double lo, double hi, double Nxx, double Nyy, double iNyy) {
    const double y = fmin(fmax(-N12 * x * iNyy, lo), hi);
    return fma(Nyy * y, y, fma(2.0 * N12 * x, y, fma(Nxx * x, x, qmin))) <= slack;
  };
  return edge(a0, b0, b1, N11, N22, iN22) || edge(a1, b0, b1, N11, N22, iN22) ||
         edge(b0, a0, a1, N22, N11, iN11) || edge(b1, a0, a1, N22, N11, iN11);
}

// Forms a pair's slots (FP64 -> FP32) and returns one bit per wave of the
// block: bit k set when wave k's pixel box may see alpha >= alpha_min.  GEN:
// the response has degree th.kdeg > 2, and the threshold kept in Kp is the
// one on omega'^2 where the degree-n exponent reaches log2(sigma / alpha_min).
// CLIP (hybrid rendering): a wave whose largest clip distance (wb.cmax) lies
// before the particle's alpha_min ellipsoid loses its bit too -- every hit it
// could see would be clipped.
template <bool RS, bool BWD, bool GEN, bool CLIP>
__device__ inline unsigned pair_setup(const float4* __restrict__ record,
                                      const float* __restrict__ rgb, long long e, int i,
                                      const TileFrameD& F, const DevCam& cam, float umax,
                                      float vmax, float dtmax, const Thresholds& th,
                                      float log2_amin, const WaveBoxes& wb, int nwaves, float4* out) {
  const float amin = th.alpha_min;
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
  double spread = fma(umax, fabs(ta), vmax * fabs(tb));
  d3 w2 = mk3(0, 0, 0), A2 = w2, B2 = w2;
  double s2 = 0, ta2 = 0, tb2 = 0, mlen = 0;
  if (RS) {
    d3 m = mv(M, mk3(cam.dc[0], cam.dc[1], cam.dc[2]));
    w2 = cross(m, dn); A2 = cross(m, da); B2 = cross(m, db);
    s2 = dot(m, dn); ta2 = dot(m, da); tb2 = dot(m, db);
    spread = fma(dtmax, fma(umax, fabs(ta2), fma(vmax, fabs(tb2), fabs(s2))), spread);
    mlen = sqrt(dot(m, m));
  }
  const double oo = dot(og, og);
  const float sigma = r0.w;
  bool never = false, mixed = false;
  if (s + spread < 0.0) {
    // o_g . d_g < 0 (tau_max > 0) for every ray of the tile
  } else if (s - spread >= 0.0) {
    never = true;  // tau_max <= 0 for every ray
  } else {
    mixed = true;  // decide per pixel
  }
  const float lsig = log2f(sigma);
  float Kp = (!never && sigma >= amin) ? lsig - log2_amin : -1.0f;
  // degree n: 2^(k_h log2 q + k_l) <= Kp  <=>  q <= 2^((log2 Kp - k_l) / k_h)
  if (GEN && Kp > 0.0f) Kp = exp2f((log2f(Kp) - th.k_l) * th.k_inv_h);
  const float mflag = mixed ? -1.0f : 1.0f;
  // the per-pixel test uses this FP32 Kp; cull with it in natural units
  double Kc = (double)Kp / kHalfLog2e * (1.0 + 1e-3) + 1e-5;
  if (RS) {
    const double r = sqrt(Kc) + dtmax * mlen * (1.0 + 1e-6);
    Kc = r * r;
  }
  // The culling ellipse's matrix N (below).  Without a rolling shutter the
  // slots' factorised forms are made first and N is read off them, so that
  // the FP64 vectors are dead before the culling: from
  // |c0 + u c1 + v c2|^2 = (q0 + q1 u + q2 v)^2 + (q3 + q4 v)^2 + q5,
  // |c0|^2 = q0^2 + q3^2 + q5, c0.c1 = q0 q1, c0.c2 = q0 q2 + q3 q4,
  // |c1|^2 = q1^2, c1.c2 = q1 q2, |c2|^2 = q2^2 + q4^2.  qc carries the
  // factor log2(e)/2, so N comes scaled by it, which leaves the ellipse.
  double N00 = 0.0, N01 = 0.0, N02 = 0.0, N11 = 0.0, N12 = 0.0, N22 = 0.0;
  if (!RS) {
    double qc[6], qd[6];
    const double sc = sqrt(kHalfLog2e);
    affine_qr(scl(w, sc), scl(A, sc), scl(B, sc), qc);
    affine_qr(dn, da, db, qd);
    out[0] = make_float4((float)qc[0], (float)qc[1], (float)qc[2], Kp);
    out[1] = make_float4((float)qc[3], (float)qc[4], (float)qc[5], lsig);
    out[2] = make_float4((float)qd[0], (float)qd[1], (float)qd[2], mflag);
    out[3] = make_float4((float)qd[3], (float)qd[4], (float)qd[5], 0.0f);
    out[5] = make_float4((float)s, (float)ta, (float)tb, 0.0f);
    if (BWD) {
      out[7] = make_float4((float)dn.x, (float)dn.y, (float)dn.z, (float)w.x);
      out[8] = make_float4((float)da.x, (float)da.y, (float)da.z, (float)w.y);
      out[9] = make_float4((float)db.x, (float)db.y, (float)db.z, (float)w.z);
      out[10] = make_float4((float)A.x, (float)A.y, (float)A.z, (float)B.x);
      out[11] = make_float4((float)B.y, (float)B.z, 0.0f, 0.0f);
    }
    const double K2 = Kc * kHalfLog2e;
    N00 = fma(-K2, fma(qd[0], qd[0], fma(qd[3], qd[3], qd[5])), fma(qc[0], qc[0], fma(qc[3], qc[3], qc[5])));
    N01 = fma(-K2, qd[0] * qd[1], qc[0] * qc[1]);
    N02 = fma(-K2, fma(qd[0], qd[2], qd[3] * qd[4]), fma(qc[0], qc[2], qc[3] * qc[4]));
    N11 = fma(-K2, qd[1] * qd[1], qc[1] * qc[1]);
    N12 = fma(-K2, qd[1] * qd[2], qc[1] * qc[2]);
    N22 = fma(-K2, fma(qd[2], qd[2], qd[4] * qd[4]), fma(qc[2], qc[2], qc[4] * qc[4]));
  }
  unsigned flags = 0;
  if (Kp >= 0.0f) {
    const unsigned all = (1u << nwaves) - 1u;
    if (oo <= Kc) {
      flags = all;  // the ray origin is inside the particle's alpha_min ellipsoid
    } else {
      if (RS) {
        N00 = fma(-Kc, dot(dn, dn), dot(w, w));
        N01 = fma(-Kc, dot(dn, da), dot(w, A));
        N02 = fma(-Kc, dot(dn, db), dot(w, B));
        N11 = fma(-Kc, dot(da, da), dot(A, A));
        N12 = fma(-Kc, dot(da, db), dot(A, B));
        N22 = fma(-Kc, dot(db, db), dot(B, B));
      }
      const double det = fma(N11, N22, -N12 * N12);
      if (!(N11 > 0.0) || !(N22 > 0.0) || !(det > 1e-9 * N11 * N22)) {
        flags = all;  // not a well-conditioned ellipse in the tile plane: no culling
      } else {
        // 1/det, 1/N11 and 1/N22 from one division
        const double p11 = N11 * N22, rq = 1.0 / (det * p11);
        const double idet = p11 * rq;
        const double uc = fma(N02, N12, -N01 * N22) * idet, vc = fma(N01, N12, -N02 * N11) * idet;
        const double qmin = fma(N02, vc, fma(N01, uc, N00));
        if (qmin < 0.0) {
          const double iN11 = det * N22 * rq, iN22 = det * N11 * rq;
          for (int k = 0; k < nwaves; k++)
            if (ellipse_meets_box(qmin, N11, N12, N22, iN11, iN22, wb.u0[k] - uc, wb.u1[k] - uc,
                                  wb.v0[k] - vc, wb.v1[k] - vc))
              flags |= 1u << k;
        }
      }
    }
  }
  if (CLIP && flags) {
    // Any accepted hit is a point of the ellipsoid |M (x - mu)|^2 <= Kc, whose
    // world radius is at most sqrt(Kc) s_max (s_k = 1 / |row k of M|), so it
    // lies at least |o - mu| - sqrt(Kc) s_max from the ray origin o, which
    // under a rolling shutter moves up to dtmax |c1 - c0| from o_T.  The
    // per-pixel test carries ~1e-6 relative error: a 1e-4 margin keeps every
    // culled pair clipped there too.
    const double Kc0 = (double)Kp / kHalfLog2e * (1.0 + 1e-3) + 1e-5;
    double rmin = 3e300;
    for (int k = 0; k < 3; k++) rmin = fmin(rmin, M[3 * k] * M[3 * k] + M[3 * k + 1] * M[3 * k + 1] +
                                                      M[3 * k + 2] * M[3 * k + 2]);
    double lb = sqrt(dot(rel, rel)) - sqrt(Kc0 / rmin);
    if (RS) lb -= (double)dtmax * sqrt(cam.dc[0] * cam.dc[0] + cam.dc[1] * cam.dc[1] + cam.dc[2] * cam.dc[2]);
    for (int k = 0; k < nwaves; k++)
      if (lb > (double)wb.cmax[k] * (1.0 + 1e-4)) flags &= ~(1u << k);
  }
  if (mixed && flags) flags |= kMixedBit;
  const float* c = rgb + 3 * e;
  if (!RS) {
    reinterpret_cast<double2*>(out + 4)[0] = make_double2(c[0], c[1]);
    reinterpret_cast<double2*>(out + 6)[0] = make_double2(c[2], 0.0);
  } else {
    out[0] = make_float4((float)dn.x, (float)dn.y, (float)dn.z, mflag);
    out[1] = make_float4((float)da.x, (float)da.y, (float)da.z, lsig);
    out[2] = make_float4((float)db.x, (float)db.y, (float)db.z, Kp);
    out[3] = make_float4((float)w.x, (float)w.y, (float)w.z, (float)ta);
    out[4] = make_float4((float)A.x, (float)A.y, (float)A.z, (float)tb);
    out[5] = make_float4((float)B.x, (float)B.y, (float)B.z, (float)s);
    reinterpret_cast<double2*>(out + 6)[0] = make_double2(c[0], c[1]);
    out[7] = make_float4((float)w2.x, (float)w2.y, (float)w2.z, (float)s2);
    out[8] = make_float4((float)A2.x, (float)A2.y, (float)A2.z, (float)ta2);
    out[9] = make_float4((float)B2.x, (float)B2.y, (float)B2.z, (float)tb2);
    reinterpret_cast<double2*>(out + 10)[0] = make_double2(c[2], 0.0);
  }
  return flags;
}

struct Eval {
  float a;       // alpha after the alpha_max clamp (0 when the pair is skipped)
  float lq;      // degree-n responses: log2 of omega'^2
  bool ok;       // tau_max > 0 and omega^2 <= K (alpha >= alpha_min)
  bool clamped;  // sigma rho > alpha_max
  float cc;      // omega'^2 |d_g|^2 (omega'^2 = omega^2 log2(e) / 2)
  float dd;      // |d_g|^2
  float idd;     // 1 / |d_g|^2
  float araw;    // sigma rho before the alpha_max clamp
  float3 dg, cr; // rolling shutter only: d_g and o_g x d_g
};

// One pair's decision terms, loaded from LDS once and shared by the pixels a thread owns.
template <bool RS>
struct PairRegs {
  float4 p0, p1, p2, p3, p4, p5;
  float4 p7, p8, p9;
  bool mixed;  // sign of o_g . d_g varies across the tile (wave-uniform)
  float lsig, Kp;
};

template <bool RS>
__device__ __forceinline__ void load_pair(const float4* P, PairRegs<RS>& r) {
  r.p0 = P[0]; r.p1 = P[1]; r.p2 = P[2]; r.p3 = P[3];
  if (RS) {
    r.p4 = P[4]; r.p5 = P[5]; r.p7 = P[7]; r.p8 = P[8]; r.p9 = P[9];
    r.lsig = r.p1.w; r.Kp = r.p2.w;
    // every lane reads the same pair: move the flag to a scalar register
    r.mixed = __builtin_amdgcn_readfirstlane(__float_as_int(r.p0.w)) < 0;
  } else {
    r.lsig = r.p1.w; r.Kp = r.p0.w;
    r.mixed = __builtin_amdgcn_readfirstlane(__float_as_int(r.p2.w)) < 0;
  }
}

// Stage 1 of the response on one pixel ray (Eq. 11): omega'^2 |d_g|^2 and
// |d_g|^2, and the test omega'^2 <= Kp (<=> alpha >= alpha_min) without any
// transcendental.
template <bool RS>
__device__ __forceinline__ void eval_test(const PairRegs<RS>& r, const float4* P, float u, float v,
                                          float dt, Eval* o) {
  bool ok = true;
  if (!RS) {
    const float t1 = fmaf(v, r.p0.z, fmaf(u, r.p0.y, r.p0.x));
    const float t2 = fmaf(v, r.p1.y, r.p1.x);
    o->cc = fmaf(t1, t1, fmaf(t2, t2, r.p1.z));
    const float e1 = fmaf(v, r.p2.z, fmaf(u, r.p2.y, r.p2.x));
    const float e2 = fmaf(v, r.p3.y, r.p3.x);
    o->dd = fmaf(e1, e1, fmaf(e2, e2, r.p3.z));
    if (r.mixed) {  // rare, and uniform across the wave
      const float4 p5 = P[5];
      ok = fmaf(v, p5.z, fmaf(u, p5.y, p5.x)) < 0.0f;
    }
  } else {
    float3 dg = f3(fmaf(v, r.p2.x, fmaf(u, r.p1.x, r.p0.x)), fmaf(v, r.p2.y, fmaf(u, r.p1.y, r.p0.y)),
                   fmaf(v, r.p2.z, fmaf(u, r.p1.z, r.p0.z)));
    float3 cr = f3(fmaf(v, r.p5.x, fmaf(u, r.p4.x, r.p3.x)), fmaf(v, r.p5.y, fmaf(u, r.p4.y, r.p3.y)),
                   fmaf(v, r.p5.z, fmaf(u, r.p4.z, r.p3.z)));
    float3 m = f3(fmaf(v, r.p9.x, fmaf(u, r.p8.x, r.p7.x)), fmaf(v, r.p9.y, fmaf(u, r.p8.y, r.p7.y)),
                  fmaf(v, r.p9.z, fmaf(u, r.p8.z, r.p7.z)));
    cr = f3(fmaf(dt, m.x, cr.x), fmaf(dt, m.y, cr.y), fmaf(dt, m.z, cr.z));
    if (r.mixed) {
      float sg = fmaf(v, r.p4.w, fmaf(u, r.p3.w, r.p5.w));
      sg = fmaf(dt, fmaf(v, r.p9.w, fmaf(u, r.p8.w, r.p7.w)), sg);
      ok = sg < 0.0f;
    }
    o->dd = fmaf(dg.z, dg.z, fmaf(dg.y, dg.y, dg.x * dg.x));
    o->cc = fmaf(cr.z, cr.z, fmaf(cr.y, cr.y, cr.x * cr.x)) * (float)kHalfLog2e;
    o->dg = dg;
    o->cr = cr;
  }
  o->ok = ok & (o->cc <= r.Kp * o->dd);
}

// Stage 2 (only for waves where some pixel passed): alpha = min(sigma rho, alpha_max)
// with sigma rho = 2^(lsig - omega'^2), or for a degree-n response (GEN)
// 2^(lsig - x), x = 2^(k_h log2 omega'^2 + k_l).
template <bool RS, bool GEN>
__device__ __forceinline__ void eval_alpha(const PairRegs<RS>& r, const Thresholds& th, Eval* o) {
  const float amax = th.alpha_max;
  const float idd = __builtin_amdgcn_rcpf(o->dd);
  float araw;
  if (GEN) {
    o->lq = __builtin_amdgcn_logf(o->cc * idd);  // log2; -inf at the centre line
    araw = __builtin_amdgcn_exp2f(r.lsig - __builtin_amdgcn_exp2f(fmaf(th.k_h, o->lq, th.k_l)));
  } else {
    araw = __builtin_amdgcn_exp2f(fmaf(-o->cc, idd, r.lsig));
  }
  o->idd = idd;
  o->araw = araw;
  o->clamped = araw > amax;
  // araw >= 0, so med3(araw, 0, amax) = min(araw, amax) in one instruction;
  // callers use a only where ok holds (their live / hit masks include it)
  o->a = __builtin_amdgcn_fmed3f(araw, 0.0f, amax);
}

// Hybrid rendering (Sec. 6.2): does the pair's maximum-response point lie
// beyond the pixel's clip distance (its closest surface intersection)?  With
// d = n + u e1 + v e2 (|d| = dlen = sqrt(1 + u^2 + v^2)) the hit is at
// tau' = -(o_g . d_g) / |d_g|^2 along d, i.e. at distance tau' dlen, so it is
// behind when -(o_g . d_g) dlen > clip |d_g|^2.  o_g . d_g is the same affine
// (bilinear under a rolling shutter) form as the tau_max sign test.  Forward
// and backward call this with the same operands.
template <bool RS>
__device__ __forceinline__ bool behind_clip(const PairRegs<RS>& r, const float4* P, float u, float v,
                                            float dt, float dlen, float clip, float dd) {
  float odg;
  if (!RS) {
    const float4 p5 = P[5];
    odg = fmaf(v, p5.z, fmaf(u, p5.y, p5.x));
  } else {
    odg = fmaf(v, r.p4.w, fmaf(u, r.p3.w, r.p5.w));
    odg = fmaf(dt, fmaf(v, r.p9.w, fmaf(u, r.p8.w, r.p7.w)), odg);
  }
  return -odg * dlen > clip * dd;
}

// Colour of a pair (FP64 slots).
template <bool RS>
__device__ __forceinline__ void pair_colour(const float4* P, double c[3]) {
  const double2 rg = reinterpret_cast<const double2*>(P + (RS ? 6 : 4))[0];
  const double2 b = reinterpret_cast<const double2*>(P + (RS ? 10 : 6))[0];
  c[0] = rg.x;
  c[1] = rg.y;
  c[2] = b.x;
}

// Backward only: d_g and o_g x d_g on the pixel ray (unscaled), for the
// closest point p = d_g x (o_g x d_g) / |d_g|^2.
template <bool RS>
__device__ __forceinline__ void pair_vectors(const float4* P, const Eval& ev, float u, float v,
                                             float3* dg, float3* cr) {
  if (RS) {
    *dg = ev.dg;
    *cr = ev.cr;
  } else {
    const float4 q6 = P[7], q7 = P[8], q8 = P[9], q9 = P[10], q10 = P[11];
    *dg = f3(fmaf(v, q8.x, fmaf(u, q7.x, q6.x)), fmaf(v, q8.y, fmaf(u, q7.y, q6.y)),
             fmaf(v, q8.z, fmaf(u, q7.z, q6.z)));
    *cr = f3(fmaf(v, q9.w, fmaf(u, q9.x, q6.w)), fmaf(v, q10.x, fmaf(u, q9.y, q7.w)),
             fmaf(v, q10.y, fmaf(u, q9.z, q8.w)));
  }
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

// Pixel box (u, v) of each wave's pixels, written to LDS by lane 0 of each
// wave (NP pixels per thread).
template <int NP>
__device__ inline void wave_box(const float* u, const float* v, const bool* valid, WaveBoxes* wb) {
  float a0 = 3e38f, a1 = -3e38f, b0 = 3e38f, b1 = -3e38f;
#pragma unroll
  for (int k = 0; k < NP; k++)
    if (valid[k]) {
      a0 = fminf(a0, u[k]); a1 = fmaxf(a1, u[k]);
      b0 = fminf(b0, v[k]); b1 = fmaxf(b1, v[k]);
    }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a0 = fminf(a0, __shfl_xor(a0, o, 64));
    a1 = fmaxf(a1, __shfl_xor(a1, o, 64));
    b0 = fminf(b0, __shfl_xor(b0, o, 64));
    b1 = fmaxf(b1, __shfl_xor(b1, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    const int w = threadIdx.x >> 6;
    wb->u0[w] = a0; wb->u1[w] = a1; wb->v0[w] = b0; wb->v1[w] = b1;
  }
}

// Largest clip distance over each wave's valid pixels (+inf if any is
// unclipped; -inf if the wave has no valid pixel).
template <int NP>
__device__ inline void wave_clip_max(const float* clip, const bool* valid, WaveBoxes* wb) {
  float c = -INFINITY;
#pragma unroll
  for (int k = 0; k < NP; k++)
    if (valid[k]) c = fmaxf(c, clip[k]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c = fmaxf(c, __shfl_xor(c, o, 64));
  if ((threadIdx.x & 63) == 0) wb->cmax[threadIdx.x >> 6] = c;
}

// True when pred holds on some active lane (the wave's lane mask, without a
// round trip through a vector register).
__device__ __forceinline__ bool wave_any(bool pred) {
  return __builtin_amdgcn_ballot_w64(pred) != 0ull;
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
