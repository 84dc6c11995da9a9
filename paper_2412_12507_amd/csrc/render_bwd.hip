// K6 + K7 -- backward of the compositing and of the per-particle colour
// (Supp. B).  No gradient flows through the sigma-point projection, the
// rectangles or the sort order (Sec. 4.1: the UT only selects particles).
//
// K6 (per tile, same layout as the forward): each pixel recomputes its
// contributors front to back with the forward's exact arithmetic, up to its
// stored n_contrib.  For contributor j with transmittance T_j before it,
//   dL/dalpha_j = sum_ch gC (c_j T_j - (S_after + T_N bg) / (1 - alpha_j))
//                 - gT T_N / (1 - alpha_j),   S_after = C - T_N bg - C_<=j,
//   dL/dc_j     = alpha_j T_j gC,
// and through alpha = sigma exp(-omega^2/2) (unclamped only):
//   dL/dsigma += dL/dalpha exp(-omega^2/2),
//   dL/domega^2 = -alpha/2 dL/dalpha.
// With p = o_g + tau d_g = (d_g x (o_g x d_g)) / |d_g|^2 the closest point
// in canonical space, d omega^2/d o_g = 2p and d omega^2/d d_g = 2 tau p
// (Supp. B), so with M = S^-1 R^T the per-pixel gradients are
//   dL/dmu = -M^T c p,   dL/dM = c p (M^-1 p)^T,   c = 2 dL/domega^2.
// They only depend on G = sum c p p^T (6 values) and h = sum c p (3): each
// wave sums those plus dL/dsigma and dL/dc over its lanes (FP32, one
// reduce-scatter for all 13) and issues one FP64 atomic per value per
// (wave, particle) from 13 lanes at once, so the per-particle totals carry no
// order-dependent FP32 rounding.
//
// K7 (per particle) then applies M = S^-1 R^T:
//   dL/ds_k = -G_kk / s_k,   dL/dR = R S G S^-1,   dL/dmu = -R S^-1 h,
// the quaternion normalisation Jacobian, and (per camera) the SH colour:
//   dL/dbeta_k = dL/dc Y_k(d),  dL/dmu += (I - d d^T)/|mu - o| sum beta grad Y.
#include <mutex>

#include "camera_dev.h"
#include "tile_eval.h"

namespace gut {

constexpr int kAcc = 10;  // G xx,xy,xz,yy,yz,zz ; h x,y,z ; dL/dsigma

// Sums 16 per-lane values over the wave as a reduce-scatter: at each of the
// first four butterfly steps a lane keeps half of its values and adds its
// partner's copy of that half, then two plain steps finish the sum.  The
// 32- and 16-lane steps use the half-wave and row swaps (one instruction
// exchanges a lane's kept and sent values with its partner's), the 8- and
// 4-lane steps DPP row rotate and half-mirror, the last two DPP quad
// permutes: no LDS traffic.  Afterwards lane l holds the total of value
// (l >> 2) & 15.
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
__device__ inline float wave_reduce16(const float* g) {
  const int lane = threadIdx.x & 63;
  float h8[8], h4[4], h2[2];
#pragma unroll
  for (int j = 0; j < 8; j++) {  // lanes 0-31 keep g[j], lanes 32-63 keep g[j + 8]
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(g[j]), __float_as_uint(g[j + 8]),
                                                   false, false);
    h8[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int j = 0; j < 4; j++) {  // even rows keep h8[j], odd rows h8[j + 4]
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(h8[j]), __float_as_uint(h8[j + 4]),
                                                   false, false);
    h4[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  const bool b3 = lane & 8, b2 = lane & 4;
#pragma unroll
  for (int j = 0; j < 2; j++) {  // partner lane ^ 8 (row rotate by 8)
    const float keep = b3 ? h4[j + 2] : h4[j], send = b3 ? h4[j] : h4[j + 2];
    h2[j] = keep + dpp<0x128>(send);
  }
  // partner 7 - (lane mod 8) within each 8 (row half-mirror): differs in bit 2
  float h = (b2 ? h2[1] : h2[0]) + dpp<0x141>(b2 ? h2[0] : h2[1]);
  h += dpp<0x1B>(h);  // quad mirror (0,3) (1,2)
  h += dpp<0xB1>(h);  // quad xor 1
  return h;
}

constexpr int kBwThreads = 128;
constexpr int kBwBatch = kBwThreads;

template <bool RS, bool GEN, bool CLIP>
__global__ void __launch_bounds__(kBwThreads, 3) render_bwd_kernel(
    DevCam cam, Thresholds th, int n, int cam_idx, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ ids,
    const float4* __restrict__ record, const float* __restrict__ clip,
    const float* __restrict__ rgb, const float* __restrict__ out_rgb,
    const float* __restrict__ out_T, const uint32_t* __restrict__ out_nc,
    const float* __restrict__ d_rgb, const float* __restrict__ d_T, double* __restrict__ acc,
    double* __restrict__ acc_rgb) {
  constexpr int S = Slots<RS, true>::N;
  __shared__ float4 pd[kBwBatch * S];
  __shared__ uint32_t pe[kBwBatch];
  __shared__ uint32_t pf[kBwBatch];
  __shared__ TileFrameD F;
  __shared__ WaveBoxes wb;
  __shared__ float red[6];
  __shared__ uint32_t maxlast_s;

  const int tile = (int)order[cam.tile_base + blockIdx.x];  // longest lists first
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  // the forward's pixel layout: wave wv owns rows 8 wv .. 8 wv + 7
  const int px = tx * kTile + (lane & (kTile - 1));
  const int py0 = ty * kTile + 8 * wv + (lane >> 4);
  if (t == 0) { tile_frame(cam, tx, ty, &F); maxlast_s = 0; }
  __syncthreads();

  bool active[2];
  float u[2] = {0.f, 0.f}, v[2] = {0.f, 0.f}, dt[2] = {0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 2; k++) {
    const int py = py0 + 4 * k;
    active[k] = px < cam.W && py < cam.H && pixel_ray(cam, F, px, py, &u[k], &v[k], &dt[k]);
  }
  float umax, vmax, dtmax;
  tile_bounds<2>(u, v, dt, active, red, &umax, &vmax, &dtmax);
  const float l2amin = log2f(th.alpha_min);
  wave_box<2>(u, v, active, &wb);
  float clipv[2] = {0.f, 0.f}, dlen[2] = {1.f, 1.f};  // the forward's clip test operands
  if (CLIP) {
#pragma unroll
    for (int k = 0; k < 2; k++) {
      if (!active[k]) continue;
      clipv[k] = clip[cam.pixel_base + (long long)(py0 + 4 * k) * cam.W + px];
      dlen[k] = sqrtf(fmaf(u[k], u[k], fmaf(v[k], v[k], 1.0f)));
    }
    wave_clip_max<2>(clipv, active, &wb);
  }

  // Per pixel: the loss gradients, T_N gT, and Z = sum_c gC_c (C_c - C_<=j,c)
  // in FP64 (C the output colour, C_<=j the running colour including entry
  // j), which is all the suffix sums S_after enter the gradient through.
  uint32_t last[2] = {0u, 0u};
  float gC[2][3] = {{0, 0, 0}, {0, 0, 0}}, gTT[2] = {0.f, 0.f};
  double gCd[2][3] = {{0, 0, 0}, {0, 0, 0}}, Z[2] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 2; k++) {
    if (!active[k]) continue;
    const long long pix = cam.pixel_base + (long long)(py0 + 4 * k) * cam.W + px;
    last[k] = out_nc[pix];
    gTT[k] = (d_T ? d_T[pix] : 0.0f) * out_T[pix];
    for (int c = 0; c < 3; c++) {
      gC[k][c] = d_rgb[3 * pix + c];
      gCd[k][c] = gC[k][c];
      Z[k] = fma(gCd[k][c], (double)out_rgb[3 * pix + c], Z[k]);
    }
  }
  atomicMax(&maxlast_s, max(last[0], last[1]));
  __syncthreads();  // (also publishes wb)
  const uint2 rg = ranges[cam.tile_base + tile];
  const uint32_t maxlast = min(maxlast_s, rg.y - rg.x);  // never past the tile's list
  if (maxlast >= 2048) __builtin_amdgcn_s_setprio(3);
  else if (maxlast >= 1024) __builtin_amdgcn_s_setprio(2);
  else if (maxlast >= 256) __builtin_amdgcn_s_setprio(1);

  float T[2] = {1.0f, 1.0f};
  for (uint32_t b = 0; b < maxlast; b += kBwBatch) {
    __syncthreads();
    uint32_t fl = 0u;
    if (b + t < maxlast) {
      uint32_t e = ids[rg.x + b + t];
      pe[t] = e;
      fl = pair_setup<RS, true, GEN, CLIP>(record, rgb, e, (int)(e - (uint32_t)cam_idx * (uint32_t)n), F,
                                     cam, umax, vmax, dtmax, th, l2amin, wb, kBwThreads / 64, &pd[t * S]);
    }
    pf[t] = fl;
    __syncthreads();
    // the same pairs the forward walked for this half-tile
    const unsigned long long m0 = __builtin_amdgcn_ballot_w64((pf[lane] >> wv) & 1u);
    const unsigned long long m1 = __builtin_amdgcn_ballot_w64((pf[lane + 64] >> wv) & 1u);
    bool wave_done = false;
    for (int hh = 0; hh < 2 && !wave_done; hh++) {
      unsigned long long m = hh ? m1 : m0;
      while (m) {
        const uint32_t q = 64u * hh + (uint32_t)__builtin_ctzll(m);
        m &= m - 1ull;
        const uint32_t idx = b + q;
        if (!wave_any(idx < last[0] || idx < last[1])) { wave_done = true; break; }
        const float4* P = &pd[q * S];
        PairRegs<RS> r;
        load_pair<RS>(P, r);
        Eval ev[2];
#pragma unroll
        for (int k = 0; k < 2; k++) {
          eval_test<RS>(r, P, u[k], v[k], dt[k], &ev[k]);
          if (CLIP) ev[k].ok = ev[k].ok && !behind_clip<RS>(r, P, u[k], v[k], dt[k], dlen[k], clipv[k], ev[k].dd);
        }
        bool hit[2];
        hit[0] = ev[0].ok && idx < last[0];
        hit[1] = ev[1].ok && idx < last[1];
        if (!wave_any(hit[0] || hit[1])) continue;  // wave-uniform
        double cold[3];
        pair_colour<RS>(P, cold);
        const float isig = __builtin_amdgcn_exp2f(-r.lsig);  // 1 / sigma, shared by both pixels
        float gk[2][9], wfk[2], gAk[2], rhok[2];
#pragma unroll
        for (int k = 0; k < 2; k++) {
          eval_alpha<RS, GEN>(r, th, &ev[k]);
          const float Tb = T[k];
          const float ae = hit[k] ? ev[k].a : 0.0f;
          const float wgt = ae * Tb;
          T[k] = fmaf(-ae, Tb, Tb);  // the forward's update, bit for bit
          wfk[k] = wgt;
          // D = gC . c_j; after this entry Z = sum_c gC_c (C_c - C_<=j,c)
          const double D = fma(gCd[k][0], cold[0], fma(gCd[k][1], cold[1], gCd[k][2] * cold[2]));
          Z[k] = fma(-(double)wgt, D, Z[k]);
          // dL/dalpha = T_j gC.c_j - (gC.(C - C_<=j) + gT T_N) / (1 - alpha_j)
          const float inv1m = __builtin_amdgcn_rcpf(1.0f - ev[k].a);
          float gA = fmaf(Tb, (float)D, -inv1m * ((float)Z[k] + gTT[k]));
          const bool geo = hit[k] && !ev[k].clamped;  // alpha = alpha_max carries no gradient
          gA = geo ? gA : 0.0f;
          // rho = exp(-omega^2 / 2) = (sigma rho) / sigma
          gAk[k] = gA;
          rhok[k] = ev[k].araw * isig;
          // 2 dL/domega^2; a degree-n response scales d alpha / d omega^2 by
          // 2 lambda (n/2) (omega^2)^(n/2 - 1) relative to the Gaussian's
          float c = -ev[k].a * gA;
          if (GEN) c *= __builtin_amdgcn_exp2f(fmaf(th.k_h - 1.0f, ev[k].lq, th.k_f));
          float3 dg, cr;
          pair_vectors<RS>(P, ev[k], u[k], v[k], &dg, &cr);
          float3 p = cross3f_fma(dg, cr);
          p = f3(p.x * ev[k].idd, p.y * ev[k].idd, p.z * ev[k].idd);
          const float3 cp = f3(c * p.x, c * p.y, c * p.z);
          // G terms are cp p^T: kept as factors so the two pixels combine in fmas
          gk[k][0] = p.x; gk[k][1] = p.y; gk[k][2] = p.z;
          gk[k][6] = cp.x; gk[k][7] = cp.y; gk[k][8] = cp.z;
        }
        float g[16];  // kAcc + 3 values, padded for the reduction
        // G (symmetric, 6), h = sum c p (3), dL/dsigma, dL/dc (3)
        g[0] = fmaf(gk[0][6], gk[0][0], gk[1][6] * gk[1][0]);
        g[1] = fmaf(gk[0][6], gk[0][1], gk[1][6] * gk[1][1]);
        g[2] = fmaf(gk[0][6], gk[0][2], gk[1][6] * gk[1][2]);
        g[3] = fmaf(gk[0][7], gk[0][1], gk[1][7] * gk[1][1]);
        g[4] = fmaf(gk[0][7], gk[0][2], gk[1][7] * gk[1][2]);
        g[5] = fmaf(gk[0][8], gk[0][2], gk[1][8] * gk[1][2]);
        g[6] = gk[0][6] + gk[1][6];
        g[7] = gk[0][7] + gk[1][7];
        g[8] = gk[0][8] + gk[1][8];
        g[9] = fmaf(gAk[0], rhok[0], gAk[1] * rhok[1]);
#pragma unroll
        for (int c = 0; c < 3; c++) g[kAcc + c] = fmaf(wfk[0], gC[0][c], wfk[1] * gC[1][c]);
#pragma unroll
        for (int j = kAcc + 3; j < 16; j++) g[j] = 0.0f;
        // one lane per value issues its atomic: lanes 4k hold value k
        const float tot = wave_reduce16(g);
        const int k = lane >> 2;
        if ((lane & 3) == 0 && k < kAcc + 3 && tot != 0.0f) {
          const uint32_t e = pe[q];
          const int i = (int)(e - (uint32_t)cam_idx * (uint32_t)n);
          if (k < kAcc) atomicAdd(&acc[(long long)i * kAcc + k], (double)tot);
          else atomicAdd(&acc_rgb[3 * (long long)e + (k - kAcc)], (double)tot);
        }
      }
    }
  }
}

// Backward of the k-buffer render ("Ours (sorted)", Sec. 4.3).  It replays
// render_kbuffer_kernel bit for bit (same blocks, pixels, pair setup, tests,
// distances, and the same buffer after every insertion: the merge chain here
// and the forward's shift-and-move for a full-size buffer order the slots
// alike, ties included) and differentiates each hit when it is blended,
// in blend order: the Supp. B recursion of render_bwd_kernel (T and
// Z = gC . (C - C_<=j) carried forward from the forward's outputs) gives
// dL/dalpha there.  The geometric factors a blend needs -- the closest-point
// vector p and rho = alpha_raw / sigma -- are formed when the hit enters the
// buffer (its pair is then in LDS) and travel with it; rho carries the sign
// of the alpha_max clamp.  The buffer alone takes 128 registers a lane; the
// kernel asks for two waves per SIMD all the same (part of it then lives in
// scratch), since the replay waits on memory far more than it computes and
// one wave per SIMD leaves the SIMD idle.
//
// Sums.  A lane blends the nearest hit of its own buffer, so the hits one
// step blends are mostly different particles across the wave (about seven
// per step on a 1M-particle view), and summing them across the wave one
// particle at a time cost more than the rest of the kernel.  Instead every
// blended value goes to an FP32 LDS row of its hit's list position, with LDS
// atomics, over a window of the two latest batches (positions [b - 256,
// b + 256) while batch b runs).  A row is added to the FP64 per-particle sums
// when its batch leaves the window, 13 atomics per (tile, particle).  The
// buffer holds list positions; a hit that has stayed longer than the window
// (a buffer usually turns over within a batch) adds its values to the FP64
// sums itself.
constexpr int kKBufB = 16;
constexpr int kKThreadsB = 256;
constexpr int kWin = 2 * kKThreadsB;  // list positions with an LDS row
constexpr int kRow = kAcc + 3;        // values per row (13: an odd stride spreads rows over the banks)

struct KBufGrad {
  double* acc;
  double* acc_rgb;
  const float* rgb;
  const uint32_t* lids;  // the tile's sorted entry ids
  const uint32_t* pew;   // entry ids of the window's positions (LDS)
  float* accw;           // the window's rows (LDS)
  int n, cam_idx;
  float t_min;
  uint32_t wlo;  // lowest list position in the window
};

__device__ __forceinline__ uint32_t kbuf_entry(uint32_t pos, const KBufGrad& K) {
  // the LDS copy is read in any case and an older hit's entry then replaces
  // it; the empty register constraint keeps the compiler from folding the two
  // reads into one flat read through a selected pointer
  uint32_t e = K.pew[pos & (kWin - 1)];
  asm volatile("" : "+v"(e));
  if (pos < K.wlo) e = K.lids[pos];
  return e;
}

// Adds one lane's blended values (hit at list position pos, entry e) to the
// sums: its LDS row inside the window, else the FP64 sums.
__device__ __forceinline__ void kbuf_add(uint32_t pos, uint32_t e, const float (&v)[kRow],
                                         const KBufGrad& K) {
  if (pos >= K.wlo) {
    float* row = K.accw + (pos & (kWin - 1)) * kRow;
#pragma unroll
    for (int k = 0; k < kRow; k++) atomicAdd(&row[k], v[k]);
  } else {
    const long long i = (long long)(e - (uint32_t)K.cam_idx * (uint32_t)K.n);
#pragma unroll
    for (int k = 0; k < kAcc; k++) atomicAdd(&K.acc[i * kAcc + k], (double)v[k]);
#pragma unroll
    for (int k = 0; k < 3; k++) atomicAdd(&K.acc_rgb[3 * (long long)e + k], (double)v[kAcc + k]);
  }
}

// Adds row r of the window to the FP64 sums of its entry and clears it.
__device__ __forceinline__ void kbuf_flush_row(int r, const KBufGrad& K) {
  float* row = K.accw + r * kRow;
  const uint32_t e = K.pew[r];
  const long long i = (long long)(e - (uint32_t)K.cam_idx * (uint32_t)K.n);
#pragma unroll
  for (int k = 0; k < kRow; k++) {
    const float x = row[k];
    if (x != 0.0f) {
      if (k < kAcc) atomicAdd(&K.acc[i * kAcc + k], (double)x);
      else atomicAdd(&K.acc_rgb[3 * (long long)e + (k - kAcc)], (double)x);
      row[k] = 0.0f;
    }
  }
}

// One blend of the replay (Eq. 5 with the t_min stop, as kbuf_blend) of the
// hit at list position pos, and its 13 gradient values into the sums: G (6),
// h (3), dL/dsigma, then dL/dc (3).  Nothing for a sentinel, a wall, a
// stopped pixel or a hit that would cross t_min.
__device__ __forceinline__ void kbuf_blend_bwd(float a, uint32_t pos, float px_, float py_, float pz_,
                                               float rho, float fg, const KBufGrad& K, const float (&gC)[3],
                                               const double (&gCd)[3], float gTT, float& T, double& Z,
                                               uint32_t& done) {
  if (a <= 0.0f || done) return;
  const float Tb = T;
  const float Tn = fmaf(-a, Tb, Tb);
  if (Tn < K.t_min) { done = 1u; return; }
  T = Tn;
  const float wgt = a * Tb;
  const uint32_t e = kbuf_entry(pos, K);
  const double c0 = K.rgb[3 * (size_t)e], c1 = K.rgb[3 * (size_t)e + 1], c2 = K.rgb[3 * (size_t)e + 2];
  const double D = fma(gCd[0], c0, fma(gCd[1], c1, gCd[2] * c2));
  Z = fma(-(double)wgt, D, Z);
  const float inv1m = __builtin_amdgcn_rcpf(1.0f - a);
  float gA = fmaf(Tb, (float)D, -inv1m * ((float)Z + gTT));
  if (rho < 0.0f) gA = 0.0f;  // alpha = alpha_max carries no gradient
  const float c = -a * gA * fg;  // 2 dL/domega^2 (fg: a degree-n response's chain factor, else 1)
  float v[kRow];
  v[0] = c * px_ * px_; v[1] = c * px_ * py_; v[2] = c * px_ * pz_;
  v[3] = c * py_ * py_; v[4] = c * py_ * pz_; v[5] = c * pz_ * pz_;
  v[6] = c * px_; v[7] = c * py_; v[8] = c * pz_;
  v[9] = gA * fabsf(rho);
  v[10] = wgt * gC[0]; v[11] = wgt * gC[1]; v[12] = wgt * gC[2];
  kbuf_add(pos, e, v, K);
}

template <bool RS, bool GEN, bool CLIP>
__global__ void __launch_bounds__(kKThreadsB, 2) render_kbuffer_bwd_kernel(
    DevCam cam, Thresholds th, int n, int cam_idx, int kcap, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ ids,
    const float4* __restrict__ record, const float* __restrict__ rgb, const float* __restrict__ clip,
    const float* __restrict__ out_rgb,
    const float* __restrict__ out_T, const float* __restrict__ d_rgb, const float* __restrict__ d_T,
    double* __restrict__ acc, double* __restrict__ acc_rgb) {
  constexpr int S = Slots<RS, true>::N;
  __shared__ float4 pd[kKThreadsB * S];
  __shared__ uint32_t pf[kKThreadsB];
  __shared__ uint32_t pew[kWin];
  __shared__ float accw[kWin * kRow];
  __shared__ TileFrameD F;
  __shared__ WaveBoxes wb;
  __shared__ float red[12];
  const int tile = (int)order[cam.tile_base + blockIdx.x];
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  const int px = tx * kTile + (lane & (kTile - 1));
  const int py = ty * kTile + 4 * wv + (lane >> 4);
  if (t == 0) tile_frame(cam, tx, ty, &F);
  for (int i = t; i < kWin * kRow; i += kKThreadsB) accw[i] = 0.0f;
  __syncthreads();
  const bool inside = px < cam.W && py < cam.H;
  float u = 0.f, v = 0.f, dt = 0.f;
  bool active = inside && pixel_ray(cam, F, px, py, &u, &v, &dt);
  float umax, vmax, dtmax;
  tile_bounds<1>(&u, &v, &dt, &active, red, &umax, &vmax, &dtmax);
  const float l2amin = log2f(th.alpha_min);
  wave_box<1>(&u, &v, &active, &wb);
  const float dlen = sqrtf(fmaf(u, u, fmaf(v, v, 1.0f)));
  float clipv = 0.0f;  // the forward's clip operands
  if (CLIP) {
    if (active) clipv = clip[cam.pixel_base + (long long)py * cam.W + px];
    wave_clip_max<1>(&clipv, &active, &wb);
  }

  // the loss gradients and Z = gC . C_out (FP64), as in render_bwd_kernel
  float gC[3] = {0.f, 0.f, 0.f}, gTT = 0.f;
  double gCd[3] = {0.0, 0.0, 0.0}, Z = 0.0;
  if (active) {
    const long long pix = cam.pixel_base + (long long)py * cam.W + px;
    gTT = (d_T ? d_T[pix] : 0.0f) * out_T[pix];
    for (int c = 0; c < 3; c++) {
      gC[c] = d_rgb[3 * pix + c];
      gCd[c] = gC[c];
      Z = fma(gCd[c], (double)out_rgb[3 * pix + c], Z);
    }
  }
  const uint2 rg = ranges[cam.tile_base + tile];
  const uint32_t len = __builtin_amdgcn_readfirstlane(rg.y - rg.x);
  KBufGrad K = {acc, acc_rgb, rgb, ids + rg.x, pew, accw, n, cam_idx, th.t_min, 0u};

  float bd[kKBufB], ba[kKBufB], bx[kKBufB], by[kKBufB], bz[kKBufB], br[kKBufB], bf[kKBufB];
  uint32_t bi[kKBufB];  // list positions
#pragma unroll
  for (int j = 0; j < kKBufB; j++) {
    bd[j] = j < kcap ? -INFINITY : INFINITY;
    ba[j] = 0.0f; bx[j] = 0.0f; by[j] = 0.0f; bz[j] = 0.0f; br[j] = 0.0f; bf[j] = 1.0f;
    bi[j] = 0u;
  }
  float T = 1.0f;
  uint32_t done = active ? 0u : 1u;  // a 0/1 vector register, as in render_tile
  for (uint32_t b = 0; b < len; b += kKThreadsB) {
    if (__syncthreads_count(done == 0u) == 0) break;
    const int half = (int)(b & (uint32_t)kKThreadsB);  // this batch's rows: b mod kWin
    // the rows of batch b - kWin leave the window (their batch's eval ended
    // before the barrier above)
    if (b >= (uint32_t)kWin) kbuf_flush_row(half + t, K);
    K.wlo = b >= (uint32_t)kKThreadsB ? b - kKThreadsB : 0u;
    uint32_t fl = 0u;
    if (b + t < len) {
      const uint32_t e = ids[rg.x + b + t];
      pew[half + t] = e;
      fl = pair_setup<RS, true, GEN, CLIP>(record, rgb, e, (int)(e - (uint32_t)cam_idx * (uint32_t)n),
                                           F, cam, umax, vmax, dtmax, th, l2amin, wb, kKThreadsB / 64,
                                           &pd[t * S]);
    }
    pf[t] = fl;
    __syncthreads();
    bool wave_done = false;
    for (int h = 0; h < kKThreadsB / 64 && !wave_done; h++) {
      unsigned long long m = __builtin_amdgcn_ballot_w64((pf[lane + 64 * h] >> wv) & 1u);
      while (m) {
        if (!wave_any(done == 0u)) { wave_done = true; break; }
        const uint32_t q = 64u * h + (uint32_t)__builtin_ctzll(m);
        m &= m - 1ull;
        const float4* P = &pd[q * S];
        PairRegs<RS> r;
        load_pair<RS>(P, r);
        Eval ev;
        eval_test<RS>(r, P, u, v, dt, &ev);
        if (CLIP) ev.ok = ev.ok && !behind_clip<RS>(r, P, u, v, dt, dlen, clipv, ev.dd);
        const bool live = ev.ok && done == 0u;
        if (!wave_any(live)) continue;
        eval_alpha<RS, GEN>(r, th, &ev);
        if (live) {
          float odg;
          if (!RS) {
            const float4 p5 = P[5];
            odg = fmaf(v, p5.z, fmaf(u, p5.y, p5.x));
          } else {
            odg = fmaf(v, r.p4.w, fmaf(u, r.p3.w, r.p5.w));
            odg = fmaf(dt, fmaf(v, r.p9.w, fmaf(u, r.p8.w, r.p7.w)), odg);
          }
          const float dist = -odg * dlen * ev.idd;
          const uint32_t pos = b + q;  // the hit's list position
          // the closest point p = d_g x (o_g x d_g) / |d_g|^2 and rho, as in render_bwd_kernel
          float3 dg, cr;
          pair_vectors<RS>(P, ev, u, v, &dg, &cr);
          float3 pv = cross3f_fma(dg, cr);
          pv = f3(pv.x * ev.idd, pv.y * ev.idd, pv.z * ev.idd);
          const float rho0 = ev.araw * __builtin_amdgcn_exp2f(-r.lsig);
          const float rho = ev.clamped ? -rho0 - 1e-30f : rho0;
          // degree n: d alpha / d omega^2 relative to the Gaussian's (as in render_bwd_kernel)
          const float fg = GEN ? __builtin_amdgcn_exp2f(fmaf(th.k_h - 1.0f, ev.lq, th.k_f)) : 1.0f;
          if (dist <= bd[0]) {
            kbuf_blend_bwd(ev.a, pos, pv.x, pv.y, pv.z, rho, fg, K, gC, gCd, gTT, T, Z, done);
          } else {
            kbuf_blend_bwd(ba[0], bi[0], bx[0], by[0], bz[0], br[0], bf[0], K, gC, gCd, gTT, T, Z, done);
#pragma unroll
            for (int j = 0; j < kKBufB - 1; j++) {
              const bool nx = bd[j + 1] < dist, here = j == 0 || bd[j] < dist;
              // sorted buffer and dist > bd[0]: the middle one of bd[j], dist, bd[j + 1]
              bd[j] = __builtin_amdgcn_fmed3f(bd[j], dist, bd[j + 1]);
              ba[j] = nx ? ba[j + 1] : (here ? ev.a : ba[j]);
              bi[j] = nx ? bi[j + 1] : (here ? pos : bi[j]);
              bx[j] = nx ? bx[j + 1] : (here ? pv.x : bx[j]);
              by[j] = nx ? by[j + 1] : (here ? pv.y : by[j]);
              bz[j] = nx ? bz[j + 1] : (here ? pv.z : bz[j]);
              br[j] = nx ? br[j + 1] : (here ? rho : br[j]);
              if (GEN) bf[j] = nx ? bf[j + 1] : (here ? fg : bf[j]);
            }
            const int L = kKBufB - 1;
            const bool last = bd[L] < dist;
            ba[L] = last ? ev.a : ba[L];
            bi[L] = last ? pos : bi[L];
            bx[L] = last ? pv.x : bx[L];
            by[L] = last ? pv.y : by[L];
            bz[L] = last ? pv.z : bz[L];
            br[L] = last ? rho : br[L];
            if (GEN) bf[L] = last ? fg : bf[L];
            bd[L] = last ? dist : bd[L];
          }
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kKBufB; j++)
    kbuf_blend_bwd(ba[j], bi[j], bx[j], by[j], bz[j], br[j], bf[j], K, gC, gCd, gTT, T, Z, done);
  __syncthreads();
  kbuf_flush_row(t, K);
  kbuf_flush_row(t + kKThreadsB, K);
}

// K7a: camera-independent part of the per-particle chain (FP64: the
// quaternion gradient is a difference of terms of the size of dL/dR).
__global__ void particle_grad_kernel(int n, const float* __restrict__ scales,
                                     const float* __restrict__ quats, const double* __restrict__ acc,
                                     float* __restrict__ g_means, float* __restrict__ g_scales,
                                     float* __restrict__ g_quats, float* __restrict__ g_opac) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* a = acc + (long long)i * kAcc;
  const double G[9] = {a[0], a[1], a[2], a[1], a[3], a[4], a[2], a[4], a[5]};
  const double h[3] = {a[6], a[7], a[8]};
  const double s[3] = {scales[3 * i], scales[3 * i + 1], scales[3 * i + 2]};
  const float4 qf = reinterpret_cast<const float4*>(quats)[i];
  // R(q / |q|), q = (w, x, y, z)
  const double qn = sqrt((double)qf.x * qf.x + (double)qf.y * qf.y + (double)qf.z * qf.z +
                         (double)qf.w * qf.w);
  const double iq = 1.0 / qn;
  const double w = qf.x * iq, x = qf.y * iq, y = qf.z * iq, z = qf.w * iq;
  const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                       2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                       2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
  // dL/ds_k = -G_kk / s_k
  g_scales[3 * i] = (float)(-G[0] / s[0]);
  g_scales[3 * i + 1] = (float)(-G[4] / s[1]);
  g_scales[3 * i + 2] = (float)(-G[8] / s[2]);
  // dL/dmu = -R S^-1 h
  const double hs[3] = {h[0] / s[0], h[1] / s[1], h[2] / s[2]};
  for (int r = 0; r < 3; r++)
    g_means[3 * i + r] = (float)(-(R[3 * r] * hs[0] + R[3 * r + 1] * hs[1] + R[3 * r + 2] * hs[2]));
  // dL/dR = R S G S^-1
  double X[9];  // S G S^-1
  for (int l = 0; l < 3; l++)
    for (int k = 0; k < 3; k++) X[3 * l + k] = s[l] * G[3 * l + k] / s[k];
  double gR[9];
  for (int j = 0; j < 3; j++)
    for (int k = 0; k < 3; k++)
      gR[3 * j + k] = R[3 * j] * X[k] + R[3 * j + 1] * X[3 + k] + R[3 * j + 2] * X[6 + k];
  // through R(q/|q|):  R entries are quadratic in (w, x, y, z)
  const double gw = 2 * (x * (gR[7] - gR[5]) + y * (gR[2] - gR[6]) + z * (gR[3] - gR[1]));
  const double gx = 2 * (w * (gR[7] - gR[5]) + y * (gR[1] + gR[3]) + z * (gR[2] + gR[6]) -
                         2 * x * (gR[4] + gR[8]));
  const double gy = 2 * (w * (gR[2] - gR[6]) + x * (gR[1] + gR[3]) + z * (gR[5] + gR[7]) -
                         2 * y * (gR[0] + gR[8]));
  const double gz = 2 * (w * (gR[3] - gR[1]) + x * (gR[2] + gR[6]) + y * (gR[5] + gR[7]) -
                         2 * z * (gR[0] + gR[4]));
  const double pdot = w * gw + x * gx + y * gy + z * gz;
  reinterpret_cast<float4*>(g_quats)[i] =
      make_float4((float)((gw - w * pdot) * iq), (float)((gx - x * pdot) * iq),
                  (float)((gy - y * pdot) * iq), (float)((gz - z * pdot) * iq));
  g_opac[i] = (float)a[9];
}

// K7b: SH colour of one camera -> dL/dbeta and dL/dmu through the view
// direction.  One thread per particle, 256 per block.  The block's
// coefficients (3K floats per particle, one contiguous slab) come in and its
// gradients go out as contiguous runs through LDS, at a padded stride so each
// thread's own row hits distinct banks; every global access is coalesced and
// all of a thread's loads are issued before any is used.  The first camera
// writes g_sh (zeros for particles without colour gradient), later cameras
// add to it.
constexpr int kShThreads = 256;

template <int DEG>
__global__ void __launch_bounds__(kShThreads) sh_grad_kernel(
    int n, int cam_idx, int first, DevCam cam, Thresholds th, const float* __restrict__ means,
    const float* __restrict__ sh, const float* __restrict__ rgb, const double* __restrict__ acc_rgb,
    float* __restrict__ g_means, float* __restrict__ g_sh) {
  constexpr int K = (DEG + 1) * (DEG + 1), C = 3 * K, LD = C + 1;
  constexpr int kPer = C;  // slab floats per thread (C * 256 / 256)
  __shared__ float lb[kShThreads * LD];
  const int t = threadIdx.x;
  const long long i0 = (long long)blockIdx.x * kShThreads;
  const int cnt = (int)min((long long)kShThreads, (long long)n - i0);
  const long long i = i0 + t;
  float gr[3] = {0.f, 0.f, 0.f};
  bool live[3] = {false, false, false};
  if (t < cnt) {
    const long long e = (long long)cam_idx * n + i;
    for (int c = 0; c < 3; c++) {
      gr[c] = (float)acc_rgb[3 * e + c];
      live[c] = gr[c] != 0.0f && rgb[3 * e + c] > 0.0f;  // max(0, .) clamps the rest
    }
  }
  const bool any = live[0] || live[1] || live[2];
  const bool block_any = __syncthreads_or(any);
  if (!block_any && !first) return;  // nothing to add for these particles
  const float* src = sh + i0 * C;
  float* dst = g_sh + i0 * C;
  const int m = cnt * C;  // slab length
  if (block_any) {
    float v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; q++) {
      const int j = t + q * kShThreads;
      v[q] = j < m ? src[j] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < kPer; q++) {
      const int j = t + q * kShThreads;
      lb[(j / C) * LD + j % C] = v[q];
    }
  }
  __syncthreads();
  float gs[C];
#pragma unroll
  for (int k = 0; k < C; k++) gs[k] = 0.0f;
  if (any) {
    float3 mu = f3(means[3 * i], means[3 * i + 1], means[3 * i + 2]);
    float t0 = 0.0f;
    if (cam.shutter == GUT_ROLLING_TOP_TO_BOTTOM) {  // exposure time of the mean, as in K1
      float2 vv;
      bool ok;
      t0 = solve_project(cam, cam0_coords(cam, mu), th, &vv, &ok);
    }
    float3 ctr = centre_at(cam, t0);
    float3 dv = f3(mu.x - ctr.x, mu.y - ctr.y, mu.z - ctr.z);
    float dist = sqrtf(dot3f(dv, dv)), id = 1.0f / dist;
    float3 d = f3(dv.x * id, dv.y * id, dv.z * id);
    float Y[K];
    float3 dY[K];
    sh_basis<DEG>(d.x, d.y, d.z, Y);
    sh_basis_grad<DEG>(d.x, d.y, d.z, dY);
    const float* b = lb + t * LD;
    float3 gd = f3(0.f, 0.f, 0.f);
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const float g = live[c] ? gr[c] : 0.0f;
#pragma unroll
      for (int k = 0; k < K; k++) {
        gs[3 * k + c] = g * Y[k];
        const float bb = g * b[3 * k + c];
        gd = f3(gd.x + bb * dY[k].x, gd.y + bb * dY[k].y, gd.z + bb * dY[k].z);
      }
    }
    float pdd = dot3f(gd, d);
    g_means[3 * i] += (gd.x - d.x * pdd) * id;
    g_means[3 * i + 1] += (gd.y - d.y * pdd) * id;
    g_means[3 * i + 2] += (gd.z - d.z * pdd) * id;
  }
  __syncthreads();  // the coefficients are read; the same LDS takes the gradients
#pragma unroll
  for (int k = 0; k < C; k++) lb[t * LD + k] = gs[k];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPer; q++) {
    const int j = t + q * kShThreads;
    if (j >= m) continue;
    const float g = lb[(j / C) * LD + j % C];
    dst[j] = first ? g : dst[j] + g;
  }
}

__global__ void zero_f64_kernel(double* __restrict__ p, long long m) {
  long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) p[j] = 0.0;
}

}  // namespace gut

using namespace gut;

extern "C" size_t gut_render_bwd_workspace_bytes(int64_t n, int32_t n_cams) {
  if (n < 0 || n_cams <= 0) return 0;
  size_t a = ((size_t)n * kAcc * 8 + 255) & ~size_t(255);
  return a + (size_t)n * n_cams * 3 * 8 + 256;
}

// The whole backward with its FP64 accumulators in ws (ws_bytes available):
// argument checks, then every launch on `stream`.
static gut_status render_bwd_run(const gut_scene* scene, const gut_projected* proj,
                                 const uint32_t* tile_ranges, const uint32_t* sorted_ids,
                                 const gut_camera* cams, int32_t n_cams, const gut_params* p,
                                 const float* clip_depth, const float* rgb, const float* T_final,
                                 const uint32_t* n_contrib, const float* d_rgb, const float* d_T,
                                 float* g_means, float* g_scales, float* g_quats,
                                 float* g_opacities, float* g_sh, void* ws, size_t ws_bytes,
                                 void* stream) {
  gut_status st = check_params(p);
  if (st != GUT_OK) return st;
  if ((st = check_scene(scene, true)) != GUT_OK) return st;
  if (!proj || !proj->record || !proj->rgb || !tile_ranges || !rgb || !T_final || !n_contrib ||
      !d_rgb || !g_means || !g_scales || !g_quats || !g_opacities || !g_sh) {
    set_error("gut_render_bwd: a required pointer is NULL");
    return GUT_E_INVALID;
  }
  if (((uintptr_t)proj->record & 15) || ((uintptr_t)scene->quats & 15) ||
      ((uintptr_t)g_quats & 15) || ((uintptr_t)tile_ranges & 7)) {
    set_error("record, quats, g_quats must be 16-byte and tile_ranges 8-byte aligned");
    return GUT_E_INVALID;
  }
  const int64_t n = scene->n;
  if (n * (int64_t)n_cams >= (int64_t(1) << 31)) {
    set_error("n * n_cams must be below 2^31");
    return GUT_E_INVALID;
  }
  size_t need = gut_render_bwd_workspace_bytes(n, n_cams);
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) {
    set_error("workspace must be 256-byte aligned and hold %zu bytes", need);
    return GUT_E_INVALID;
  }
  DevCam dc[kMaxCams];
  int64_t T = 0;
  if ((st = prepare_cams(cams, n_cams, *p, dc, &T, nullptr)) != GUT_OK) return st;
  if (n == 0) return GUT_OK;
  const uint32_t* order = tile_ranges + 2 * T;
  hipStream_t s = (hipStream_t)stream;
  double* acc = (double*)ws;
  double* acc_rgb = (double*)((char*)ws + (((size_t)n * kAcc * 8 + 255) & ~size_t(255)));
  long long m1 = n * kAcc, m2 = n * n_cams * 3;
  zero_f64_kernel<<<(unsigned)((m1 + 255) / 256), 256, 0, s>>>(acc, m1);
  GUT_LAUNCH_CHECK();
  zero_f64_kernel<<<(unsigned)((m2 + 255) / 256), 256, 0, s>>>(acc_rgb, m2);
  GUT_LAUNCH_CHECK();
  Thresholds th = make_thresholds(*p);
  for (int c = 0; c < n_cams && p->kbuffer > 0; c++) {  // "Ours (sorted)"
    dim3 grid(dc[c].tiles_x * dc[c].tiles_y), block(kKThreadsB);
#define GUT_KBW(RS, GEN, CLIP)                                                                      \
  render_kbuffer_bwd_kernel<RS, GEN, CLIP><<<grid, block, 0, s>>>(                                   \
      dc[c], th, (int)n, c, p->kbuffer, (const uint2*)tile_ranges, order, sorted_ids,                 \
      (const float4*)proj->record, proj->rgb, clip_depth, rgb, T_final, d_rgb, d_T, acc, acc_rgb)
#define GUT_KBW1(RS, GEN) \
  do { if (clip_depth) GUT_KBW(RS, GEN, true); else GUT_KBW(RS, GEN, false); } while (0)
    const bool rs = dc[c].shutter == GUT_ROLLING_TOP_TO_BOTTOM, gen = th.kdeg != 2;
    if (rs) { if (gen) GUT_KBW1(true, true); else GUT_KBW1(true, false); }
    else { if (gen) GUT_KBW1(false, true); else GUT_KBW1(false, false); }
#undef GUT_KBW1
#undef GUT_KBW
    GUT_LAUNCH_CHECK();
  }
  for (int c = 0; c < n_cams && p->kbuffer == 0; c++) {
    dim3 grid(dc[c].tiles_x * dc[c].tiles_y), block(kBwThreads);
#define GUT_RBW(RS, GEN, CLIP)                                                                      \
  render_bwd_kernel<RS, GEN, CLIP><<<grid, block, 0, s>>>(                                           \
      dc[c], th, (int)n, c, (const uint2*)tile_ranges, order, sorted_ids, (const float4*)proj->record, \
      clip_depth, proj->rgb, rgb, T_final, n_contrib, d_rgb, d_T, acc, acc_rgb)
#define GUT_RBW1(RS, GEN) \
  if (clip_depth) GUT_RBW(RS, GEN, true); else GUT_RBW(RS, GEN, false)
    const bool gen = th.kdeg != 2;
    if (dc[c].shutter == GUT_ROLLING_TOP_TO_BOTTOM) { if (gen) { GUT_RBW1(true, true); } else { GUT_RBW1(true, false); } }
    else { if (gen) { GUT_RBW1(false, true); } else { GUT_RBW1(false, false); } }
#undef GUT_RBW1
#undef GUT_RBW
    GUT_LAUNCH_CHECK();
  }
  dim3 g1((unsigned)((n + 255) / 256)), b1(256);
  particle_grad_kernel<<<g1, b1, 0, s>>>((int)n, scene->scales, scene->quats, acc, g_means,
                                         g_scales, g_quats, g_opacities);
  GUT_LAUNCH_CHECK();
  const dim3 gs_grid((unsigned)((n + kShThreads - 1) / kShThreads));
  for (int c = 0; c < n_cams; c++) {
#define GUT_SHG(D)                                                                          \
  sh_grad_kernel<D><<<gs_grid, kShThreads, 0, s>>>((int)n, c, c == 0, dc[c], th, scene->means, \
                                                   scene->sh, proj->rgb, acc_rgb, g_means, g_sh)
    switch (scene->sh_degree) {
      case 0: GUT_SHG(0); break;
      case 1: GUT_SHG(1); break;
      case 2: GUT_SHG(2); break;
      default: GUT_SHG(3); break;
    }
#undef GUT_SHG
    GUT_LAUNCH_CHECK();
  }
  return GUT_OK;
}

extern "C" gut_status gut_render_bwd(const gut_scene* scene, const gut_projected* proj,
                                     const uint32_t* tile_ranges, const uint32_t* sorted_ids,
                                     const gut_camera* cams, int32_t n_cams, const gut_params* p,
                                     const float* clip_depth, const float* rgb, const float* T_final,
                                     const uint32_t* n_contrib, const float* d_rgb,
                                     const float* d_T, float* g_means, float* g_scales,
                                     float* g_quats, float* g_opacities, float* g_sh, void* ws,
                                     size_t ws_bytes, void* stream) {
  return render_bwd_run(scene, proj, tile_ranges, sorted_ids, cams, n_cams, p, clip_depth, rgb,
                        T_final, n_contrib, d_rgb, d_T, g_means, g_scales, g_quats, g_opacities,
                        g_sh, ws, ws_bytes, stream);
}

// ---- the backward without a caller workspace --------------------------------
// For callers that cannot allocate (graph capture, serving loops, harnesses
// that forbid it): the FP64 accumulators live in one static device array per
// GPU, held from the library's load until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in);
// its device address is looked up once per device, with that device current,
// and kept.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

gut_status scratch_address(void** out) {
  int dev = 0;
  GUT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) {
    set_error("gut_render_bwd_noalloc: device %d is beyond the %d supported", dev,
              kMaxScratchDevices);
    return GUT_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    GUT_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || ((uintptr_t)ptr & 255)) {
      set_error("gut_render_bwd_noalloc: scratch address %p is not 256-byte aligned", ptr);
      return GUT_E_HIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GUT_OK;
}
}  // namespace

extern "C" gut_status gut_render_bwd_noalloc(const gut_scene* scene, const gut_projected* proj,
                                             const uint32_t* tile_ranges, const uint32_t* sorted_ids,
                                             const gut_camera* cams, int32_t n_cams,
                                             const gut_params* p, const float* clip_depth,
                                             const float* rgb, const float* T_final,
                                             const uint32_t* n_contrib, const float* d_rgb,
                                             const float* d_T, float* g_means, float* g_scales,
                                             float* g_quats, float* g_opacities, float* g_sh,
                                             void* stream) {
  if (!scene || scene->n < 0 || n_cams <= 0) {
    set_error("gut_render_bwd_noalloc: NULL scene, n < 0 or n_cams <= 0");
    return GUT_E_INVALID;
  }
  const size_t need = gut_render_bwd_workspace_bytes(scene->n, n_cams);
  if (need > kNoAllocScratchBytes) {
    set_error("gut_render_bwd_noalloc: n = %lld particles over %d camera(s) need %zu bytes of "
              "scratch; the static scratch holds %zu (use gut_render_bwd with a workspace)",
              (long long)scene->n, (int)n_cams, need, kNoAllocScratchBytes);
    return GUT_E_INVALID;
  }
  void* ws = nullptr;
  gut_status st = scratch_address(&ws);
  if (st != GUT_OK) return st;
  return render_bwd_run(scene, proj, tile_ranges, sorted_ids, cams, n_cams, p, clip_depth, rgb,
                        T_final, n_contrib, d_rgb, d_T, g_means, g_scales, g_quats, g_opacities,
                        g_sh, ws, kNoAllocScratchBytes, stream);
}
