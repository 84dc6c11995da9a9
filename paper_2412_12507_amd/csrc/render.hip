// K5 -- per-tile front-to-back compositing (Eq. 5) with each particle's
// response evaluated in 3D at its maximum along the pixel ray (Eq. 11).
//
// One 128-thread block (2 wave64s) per 16x16 tile; each wave owns a 16x8
// half-tile and each thread two pixels of one column, 4 rows apart, so every
// pair read from LDS serves two evaluations.  The tile's sorted list is
// consumed in batches of 128: each thread gathers one pair's 64-byte render
// record, forms the pair's FP64 tile-frame terms (tile_eval.h), including
// which half-tiles the particle's alpha_min ellipse can reach, and stores
// them in LDS.  Each wave then walks only the pairs flagged for its half
// (a scalar bit loop), reading each pair as an LDS broadcast; per pixel the
// cheap test omega^2 <= K comes first and the reciprocal and exponential run
// only when some lane of the wave passes it.  The walk is branch-free per
// pixel (predicated updates); a wave leaves the batch as soon as all its
// pixels have stopped, and the block stops when no pixel is still going.
// Blocks take tiles in the render order from gut_bin (longest lists first)
// and waves of long lists raise their issue priority, so the longest tiles
// neither start last nor crawl behind short ones.  The compositing kernels
// run five waves per SIMD (96 VGPRs; the FP64 pair setup keeps 12 values in
// scratch): 8% faster than four waves without spills (114 VGPRs).  The walk
// is a chain of dependent LDS reads, compares and transcendentals, and a
// fifth wave hides more of it than the setup's spills cost.
#include "tile_eval.h"

namespace gut {

constexpr int kRThreads = 128;
constexpr int kRBatch = kRThreads;

// One tile of one camera.  pd, pf, F, wb and red are the block's LDS; out_*
// are indexed by pix_base + y * W + x.  GEN: response of degree th.kdeg > 2.
// CLIP: per-pixel clip distances (hybrid rendering, Sec. 6.2), indexed as
// the outputs; hits beyond them are discarded.
template <bool RS, bool NE, bool GEN, bool CLIP>
__device__ __forceinline__ void render_tile(
    const DevCam& cam, const Thresholds& th, int n, int cam_idx, int tile,
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ ids,
    const float4* __restrict__ record, const float* __restrict__ rgb, const float* __restrict__ clip,
    float* __restrict__ out_rgb,
    float* __restrict__ out_T, uint32_t* __restrict__ out_nc, uint32_t* __restrict__ out_ne,
    long long pix_base, float4* pd, uint32_t* pf, TileFrameD& F, WaveBoxes& wb, float* red) {
  constexpr int S = Slots<RS, false>::N;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  // wave wv owns the 16 x 8 half-tile of rows 8 wv .. 8 wv + 7; a thread
  // owns the pixels (px, py0) and (px, py0 + 4)
  const int px = tx * kTile + (lane & (kTile - 1));
  const int py0 = ty * kTile + 8 * wv + (lane >> 4);
  if (t == 0) tile_frame(cam, tx, ty, &F);
  __syncthreads();

  bool inside[2], active[2];
  float u[2] = {0.f, 0.f}, v[2] = {0.f, 0.f}, dt[2] = {0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 2; k++) {
    const int py = py0 + 4 * k;
    inside[k] = px < cam.W && py < cam.H;
    active[k] = inside[k] && pixel_ray(cam, F, px, py, &u[k], &v[k], &dt[k]);
  }
  float umax, vmax, dtmax;
  tile_bounds<2>(u, v, dt, active, red, &umax, &vmax, &dtmax);
  // The pair setup reads the tile's bounds from LDS at each batch (published
  // by the batch's first barrier): kept in registers across the walk, they
  // were among the values the setup spilled at five waves per SIMD.
  if (t == 0) {
    F.umax = umax;
    F.vmax = vmax;
    F.dtmax = dtmax;
    F.l2amin = log2f(th.alpha_min);
  }
  wave_box<2>(u, v, active, &wb);
  float clipv[2] = {0.f, 0.f}, dlen[2] = {1.f, 1.f};
  if (CLIP) {
#pragma unroll
    for (int k = 0; k < 2; k++) {
      if (!active[k]) continue;
      clipv[k] = clip[pix_base + (long long)(py0 + 4 * k) * cam.W + px];
      dlen[k] = sqrtf(fmaf(u[k], u[k], fmaf(v[k], v[k], 1.0f)));
    }
    wave_clip_max<2>(clipv, active, &wb);
  }

  const uint2 rg = ranges[cam.tile_base + tile];
  const uint32_t len = __builtin_amdgcn_readfirstlane(rg.y - rg.x);
  // long lists first in the schedule, and their waves first at issue
  if (len >= 2048) __builtin_amdgcn_s_setprio(3);
  else if (len >= 1024) __builtin_amdgcn_s_setprio(2);
  else if (len >= 256) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
  // Colour accumulates in FP64 (three FMAs per contributing entry) so that
  // the backward can form suffix sums C - C_<=j without FP32 cancellation.
  // A stopped pixel keeps -T (T >= t_min > 0 while it runs): the stop is
  // then one select on T instead of a flag of its own.
  float T[2] = {active[0] ? 1.0f : -1.0f, active[1] ? 1.0f : -1.0f};
  double C[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  uint32_t last[2] = {0u, 0u}, nev[2] = {active[0] ? len : 0u, active[1] ? len : 0u};
  for (uint32_t b = 0; b < len; b += kRBatch) {
    // (also publishes wb before the first setup)
    if (__syncthreads_count(T[0] > 0.0f || T[1] > 0.0f) == 0) break;
    b = __builtin_amdgcn_readfirstlane(b);
    uint32_t fl = 0u;
    if (b + t < len) {
      uint32_t e = ids[rg.x + b + t];
      fl = pair_setup<RS, false, GEN, CLIP>(record, rgb, e, (int)(e - (uint32_t)cam_idx * (uint32_t)n), F,
                                      cam, F.umax, F.vmax, F.dtmax, th, F.l2amin, wb, kRThreads / 64,
                                      &pd[t * S]);
    }
    pf[t] = fl;
    __syncthreads();
    // the batch's pairs that may reach alpha_min somewhere in this wave's half-tile
    const uint32_t f0 = pf[lane], f1 = pf[lane + 64];
    const unsigned long long m0 = __builtin_amdgcn_ballot_w64((f0 >> wv) & 1u);
    const unsigned long long m1 = __builtin_amdgcn_ballot_w64((f1 >> wv) & 1u);
    const unsigned long long x0 = __builtin_amdgcn_ballot_w64((f0 & kMixedBit) != 0u);
    const unsigned long long x1 = __builtin_amdgcn_ballot_w64((f1 & kMixedBit) != 0u);
    bool wave_done = false;
    for (int h = 0; h < 2 && !wave_done; h++) {
      unsigned long long m = h ? m1 : m0;
      const unsigned long long xm = h ? x1 : x0;
      while (m) {
        if (!wave_any(T[0] > 0.0f || T[1] > 0.0f)) { wave_done = true; break; }
        const uint32_t ql = (uint32_t)__builtin_ctzll(m), q = 64u * h + ql;
        m &= m - 1ull;
        const uint32_t idx1 = b + q + 1;  // the entry's 1-based place in the list
        const float4* P = &pd[q * S];
        PairRegs<RS> r;
        load_pair<RS>(P, r);
        r.mixed = (xm >> ql) & 1ull;  // (from the flags: no wait on the LDS read)
        Eval ev[2];
#pragma unroll
        for (int k = 0; k < 2; k++) {
          eval_test<RS>(r, P, u[k], v[k], dt[k], &ev[k]);
          if (CLIP) ev[k].ok = ev[k].ok && !behind_clip<RS>(r, P, u[k], v[k], dt[k], dlen[k], clipv[k], ev[k].dd);
        }
        const bool live0 = ev[0].ok & (T[0] > 0.0f), live1 = ev[1].ok & (T[1] > 0.0f);
        if (!wave_any(live0 | live1)) continue;  // nothing reaches alpha_min here
        bool contrib[2];
        float wgt[2];
#pragma unroll
        for (int k = 0; k < 2; k++) {
          eval_alpha<RS, GEN>(r, th, &ev[k]);
          const bool live = k ? live1 : live0;
          const float Tn = fmaf(-ev[k].a, T[k], T[k]);  // T (1 - alpha)
          const bool stop = live & (Tn < th.t_min);  // stop before adding this particle
          contrib[k] = live ^ stop;
          const float ae = contrib[k] ? ev[k].a : 0.0f;
          wgt[k] = ae * T[k];
          const float Tk = contrib[k] ? Tn : T[k];
          T[k] = stop ? -T[k] : Tk;
          last[k] = contrib[k] ? idx1 : last[k];
          if (NE) nev[k] = stop ? idx1 : nev[k];
        }
        // some lane passed the alpha_min test, so almost always some lane
        // contributes: accumulate unconditionally (zero weights add nothing)
        double col[3];
        pair_colour<RS>(P, col);
#pragma unroll
        for (int k = 0; k < 2; k++) {
          const double w = (double)wgt[k];
          C[k][0] = fma(w, col[0], C[k][0]);
          C[k][1] = fma(w, col[1], C[k][1]);
          C[k][2] = fma(w, col[2], C[k][2]);
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 2; k++) {
    if (!inside[k]) continue;
    const int py = py0 + 4 * k;
    long long pix = pix_base + (long long)py * cam.W + px;
    const float Tf = fabsf(T[k]);
    out_rgb[3 * pix] = (float)fma((double)Tf, (double)th.bg[0], C[k][0]);
    out_rgb[3 * pix + 1] = (float)fma((double)Tf, (double)th.bg[1], C[k][1]);
    out_rgb[3 * pix + 2] = (float)fma((double)Tf, (double)th.bg[2], C[k][2]);
    if (out_T) out_T[pix] = Tf;
    if (out_nc) out_nc[pix] = last[k];
    if (NE) out_ne[pix] = nev[k];
  }
}

// One block per tile, taken in the render order (longest lists first).  NE:
// also count each pixel's evaluated entries (out_ne non-null).
template <bool RS, bool NE, bool GEN, bool CLIP>
__global__ void __launch_bounds__(kRThreads, 5) render_kernel(
    DevCam cam, Thresholds th, int n, int cam_idx, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ ids,
    const float4* __restrict__ record, const float* __restrict__ rgb, const float* __restrict__ clip,
    float* __restrict__ out_rgb,
    float* __restrict__ out_T, uint32_t* __restrict__ out_nc, uint32_t* __restrict__ out_ne) {
  __shared__ float4 pd[kRBatch * Slots<RS, false>::N];
  __shared__ uint32_t pf[kRBatch];
  __shared__ TileFrameD F;
  __shared__ WaveBoxes wb;
  __shared__ float red[6];
  const int tile = (int)order[cam.tile_base + blockIdx.x];
  render_tile<RS, NE, GEN, CLIP>(cam, th, n, cam_idx, tile, ranges, ids, record, rgb, clip, out_rgb,
                                 out_T, out_nc, out_ne, cam.pixel_base, pd, pf, F, wb, red);
}

// Several cameras of one shutter type and one tile count in one launch
// (kMultiCams at most, passed by value): block b takes tile b / n of camera
// b % n in that camera's render order, so the cameras' longest tiles start
// together and one camera's tail overlaps the others' work instead of ending
// a launch of its own.  Blocks are dealt to the 8 XCDs round-robin, so with
// two cameras each XCD renders one of them and its L2 holds that camera's
// records only.  The XCDs of the heavier view then finish later (a fisheye
// view's about a tenth after a pinhole view's); dealing 32 tiles of each
// camera in turn balances the XCDs but mixes the cameras in every L2, and
// took as long with 18% more memory traffic.
constexpr int kMultiCams = 4;
struct MultiCams {
  DevCam cam[kMultiCams];
  int idx[kMultiCams];  // the cameras' indices in the call
  int n;
};

template <bool RS, bool NE, bool GEN, bool CLIP>
__global__ void __launch_bounds__(kRThreads, 5) render_multi_kernel(
    MultiCams mc, Thresholds th, int n, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ ids,
    const float4* __restrict__ record, const float* __restrict__ rgb, const float* __restrict__ clip,
    float* __restrict__ out_rgb,
    float* __restrict__ out_T, uint32_t* __restrict__ out_nc, uint32_t* __restrict__ out_ne) {
  __shared__ float4 pd[kRBatch * Slots<RS, false>::N];
  __shared__ uint32_t pf[kRBatch];
  __shared__ TileFrameD F;
  __shared__ WaveBoxes wb;
  __shared__ float red[6];
  const int c = (int)(blockIdx.x % (unsigned)mc.n), k = (int)(blockIdx.x / (unsigned)mc.n);
  const DevCam& cam = mc.cam[c];
  const int tile = (int)order[cam.tile_base + k];
  render_tile<RS, NE, GEN, CLIP>(cam, th, n, mc.idx[c], tile, ranges, ids, record, rgb, clip, out_rgb,
                                 out_T, out_nc, out_ne, cam.pixel_base, pd, pf, F, wb, red);
}

// Persistent render of the cameras of one shutter type in a multi-camera
// batch.  Items are (camera, k-th tile of its render order) over the listed
// cameras, in order.  Item i belongs to XCD i % 8 (blocks are dealt to XCDs
// round-robin), and each XCD has its own counter, so every XCD walks its
// share longest-first; a block that drains its XCD's share steals from the
// others, and leaves once every counter is past its share.  Images go to
// outs[camera] ([H, W, 3]).
template <bool RS, bool GEN>
__global__ void __launch_bounds__(kRThreads, 4) render_batch_kernel(
    const DevCam* __restrict__ cams, const int* __restrict__ cam_list,
    const int* __restrict__ item_start, int n_list, int n_items, unsigned* __restrict__ counters,
    Thresholds th, int n, const uint2* __restrict__ ranges, const uint32_t* __restrict__ order,
    const uint32_t* __restrict__ ids,
    const float4* __restrict__ record, const float* __restrict__ rgb, float* const* __restrict__ outs) {
  __shared__ float4 pd[kRBatch * Slots<RS, false>::N];
  __shared__ uint32_t pf[kRBatch];
  __shared__ TileFrameD F;
  __shared__ WaveBoxes wb;
  __shared__ float red[6];
  __shared__ int item_s;
  const int nx = 8;
  const int my = blockIdx.x % nx;
  const int q = n_items / nx, r = n_items % nx;
  int probe = 0;  // which XCD share this block is draining (its own first)
  while (true) {
    if (threadIdx.x == 0) {
      int it = -1;
      while (probe < nx) {
        int x = (my + probe) % nx;
        int len = q + (x < r ? 1 : 0);  // items x, x + 8, x + 16, ...
        unsigned k = atomicAdd(&counters[x], 1u);
        if ((int)k < len) { it = x + nx * (int)k; break; }
        probe++;
      }
      item_s = it;
    }
    __syncthreads();
    const int item = item_s;
    __syncthreads();
    if (item < 0) break;
    int j = 0;
    while (j + 1 < n_list && item_start[j + 1] <= item) j++;
    // the camera is read where it lies, at a wave-uniform index, so its
    // fields load into scalar registers
    const int c = __builtin_amdgcn_readfirstlane(cam_list[j]);
    const DevCam& cam = cams[c];
    const int tile = (int)order[cam.tile_base + (item - item_start[j])];
    render_tile<RS, false, GEN, false>(cam, th, n, c, tile, ranges, ids, record, rgb, nullptr, outs[c],
                                       nullptr, nullptr, nullptr, 0, pd, pf, F, wb, red);
  }
}

// Launch the batch render: one persistent kernel per shutter type present.
// d_lists holds, per type, the camera indices and item prefix sums
// (2 x (kMaxCams + kMaxCams + 1) ints); d_counters 16 counters.
gut_status render_batch_launch(const DevCam* d_cams, const DevCam* h_cams, int n_cams,
                               const Thresholds& th, int n, const uint32_t* ranges,
                               const uint32_t* order, const uint32_t* ids, const float* record,
                               const float* rgb, float* const* d_outs, unsigned* d_counters,
                               int* d_lists, int* h_lists, int n_blocks, hipStream_t s) {
  gut_status st = fill_u32(d_counters, 16, 0u, s);
  if (st != GUT_OK) return st;
  for (int type = 0; type < 2; type++) {
    int* hl = h_lists + type * (2 * kMaxCams + 1);
    int* cl = hl;
    int* is = hl + kMaxCams;
    int m = 0, items = 0;
    for (int c = 0; c < n_cams; c++) {
      if ((h_cams[c].shutter == GUT_ROLLING_TOP_TO_BOTTOM) != (type == 1)) continue;
      cl[m] = c;
      is[m] = items;
      items += h_cams[c].tiles_x * h_cams[c].tiles_y;
      m++;
    }
    is[m] = items;
    if (m == 0) continue;
    int* dl = d_lists + type * (2 * kMaxCams + 1);
    GUT_HIP(hipMemcpyAsync(dl, hl, (2 * kMaxCams + 1) * sizeof(int), hipMemcpyHostToDevice, s));
#define GUT_RB(RS, GEN)                                                                          \
  render_batch_kernel<RS, GEN><<<n_blocks, kRThreads, 0, s>>>(                                    \
      d_cams, dl, dl + kMaxCams, m, items, d_counters + 8 * type, th, n, (const uint2*)ranges, order, \
      ids, (const float4*)record, rgb, d_outs)
    const bool gen = th.kdeg != 2;
    if (type == 1) { if (gen) GUT_RB(true, true); else GUT_RB(true, false); }
    else { if (gen) GUT_RB(false, true); else GUT_RB(false, false); }
#undef GUT_RB
    GUT_LAUNCH_CHECK();
  }
  return GUT_OK;
}

// "Ours (sorted)" (Sec. 4.3): multi-layer alpha blending with a per-ray
// buffer of the kKBuf farthest hits.  One 256-thread block per tile, one pixel
// per thread (wave w owns rows 4w .. 4w + 3), the tile's list consumed in
// batches of 256 pairs set up as in render_tile.  A hit is a list entry that
// passes the alpha_min test; its distance along the ray is tau_max |d|.  Each
// thread keeps its buffer sorted nearest first in registers: slot 0 holds the
// nearest hit, or a -inf sentinel (alpha 0) while the buffer is not full;
// capacity k < kKBuf leaves kKBuf - k +inf walls at the far end.  A hit no
// nearer than slot 0 evicts it -- slot 0 is blended (a sentinel blends to
// nothing) and the hit is merged into the remaining sorted slots by a fixed
// compare-select chain; a hit at or before slot 0 is blended at once.  With a
// full-size buffer (k = kKBuf) the slots instead move one place nearer, the
// hit takes the last one and moves nearer level by level while some lane of
// the wave still moves: hits arrive nearly in depth order, so a third of the
// insertion steps need no level and the wave's deepest move averages about
// two.  Blending is Eq. 5 with the t_min stop; at the end of the list the
// buffer is blended nearest first.  The buffer keeps each hit's list position; the colour a
// blend needs comes from an LDS copy of the two latest batches' colours
// (a buffer usually turns over within a batch), else through the list.
constexpr int kKBuf = 16;
constexpr int kKThreads = 256;
// Four waves per SIMD (128 VGPRs, some of the buffer in scratch): the walk
// waits on LDS and on the colour fetches of evicted hits, and a fourth wave
// hides more of that than the spills cost.  (Keeping the hits' payloads in an
// LDS table instead, so that only 32-bit keys move, cuts the VALU work of an
// insertion by two thirds but takes so much LDS that two waves per SIMD fit,
// and is slower.)

// Colours of the hits at list positions [wlo, wlo + kKWin) (the two latest
// batches) are kept in LDS, row pos mod kKWin; an older hit's colour is read
// through the list.
constexpr int kKWin = 2 * kKThreads;
struct KbufColours {
  const float* cw;         // LDS rows of 3
  const uint32_t* lids;    // the tile's sorted entry ids
  const float* rgb;
  uint32_t wlo;
};

// Slot 0 leaves on the lanes with ins set: slots J.. move one place nearer and
// the hit takes the last slot.  Written as a recursion so that every slot
// index is a constant from the start: in a loop the compiler folds each
// select of two slots into one read through a lane-dependent address, and the
// whole buffer then lives in scratch memory.
template <int J>
__device__ __forceinline__ void kbuf_shift(float (&bd)[kKBuf], float (&ba)[kKBuf],
                                           uint32_t (&bi)[kKBuf], bool ins, float dist, float a,
                                           uint32_t e) {
  if constexpr (J < kKBuf - 1) {
    bd[J] = ins ? bd[J + 1] : bd[J];
    ba[J] = ins ? ba[J + 1] : ba[J];
    bi[J] = ins ? bi[J + 1] : bi[J];
    kbuf_shift<J + 1>(bd, ba, bi, ins, dist, a, e);
  } else {
    bd[J] = ins ? dist : bd[J];
    ba[J] = ins ? a : ba[J];
    bi[J] = ins ? e : bi[J];
  }
}

// One level of the move nearer: on the lanes whose hit (now in slot I + 1)
// lies at or before slot I, the two swap; the next level runs while some
// lane of the wave still moves.
template <int I>
__device__ __forceinline__ void kbuf_bubble(float (&bd)[kKBuf], float (&ba)[kKBuf],
                                            uint32_t (&bi)[kKBuf], bool mv, unsigned long long mm,
                                            float dist, float a, uint32_t e) {
  // mm: the moving lanes as a wave mask, kept from ballots of the bare
  // compare (a ballot of a combined lane flag goes through a vector register)
  const bool ge = bd[I] >= dist;
  mv = mv && ge;
  mm &= __builtin_amdgcn_ballot_w64(ge);
  if (mm == 0ull) return;
  // an empty statement with side effects: without it the compiler turns the
  // wave-uniform early exits into straight-line selects over all 15 levels
  asm volatile("");
  bd[I + 1] = mv ? bd[I] : bd[I + 1];
  ba[I + 1] = mv ? ba[I] : ba[I + 1];
  bi[I + 1] = mv ? bi[I] : bi[I + 1];
  bd[I] = mv ? dist : bd[I];
  ba[I] = mv ? a : ba[I];
  bi[I] = mv ? e : bi[I];
  if constexpr (I > 0) kbuf_bubble<I - 1>(bd, ba, bi, mv, mm, dist, a, e);
}

__device__ __forceinline__ void kbuf_blend(float a, uint32_t pos, const KbufColours& K,
                                           float t_min, float& T, double (&C)[3], uint32_t& nc,
                                           uint32_t& done) {
  if (a <= 0.0f || done) return;  // a sentinel or a wall, or the pixel has stopped
  const float Tn = fmaf(-a, T, T);
  if (Tn < t_min) { done = 1u; return; }
  const double w = (double)(a * T);
  // the LDS row is read in any case and an older hit's colour then replaces
  // it; the empty register constraint keeps the compiler from folding the two
  // reads into one flat read through a selected pointer
  const float* cl = K.cw + 3 * (pos & (kKWin - 1));
  float c0 = cl[0], c1 = cl[1], c2 = cl[2];
  asm volatile("" : "+v"(c0), "+v"(c1), "+v"(c2));
  if (pos < K.wlo) {
    const float* c = K.rgb + 3 * (size_t)K.lids[pos];
    c0 = c[0]; c1 = c[1]; c2 = c[2];
  }
  C[0] = fma(w, (double)c0, C[0]);
  C[1] = fma(w, (double)c1, C[1]);
  C[2] = fma(w, (double)c2, C[2]);
  T = Tn;
  nc++;
}

template <bool RS, bool NE, bool GEN, bool CLIP, bool FULL>
__global__ void __launch_bounds__(kKThreads, 4) render_kbuffer_kernel(
    DevCam cam, Thresholds th, int n, int cam_idx, int kcap, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ ids,
    const float4* __restrict__ record, const float* __restrict__ rgb, const float* __restrict__ clip,
    float* __restrict__ out_rgb,
    float* __restrict__ out_T, uint32_t* __restrict__ out_nc, uint32_t* __restrict__ out_ne) {
  constexpr int S = Slots<RS, false>::N;
  __shared__ float4 pd[kKThreads * S];
  __shared__ uint32_t pf[kKThreads];
  __shared__ float cw[kKWin * 3];
  __shared__ TileFrameD F;
  __shared__ WaveBoxes wb;
  __shared__ float red[12];
  const int tile = (int)order[cam.tile_base + blockIdx.x];
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  const int px = tx * kTile + (lane & (kTile - 1));
  const int py = ty * kTile + 4 * wv + (lane >> 4);
  if (t == 0) tile_frame(cam, tx, ty, &F);
  __syncthreads();
  const bool inside = px < cam.W && py < cam.H;
  float u = 0.f, v = 0.f, dt = 0.f;
  bool active = inside && pixel_ray(cam, F, px, py, &u, &v, &dt);
  float umax, vmax, dtmax;
  tile_bounds<1>(&u, &v, &dt, &active, red, &umax, &vmax, &dtmax);
  const float l2amin = log2f(th.alpha_min);
  wave_box<1>(&u, &v, &active, &wb);
  const float dlen = sqrtf(fmaf(u, u, fmaf(v, v, 1.0f)));
  float clipv = 0.0f;  // hybrid rendering (Sec. 6.2), as in render_tile
  if (CLIP) {
    if (active) clipv = clip[cam.pixel_base + (long long)py * cam.W + px];
    wave_clip_max<1>(&clipv, &active, &wb);
  }

  const uint2 rg = ranges[cam.tile_base + tile];
  const uint32_t len = __builtin_amdgcn_readfirstlane(rg.y - rg.x);
  float bd[kKBuf], ba[kKBuf];
  uint32_t bi[kKBuf];
#pragma unroll
  for (int j = 0; j < kKBuf; j++) {
    bd[j] = j < kcap ? -INFINITY : INFINITY;
    ba[j] = 0.0f;
    bi[j] = 0u;
  }
  float T = 1.0f;
  double C[3] = {0.0, 0.0, 0.0};
  uint32_t nc = 0u, nev = active ? len : 0u;
  uint32_t done = active ? 0u : 1u;  // a 0/1 vector register, as in render_tile
  KbufColours K = {cw, ids + rg.x, rgb, 0u};
  for (uint32_t b = 0; b < len; b += kKThreads) {
    if (__syncthreads_count(done == 0u) == 0) break;  // (also publishes wb before the first setup)
    K.wlo = b >= (uint32_t)kKThreads ? b - kKThreads : 0u;
    uint32_t fl = 0u;
    if (b + t < len) {
      const uint32_t e = ids[rg.x + b + t];
      float* c = cw + 3 * ((b + t) & (kKWin - 1));
      c[0] = rgb[3 * (size_t)e]; c[1] = rgb[3 * (size_t)e + 1]; c[2] = rgb[3 * (size_t)e + 2];
      fl = pair_setup<RS, false, GEN, CLIP>(record, rgb, e, (int)(e - (uint32_t)cam_idx * (uint32_t)n),
                                            F, cam, umax, vmax, dtmax, th, l2amin, wb, kKThreads / 64,
                                            &pd[t * S]);
    }
    pf[t] = fl;
    __syncthreads();
    bool wave_done = false;
    for (int h = 0; h < kKThreads / 64 && !wave_done; h++) {
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
        if (FULL) {
          // the hit's distance tau' |d|, tau' = -(o_g . d_g) / |d_g|^2 (the clip test's form)
          float odg;
          if (!RS) {
            const float4 p5 = P[5];
            odg = fmaf(v, p5.z, fmaf(u, p5.y, p5.x));
          } else {
            odg = fmaf(v, r.p4.w, fmaf(u, r.p3.w, r.p5.w));
            odg = fmaf(dt, fmaf(v, r.p9.w, fmaf(u, r.p8.w, r.p7.w)), odg);
          }
          const float dist = -odg * dlen * ev.idd;
          const uint32_t e = b + q;  // the hit's list position
          const bool ins = live && !(dist <= bd[0]);
          if (live && !ins) kbuf_blend(ev.a, e, K, th.t_min, T, C, nc, done);
          if (ins) kbuf_blend(ba[0], bi[0], K, th.t_min, T, C, nc, done);
          // slot 0 leaves: the other slots move one place nearer and the hit
          // takes the last one, then moves nearer past every slot at or beyond
          // its distance (so it goes before equal ones), level by level for as
          // long as a lane of the wave still moves (hits arrive nearly in depth
          // order: most steps need no level or a few)
          kbuf_shift<0>(bd, ba, bi, ins, dist, ev.a, e);
          kbuf_bubble<kKBuf - 2>(bd, ba, bi, ins, __builtin_amdgcn_ballot_w64(ins), dist, ev.a, e);
          if (NE && live && done) nev = b + q + 1;
        } else if (live) {
          // the hit's distance tau' |d|, tau' = -(o_g . d_g) / |d_g|^2 (the clip test's form)
          float odg;
          if (!RS) {
            const float4 p5 = P[5];
            odg = fmaf(v, p5.z, fmaf(u, p5.y, p5.x));
          } else {
            odg = fmaf(v, r.p4.w, fmaf(u, r.p3.w, r.p5.w));
            odg = fmaf(dt, fmaf(v, r.p9.w, fmaf(u, r.p8.w, r.p7.w)), odg);
          }
          const float dist = -odg * dlen * ev.idd;
          const uint32_t e = b + q;  // the hit's list position
          const uint32_t idx1 = b + q + 1;
          if (dist <= bd[0]) {
            kbuf_blend(ev.a, e, K, th.t_min, T, C, nc, done);
          } else {
            kbuf_blend(ba[0], bi[0], K, th.t_min, T, C, nc, done);
            // merge the hit into slots 1 .. kKBuf-1 (sorted), dropping slot 0
#pragma unroll
            for (int j = 0; j < kKBuf - 1; j++) {
              const bool nx = bd[j + 1] < dist, here = j == 0 || bd[j] < dist;
              // the buffer is sorted and dist > bd[0]: the slot's new distance is
              // the middle one of bd[j], dist, bd[j + 1]
              const float od = __builtin_amdgcn_fmed3f(bd[j], dist, bd[j + 1]);
              const float oa = nx ? ba[j + 1] : (here ? ev.a : ba[j]);
              const uint32_t oi = nx ? bi[j + 1] : (here ? e : bi[j]);
              bd[j] = od; ba[j] = oa; bi[j] = oi;
            }
            const bool last = bd[kKBuf - 1] < dist;
            ba[kKBuf - 1] = last ? ev.a : ba[kKBuf - 1];
            bi[kKBuf - 1] = last ? e : bi[kKBuf - 1];
            bd[kKBuf - 1] = last ? dist : bd[kKBuf - 1];
          }
          if (NE && done) nev = idx1;
        }
      }
    }
  }
  // the buffer, nearest first
#pragma unroll
  for (int j = 0; j < kKBuf; j++) kbuf_blend(ba[j], bi[j], K, th.t_min, T, C, nc, done);
  if (!inside) return;
  const long long pix = cam.pixel_base + (long long)py * cam.W + px;
  out_rgb[3 * pix] = (float)fma((double)T, (double)th.bg[0], C[0]);
  out_rgb[3 * pix + 1] = (float)fma((double)T, (double)th.bg[1], C[1]);
  out_rgb[3 * pix + 2] = (float)fma((double)T, (double)th.bg[2], C[2]);
  if (out_T) out_T[pix] = T;
  if (out_nc) out_nc[pix] = nc;
  if (NE) out_ne[pix] = nev;
}

static gut_status launch_render_kbuffer(const DevCam& cam, const Thresholds& th, int n, int cam_idx,
                                        int kcap, const uint32_t* ranges, const uint32_t* order,
                                        const uint32_t* ids, const float* record, const float* rgb,
                                        const float* clip, float* out_rgb, float* out_T,
                                        uint32_t* out_nc, uint32_t* out_ne, hipStream_t s) {
  dim3 grid(cam.tiles_x * cam.tiles_y), block(kKThreads);
#define GUT_RKB2(RS, NE, GEN, CLIP, FULL)                                                          \
  render_kbuffer_kernel<RS, NE, GEN, CLIP, FULL><<<grid, block, 0, s>>>(cam, th, n, cam_idx, kcap,     \
                                                                        (const uint2*)ranges, order, ids, \
                                                                        (const float4*)record, rgb, clip, \
                                                                        out_rgb, out_T, out_nc, out_ne)
#define GUT_RKB(RS, NE, GEN, CLIP) \
  do { if (kcap == kKBuf) GUT_RKB2(RS, NE, GEN, CLIP, true); else GUT_RKB2(RS, NE, GEN, CLIP, false); } while (0)
#define GUT_RKB0(RS, NE, GEN) \
  do { if (clip) GUT_RKB(RS, NE, GEN, true); else GUT_RKB(RS, NE, GEN, false); } while (0)
#define GUT_RKB1(RS, NE) \
  do { if (th.kdeg != 2) GUT_RKB0(RS, NE, true); else GUT_RKB0(RS, NE, false); } while (0)
  const bool rs = cam.shutter == GUT_ROLLING_TOP_TO_BOTTOM;
  if (rs) { if (out_ne) GUT_RKB1(true, true); else GUT_RKB1(true, false); }
  else { if (out_ne) GUT_RKB1(false, true); else GUT_RKB1(false, false); }
#undef GUT_RKB1
#undef GUT_RKB0
#undef GUT_RKB
#undef GUT_RKB2
  GUT_LAUNCH_CHECK();
  return GUT_OK;
}

gut_status launch_render(const DevCam& cam, const Thresholds& th, int n, int cam_idx,
                         const uint32_t* ranges, const uint32_t* order, const uint32_t* ids,
                         const float* record, const float* rgb, const float* clip, float* out_rgb,
                         float* out_T, uint32_t* out_nc, uint32_t* out_ne, hipStream_t s) {
  dim3 grid(cam.tiles_x * cam.tiles_y), block(kRThreads);
#define GUT_RK(RS, NE, GEN, CLIP)                                                                  \
  render_kernel<RS, NE, GEN, CLIP><<<grid, block, 0, s>>>(cam, th, n, cam_idx, (const uint2*)ranges, \
                                                          order, ids, (const float4*)record, rgb,     \
                                                          clip, out_rgb, out_T, out_nc, out_ne)
#define GUT_RK1(RS, NE, GEN) \
  if (clip) GUT_RK(RS, NE, GEN, true); else GUT_RK(RS, NE, GEN, false)
#define GUT_RK2(RS, NE) \
  do { if (th.kdeg != 2) { GUT_RK1(RS, NE, true); } else { GUT_RK1(RS, NE, false); } } while (0)
  const bool rs = cam.shutter == GUT_ROLLING_TOP_TO_BOTTOM;
  if (rs) { if (out_ne) GUT_RK2(true, true); else GUT_RK2(true, false); }
  else { if (out_ne) GUT_RK2(false, true); else GUT_RK2(false, false); }
#undef GUT_RK2
#undef GUT_RK1
#undef GUT_RK
  GUT_LAUNCH_CHECK();
  return GUT_OK;
}

// Consecutive cameras of one shutter type and one tile count share a launch
// (up to kMultiCams); a camera alone takes render_kernel.
static gut_status launch_render_group(const DevCam* dc, int c0, int c1, const Thresholds& th, int n,
                                      const uint32_t* ranges, const uint32_t* order,
                                      const uint32_t* ids, const float* record, const float* rgb,
                                      const float* clip, float* out_rgb, float* out_T,
                                      uint32_t* out_nc, uint32_t* out_ne, hipStream_t s) {
  if (c1 - c0 == 1)
    return launch_render(dc[c0], th, n, c0, ranges, order, ids, record, rgb, clip, out_rgb, out_T,
                         out_nc, out_ne, s);
  MultiCams mc = {};
  mc.n = c1 - c0;
  for (int k = 0; k < mc.n; k++) {
    mc.cam[k] = dc[c0 + k];
    mc.idx[k] = c0 + k;
  }
  dim3 grid(mc.n * dc[c0].tiles_x * dc[c0].tiles_y), block(kRThreads);
#define GUT_RM(RS, NE, GEN, CLIP)                                                                    \
  render_multi_kernel<RS, NE, GEN, CLIP><<<grid, block, 0, s>>>(mc, th, n, (const uint2*)ranges, order, \
                                                                ids, (const float4*)record, rgb, clip,  \
                                                                out_rgb, out_T, out_nc, out_ne)
#define GUT_RM1(RS, NE, GEN) \
  if (clip) GUT_RM(RS, NE, GEN, true); else GUT_RM(RS, NE, GEN, false)
#define GUT_RM2(RS, NE) \
  do { if (th.kdeg != 2) { GUT_RM1(RS, NE, true); } else { GUT_RM1(RS, NE, false); } } while (0)
  const bool rs = dc[c0].shutter == GUT_ROLLING_TOP_TO_BOTTOM;
  if (rs) { if (out_ne) GUT_RM2(true, true); else GUT_RM2(true, false); }
  else { if (out_ne) GUT_RM2(false, true); else GUT_RM2(false, false); }
#undef GUT_RM2
#undef GUT_RM1
#undef GUT_RM
  GUT_LAUNCH_CHECK();
  return GUT_OK;
}

}  // namespace gut

using namespace gut;

extern "C" gut_status gut_render(const gut_projected* proj, int64_t n, const uint32_t* tile_ranges,
                                 const uint32_t* sorted_ids, const gut_camera* cams, int32_t n_cams,
                                 const gut_params* p, const float* clip_depth, float* rgb,
                                 float* T_final, uint32_t* n_contrib, uint32_t* n_eval, void* stream) {
  gut_status st = check_params(p);
  if (st != GUT_OK) return st;
  if (!proj || (n > 0 && (!proj->record || !proj->rgb)) || !tile_ranges || !rgb || !T_final ||
      !n_contrib) {
    set_error("record, rgb, tile_ranges and the three outputs are required");
    return GUT_E_INVALID;
  }
  if (((uintptr_t)proj->record & 15) || ((uintptr_t)tile_ranges & 7)) {
    set_error("record must be 16-byte and tile_ranges 8-byte aligned");
    return GUT_E_INVALID;
  }
  if (n < 0 || n * (int64_t)n_cams >= (int64_t(1) << 31)) {
    set_error("n * n_cams must be below 2^31");
    return GUT_E_INVALID;
  }
  DevCam dc[kMaxCams];
  int64_t T = 0;
  if ((st = prepare_cams(cams, n_cams, *p, dc, &T, nullptr)) != GUT_OK) return st;
  Thresholds th = make_thresholds(*p);
  if (p->kbuffer > 0) {  // "Ours (sorted)": one launch per camera
    for (int c = 0; c < n_cams; c++)
      if ((st = launch_render_kbuffer(dc[c], th, (int)n, c, p->kbuffer, tile_ranges, tile_ranges + 2 * T,
                                      sorted_ids, proj->record, proj->rgb,
                                      clip_depth, rgb,
                                      T_final, n_contrib, n_eval, (hipStream_t)stream)) != GUT_OK)
        return st;
    return GUT_OK;
  }
  for (int c0 = 0; c0 < n_cams;) {
    int c1 = c0 + 1;
    while (c1 < n_cams && c1 - c0 < kMultiCams && dc[c1].shutter == dc[c0].shutter &&
           dc[c1].tiles_x * dc[c1].tiles_y == dc[c0].tiles_x * dc[c0].tiles_y)
      c1++;
    st = launch_render_group(dc, c0, c1, th, (int)n, tile_ranges, tile_ranges + 2 * T, sorted_ids,
                             proj->record, proj->rgb, clip_depth, rgb, T_final, n_contrib, n_eval,
                             (hipStream_t)stream);
    if (st != GUT_OK) return st;
    c0 = c1;
  }
  return GUT_OK;
}
