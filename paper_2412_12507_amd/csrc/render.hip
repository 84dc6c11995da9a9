// K5 -- per-tile front-to-back compositing (Eq. 5) with each particle's
// response evaluated in 3D at its maximum along the pixel ray (Eq. 11).
//
// One 256-thread block (4 wave64s) per 16x16 tile, one pixel per thread.  The
// tile's sorted list is consumed in batches of 256: each thread gathers one
// pair's 64-byte render record, forms the pair's FP64 tile-frame terms
// (tile_eval.h) and stores them in LDS; then every thread walks the batch,
// reading each pair as an LDS broadcast.  A thread stops when its
// transmittance would fall below t_min; the block stops when no thread is
// still going (__syncthreads_count).
#include "tile_eval.h"

namespace gut {

template <bool RS>
__global__ void __launch_bounds__(kTilePix) render_kernel(
    DevCam cam, Thresholds th, int n, int cam_idx, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ ids, const float4* __restrict__ record,
    const float* __restrict__ rgb, float* __restrict__ out_rgb, float* __restrict__ out_T,
    uint32_t* __restrict__ out_nc, uint32_t* __restrict__ out_ne) {
  constexpr int S = Slots<RS>::N;
  __shared__ float4 pd[kTilePix * S];
  __shared__ TileFrameD F;
  __shared__ float red[12];

  const int tile = blockIdx.x;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int t = threadIdx.x;
  const int px = tx * kTile + (t & (kTile - 1)), py = ty * kTile + t / kTile;
  if (t == 0) tile_frame(cam, tx, ty, &F);
  __syncthreads();
  const bool inside = px < cam.W && py < cam.H;
  float u = 0.0f, v = 0.0f, dt = 0.0f;
  bool active = inside && pixel_ray(cam, F, px, py, &u, &v, &dt);
  float umax, vmax, dtmax;
  tile_bounds(u, v, dt, active, red, &umax, &vmax, &dtmax);

  const uint2 rg = ranges[cam.tile_base + tile];
  const uint32_t len = rg.y - rg.x;
  // Colour accumulates in FP64 (three FMAs per contributor) so that the
  // backward can form suffix sums C - C_<=j without FP32 cancellation.
  float T = 1.0f;
  double C0 = 0.0, C1 = 0.0, C2 = 0.0;
  uint32_t last = 0, nev = active ? len : 0u;
  bool done = !active;
  for (uint32_t b = 0; b < len; b += kTilePix) {
    if (__syncthreads_count(!done) == 0) break;
    if (b + t < len) {
      uint32_t e = ids[rg.x + b + t];
      pair_setup<RS>(record, rgb, e, (int)(e - (uint32_t)cam_idx * (uint32_t)n), F, cam, umax,
                     vmax, dtmax, &pd[t * S]);
    }
    __syncthreads();
    const uint32_t cnt = min((uint32_t)kTilePix, len - b);
    for (uint32_t q = 0; q < cnt && !done; q++) {
      Eval ev;
      if (!eval_pair<RS>(&pd[q * S], u, v, dt, th.alpha_min, th.alpha_max, &ev)) continue;
      float Tn = T * (1.0f - ev.a);
      if (Tn < th.t_min) {  // stop before adding (would leave T below t_min)
        done = true;
        nev = b + q + 1;
        break;
      }
      const double wgt = (double)(ev.a * T);
      const float4* P = &pd[q * S];
      C0 = fma(wgt, (double)P[1].w, C0);
      C1 = fma(wgt, (double)P[2].w, C1);
      C2 = fma(wgt, (double)P[3].w, C2);
      T = Tn;
      last = b + q + 1;
    }
  }
  if (inside) {
    long long pix = cam.pixel_base + (long long)py * cam.W + px;
    out_rgb[3 * pix] = (float)fma((double)T, (double)th.bg[0], C0);
    out_rgb[3 * pix + 1] = (float)fma((double)T, (double)th.bg[1], C1);
    out_rgb[3 * pix + 2] = (float)fma((double)T, (double)th.bg[2], C2);
    out_T[pix] = T;
    out_nc[pix] = last;
    if (out_ne) out_ne[pix] = nev;
  }
}

gut_status launch_render(const DevCam& cam, const Thresholds& th, int n, int cam_idx,
                         const uint32_t* ranges, const uint32_t* ids, const float* record,
                         const float* rgb, float* out_rgb, float* out_T, uint32_t* out_nc,
                         uint32_t* out_ne, hipStream_t s) {
  dim3 grid(cam.tiles_x * cam.tiles_y), block(kTilePix);
  if (cam.shutter == GUT_ROLLING_TOP_TO_BOTTOM)
    render_kernel<true><<<grid, block, 0, s>>>(cam, th, n, cam_idx, (const uint2*)ranges, ids,
                                               (const float4*)record, rgb, out_rgb, out_T, out_nc,
                                               out_ne);
  else
    render_kernel<false><<<grid, block, 0, s>>>(cam, th, n, cam_idx, (const uint2*)ranges, ids,
                                                (const float4*)record, rgb, out_rgb, out_T, out_nc,
                                                out_ne);
  GUT_LAUNCH_CHECK();
  return GUT_OK;
}

}  // namespace gut

using namespace gut;

extern "C" gut_status gut_render(const gut_projected* proj, int64_t n, const uint32_t* tile_ranges,
                                 const uint32_t* sorted_ids, const gut_camera* cams, int32_t n_cams,
                                 const gut_params* p, float* rgb, float* T_final,
                                 uint32_t* n_contrib, uint32_t* n_eval, void* stream) {
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
  if ((st = prepare_cams(cams, n_cams, *p, dc, nullptr, nullptr)) != GUT_OK) return st;
  Thresholds th = make_thresholds(*p);
  for (int c = 0; c < n_cams; c++) {
    st = launch_render(dc[c], th, (int)n, c, tile_ranges, sorted_ids, proj->record, proj->rgb, rgb,
                       T_final, n_contrib, n_eval, (hipStream_t)stream);
    if (st != GUT_OK) return st;
  }
  return GUT_OK;
}
