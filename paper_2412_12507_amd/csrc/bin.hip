// Tile binning: the global per-tile depth sort of Sec. 4.3, with the tile
// culling of 3DGS and StopThePop that Sec. 4.1 and 4.4 name.
//
// Every (tile, entry) pair whose tile lies in the entry's rectangle -- and,
// with tile culling, meets the entry's extent ellipse -- goes into that
// tile's list, and each list is ordered by (depth, entry id).  Instead of a
// global sort of all pairs by a (tile, depth) key, the lists are built by a
// counting sort over tiles followed by one small sort per list:
//   K1 bin_count_kernel     each block of up to 8192 entries (128 units of 64
//                           neighbouring ones, strided over the camera)
//                           counts its pairs per tile in LDS and writes the
//                           counts as one row of a (block x tile) matrix
//   K2 bin_colscan_kernel   per tile, the exclusive prefix of its column (the
//                           block's offset inside the tile's list) and the
//                           tile's count
//   K3 bin_scan_kernel      per camera: the list starts, the render order
//                           (longest lists first), how many lists are long,
//                           and the pair total P (to the host: the one wait)
//   K4 bin_scatter_kernel   each block writes its pairs' 64-bit keys (depth
//                           bits << 32 | entry id) at its offsets in the lists
//   K5 tile_sort_*_kernel   per list, in LDS: a bucket sort on the highest
//                           bits that vary within it with a direct rank
//                           count inside each bucket; one wave per list
//                           below 1024 entries, 256 threads up to 4095, 1024
//                           threads beyond (cutting lists over 16384 into
//                           runs first); lists with a large bucket take a
//                           stable LSD radix sort instead
// Nothing needs a device-wide atomic per pair or per touched tile: blocks on
// different XCDs meet only in the count matrix, whose columns K2 scans.
// The (depth bits, id) key orders exactly as a full (tile, depth, id) sort
// would: depths are non-negative, so their bits order as the floats do.
#include <algorithm>
#include <cstring>

#include "common.h"

namespace gut {

struct CamTiles {
  int base[kMaxCams];
  int tx[kMaxCams];
  int count[kMaxCams];
};

static size_t al(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kBinThreads = 1024;
constexpr int kBinItems = 8;
constexpr int kBinChunk = kBinThreads * kBinItems;  // entries per block, at most
constexpr int kLdsTiles = 16000;  // tiles counted in LDS at once (64 KB); larger cameras go in windows

// Small per-call values after the count matrix: per-camera pair totals, the
// total P, per camera the number of lists of at least 4096 and of at least
// 1024 entries (the front of its render order), and the number of short
// lists left to the radix sort; then that list of tiles (u32 [T]).
struct SmallLayout {
  static constexpr size_t cam_pairs = 0;                     // u64 [kMaxCams]
  static constexpr size_t total = cam_pairs + 8 * kMaxCams;  // u64
  static constexpr size_t nbig = total + 256;                // u32 [kMaxCams]
  static constexpr size_t nmid = nbig + 4 * kMaxCams;        // u32 [kMaxCams]
  static constexpr size_t nfall = nmid + 4 * kMaxCams;       // u32
  static constexpr size_t bytes = nfall + 256;
};
constexpr size_t kSmallBytes = 4096;
static_assert(SmallLayout::bytes <= kSmallBytes, "small workspace");

static int64_t blocks_per_cam(int64_t n) { return n > 0 ? (n + kBinChunk - 1) / kBinChunk : 0; }

// Count phase: the (block x tile) matrix (blocks_per_cam x tiles of every
// camera, u32), the small values and the radix sort's list of tiles.
size_t bin_count_bytes(int64_t n, int64_t T) {
  return al((size_t)(blocks_per_cam(n) * T) * 4) + kSmallBytes + al((size_t)T * 4);
}
// Pair phase: the pairs' keys and a ping-pong copy for lists longer than one
// LDS chunk.
size_t bin_pair_bytes(int64_t cap) { return 2 * al((size_t)(cap > 0 ? cap : 1) * 8); }

// --------------------------------------------------------------- culling

// The tiles of one entry, row by row.  Without culling a row takes every
// column of the rectangle.  With culling it takes the columns whose tiles
// meet the extent ellipse (v - m)^T A^-1 (v - m) <= 1, A = k^2 Sigma': within
// the horizontal band of tile row ty the ellipse spans x from its left
// boundary at height yl to its right boundary at height yr, where yr is the
// height of the ellipse's rightmost point clamped into the band (the right
// boundary is concave in y) and yl likewise for the leftmost point.  The
// ellipse comes in FP32 from the projection; the geometry runs in FP64.
struct RowCull {
  double vx, vy, ylo, yhi, yR, yL, slope, wfac, inv_c;
  bool on;
};

__device__ inline RowCull row_cull_setup(bool cull, const float2* __restrict__ mean2d,
                                         const float4* __restrict__ extent, int64_t e) {
  RowCull rc;
  rc.on = false;
  if (!cull) return rc;
  const float2 m = mean2d[e];
  const float4 A = extent[e];
  const double a = A.x, b = A.y, c = A.z;
  const double det = a * c - b * b;
  if (!(det > 0.0) || !(a > 0.0) || !(c > 0.0)) return rc;  // degenerate: the whole rectangle
  const double sa = sqrt(a), sc = sqrt(c);
  rc.vx = m.x;
  rc.vy = m.y;
  rc.ylo = rc.vy - sc;
  rc.yhi = rc.vy + sc;
  rc.yR = rc.vy + b / sa;
  rc.yL = rc.vy - b / sa;
  rc.slope = b / c;
  rc.wfac = det / c;
  rc.inv_c = 1.0 / c;
  rc.on = true;
  return rc;
}

// Columns [*c0, *c1] of tile row ty kept for the entry (empty if *c0 > *c1),
// inside the rectangle's columns [x0, x1].
__device__ inline void row_cull_range(const RowCull& rc, int ty, int x0, int x1, int* c0, int* c1) {
  if (!rc.on) {
    *c0 = x0;
    *c1 = x1;
    return;
  }
  const double Y0 = (double)ty * kTile, Y1 = Y0 + kTile;
  const double lo = fmax(Y0, rc.ylo), hi = fmin(Y1, rc.yhi);
  if (lo > hi) {
    *c0 = 1;
    *c1 = 0;
    return;
  }
  const double yr = fmin(fmax(rc.yR, lo), hi), dr = yr - rc.vy;
  const double xr = rc.vx + rc.slope * dr + sqrt(fmax(0.0, rc.wfac * (1.0 - dr * dr * rc.inv_c)));
  const double yl = fmin(fmax(rc.yL, lo), hi), dl = yl - rc.vy;
  const double xl = rc.vx + rc.slope * dl - sqrt(fmax(0.0, rc.wfac * (1.0 - dl * dl * rc.inv_c)));
  const double inv_t = 1.0 / kTile;
  *c0 = max(x0, (int)fmax(floor(xl * inv_t), -1.0));
  *c1 = min(x1, (int)fmin(floor(xr * inv_t), 1e9));
}

// Calls f(ty, c0, c1) for each tile row ty of the entry inside the row window
// [w0, w1) whose kept columns [c0, c1] are not empty.  The rows are visited
// from the rot-th one on, cyclically: lanes of a wave walking similar
// entries (neighbouring ids are often neighbours in space) then work on
// different rows at each step instead of piling onto the same LDS words.
template <class F>
__device__ inline void for_each_row(int64_t e, const short4* __restrict__ rect, bool cull,
                                    const float2* __restrict__ mean2d, const float4* __restrict__ extent,
                                    int w0, int w1, int rot, F&& f) {
  const short4 r = rect[e];
  const int ty0 = max((int)r.y, w0), ty1 = min((int)r.w, w1 - 1);
  if (ty0 > ty1) return;
  const RowCull rc = row_cull_setup(cull, mean2d, extent, e);
  const int nr = ty1 - ty0 + 1;
  int k = rot % nr;
  for (int j = 0; j < nr; j++) {
    const int ty = ty0 + k;
    k = k + 1 == nr ? 0 : k + 1;
    int c0, c1;
    row_cull_range(rc, ty, r.x, r.z, &c0, &c1);
    if (c0 <= c1) f(ty, c0, c1);
  }
}

// ------------------------------------------------------ count and scatter

struct BinArgs {
  const short4* rect;
  const uint32_t* tiles;
  const float* depth;
  const float2* mean2d;
  const float4* extent;
  int n;     // particles (entries per camera)
  int bpc;   // blocks per camera
  int cull;  // tile culling on
  int n_cams;
  CamTiles ct;
};

// Entries go to blocks in units of 64 consecutive ones (one per wave
// lane): block b of a camera owns its units b, b + bpc, b + 2 bpc, ...  so
// that the dense clusters of a scene, which hold runs of neighbouring entry
// ids, spread over all blocks.  Inside a block the waves claim the block's
// units one at a time from an LDS counter until none is left, which evens out
// their work.
__device__ inline int units_of_block(int n, int bpc, int b) {
  const int nu = (n + 63) / 64;
  return nu > b ? (nu - 1 - b) / bpc + 1 : 0;
}

// Claims the wave's next unit; returns its index among the block's units.
__device__ inline int claim_unit(int* next) {
  int k = 0;
  if ((threadIdx.x & 63) == 0) k = atomicAdd(next, 1);
  return __shfl(k, 0, 64);
}

// Tile rows of a camera whose tiles fit the LDS at once (with one spare
// column per row for the count kernel's difference arrays).
// Camera widths stay below 4096 tiles, so a window holds at least 3 rows.
__host__ __device__ inline int window_rows(int txc, int tyc) {
  const int r = kLdsTiles / (txc + 1);
  return tyc < r ? tyc : r;
}

// In-place inclusive prefix sums of rows of txc words (row stride `stride`)
// in LDS, one wave per row.
__device__ inline void lds_row_scan(uint32_t* h, int nrow, int txc, int stride) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int q = (txc + 63) / 64;  // consecutive columns per lane
  for (int r = w; r < nrow; r += nw) {
    uint32_t* row = h + r * stride;
    const int c0 = lane * q;
    uint32_t sum = 0;
    for (int c = c0; c < min(c0 + q, txc); c++) sum += row[c];
    uint32_t x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    uint32_t run = x - sum;
    for (int c = c0; c < min(c0 + q, txc); c++) {
      run += row[c];
      row[c] = run;
    }
  }
}

// K1: one row of the count matrix per block (camera c, the units of it that
// the block owns).  Each visible entry adds, per
// tile row, +1 at its first kept column and -1 after its last to an LDS
// difference array of the camera's tiles (in windows of tile rows); prefix
// sums along the rows then give the counts.
__global__ void __launch_bounds__(kBinThreads) bin_count_kernel(BinArgs a, uint32_t* __restrict__ M) {
  extern __shared__ uint32_t h[];
  __shared__ int next;
  const int c = blockIdx.x / a.bpc, b = blockIdx.x % a.bpc;
  const int txc = a.ct.tx[c], Tc = a.ct.count[c], tyc = Tc / txc, S = txc + 1;
  const int64_t e0 = (int64_t)c * a.n;
  const int lane = threadIdx.x & 63, nub = units_of_block(a.n, a.bpc, b);
  uint32_t* row = M + (int64_t)a.bpc * a.ct.base[c] + (int64_t)b * Tc;
  const int RW = window_rows(txc, tyc);
  for (int w0 = 0; w0 < tyc; w0 += RW) {
    const int nrow = min(RW, tyc - w0);
    for (int i = threadIdx.x; i < nrow * S; i += kBinThreads) h[i] = 0u;
    if (threadIdx.x == 0) next = 0;
    __syncthreads();
    for (int k = claim_unit(&next); k < nub; k = claim_unit(&next)) {
      const int i = (b + k * a.bpc) * 64 + lane;
      if (i < a.n && a.tiles[e0 + i] != 0u)
        for_each_row(e0 + i, a.rect, a.cull, a.mean2d, a.extent, w0, w0 + nrow, lane, [&](int ty, int c0, int c1) {
          uint32_t* hr = h + (ty - w0) * S;
          atomicAdd(&hr[c0], 1u);
          atomicAdd(&hr[c1 + 1], ~0u);  // -1
        });
    }
    __syncthreads();
    lds_row_scan(h, nrow, txc, S);
    __syncthreads();
    for (int r = threadIdx.x >> 6; r < nrow; r += kBinThreads / 64)
      for (int x = lane; x < txc; x += 64) row[(w0 + r) * txc + x] = h[r * S + x];
    __syncthreads();
  }
}

// K2: for each tile, the exclusive prefix of its column of the count matrix,
// in place, and its count into ranges[t].y; each block adds its tiles'
// counts to their cameras' totals (one atomic per camera a block touches; the
// totals start at zero from the init kernel).  A block takes 32 tiles, and
// each tile's column is cut into kColSegs segments of rows, one per thread:
// a thread sums its segment, the segments' sums are scanned in LDS, and the
// thread writes its segment's prefixes, so a long column (many blocks of
// entries) is not walked by one thread alone.
constexpr int kColThreads = 256;
constexpr int kColTiles = 32;
constexpr int kColSegs = kColThreads / kColTiles;
constexpr int kColUnroll = 4;
__global__ void __launch_bounds__(kColThreads) bin_colscan_kernel(uint32_t* __restrict__ M, CamTiles ct,
                                                                  int n_cams, int bpc, int64_t T,
                                                                  uint2* __restrict__ ranges,
                                                                  unsigned long long* __restrict__ cam_pairs) {
  __shared__ unsigned long long cs[kMaxCams];
  __shared__ uint32_t ssum[kColSegs][kColTiles];
  const int tl = threadIdx.x % kColTiles, seg = threadIdx.x / kColTiles;
  const int64_t g = (int64_t)blockIdx.x * kColTiles + tl;
  if (threadIdx.x < kMaxCams) cs[threadIdx.x] = 0ull;
  const int chunk = (bpc + kColSegs - 1) / kColSegs;
  const int r0 = min(bpc, seg * chunk), r1 = min(bpc, r0 + chunk);
  int c = 0;
  uint32_t* col = nullptr;
  int Tc = 0;
  uint32_t sum = 0;
  if (g < T) {
    while (c + 1 < n_cams && ct.base[c + 1] <= g) c++;
    Tc = ct.count[c];
    col = M + (int64_t)bpc * ct.base[c] + (g - ct.base[c]);
    for (int r = r0; r < r1; r += kColUnroll) {
      uint32_t v[kColUnroll];
#pragma unroll
      for (int k = 0; k < kColUnroll; k++) v[k] = r + k < r1 ? col[(int64_t)(r + k) * Tc] : 0u;
#pragma unroll
      for (int k = 0; k < kColUnroll; k++) sum += v[k];
    }
  }
  ssum[seg][tl] = sum;
  __syncthreads();
  uint32_t run = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kColSegs; k++) {
    const uint32_t x = ssum[k][tl];
    if (k < seg) run += x;
    tot += x;
  }
  if (g < T) {
    for (int r = r0; r < r1; r += kColUnroll) {
      uint32_t v[kColUnroll];
#pragma unroll
      for (int k = 0; k < kColUnroll; k++) v[k] = r + k < r1 ? col[(int64_t)(r + k) * Tc] : 0u;
#pragma unroll
      for (int k = 0; k < kColUnroll; k++) {
        if (r + k < r1) col[(int64_t)(r + k) * Tc] = run;
        run += v[k];
      }
    }
    if (seg == 0) {
      ranges[g].y = tot;
      atomicAdd(&cs[c], (unsigned long long)tot);
    }
  }
  __syncthreads();
  if (threadIdx.x < n_cams && cs[threadIdx.x]) atomicAdd(&cam_pairs[threadIdx.x], cs[threadIdx.x]);
}

// Clears the per-camera totals K2 adds into and the count of lists left to
// the radix sort.
__global__ void bin_init_kernel(unsigned long long* __restrict__ sw) {
  if (threadIdx.x < kMaxCams) sw[SmallLayout::cam_pairs / 8 + threadIdx.x] = 0ull;
  if (threadIdx.x == 0) *(uint32_t*)((char*)sw + SmallLayout::nfall) = 0u;
}

// K4: each pair's key at its place: the tile's list start plus the block's
// offset in the tile (the column prefix) plus its rank among the block's
// pairs of that tile (an LDS counter; the order inside a block is arbitrary
// and fixed by K5).  Writes nothing when P exceeds the capacity.
__global__ void __launch_bounds__(kBinThreads) bin_scatter_kernel(BinArgs a, const uint32_t* __restrict__ M,
                                                                  const uint2* __restrict__ ranges,
                                                                  const unsigned long long* __restrict__ P_dev,
                                                                  unsigned long long cap,
                                                                  unsigned long long* __restrict__ keys) {
  extern __shared__ uint32_t h[];
  __shared__ int next;
  if (*P_dev > cap) return;
  const int c = blockIdx.x / a.bpc, b = blockIdx.x % a.bpc;
  const int base = a.ct.base[c], txc = a.ct.tx[c], Tc = a.ct.count[c], tyc = Tc / txc;
  const int64_t e0 = (int64_t)c * a.n;
  const int lane = threadIdx.x & 63, nub = units_of_block(a.n, a.bpc, b);
  const uint32_t* row = M + (int64_t)a.bpc * base + (int64_t)b * Tc;
  const int RW = window_rows(txc, tyc);
  for (int w0 = 0; w0 < tyc; w0 += RW) {
    const int nrow = min(RW, tyc - w0), t0 = w0 * txc;
    for (int i = threadIdx.x; i < nrow * txc; i += kBinThreads) h[i] = ranges[base + t0 + i].x + row[t0 + i];
    if (threadIdx.x == 0) next = 0;
    __syncthreads();
    for (int k = claim_unit(&next); k < nub; k = claim_unit(&next)) {
      const int i = (b + k * a.bpc) * 64 + lane;
      if (!(i < a.n && a.tiles[e0 + i] != 0u)) continue;
      const int64_t e = e0 + i;
      const unsigned long long key = ((unsigned long long)__float_as_uint(a.depth[e]) << 32) | (uint32_t)e;
      for_each_row(e, a.rect, a.cull, a.mean2d, a.extent, w0, w0 + nrow, lane, [&](int ty, int c0, int c1) {
        uint32_t* hr = h + (ty - w0) * txc;
        // four reservations in flight at a time; K1 counted the same tiles,
        // so every slot lies below P <= cap
        for (int x = c0; x <= c1; x += 4) {
          uint32_t sl[4];
#pragma unroll
          for (int j = 0; j < 4; j++) sl[j] = x + j <= c1 ? atomicAdd(&hr[x + j], 1u) : 0xffffffffu;
#pragma unroll
          for (int j = 0; j < 4; j++)
            if (sl[j] < cap) keys[sl[j]] = key;
        }
      });
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ scan

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 16;
constexpr int kMidBucket = 21;  // __clz of lengths >= 1024 is at most 21
constexpr int kBigBucket = 19;  // __clz of lengths >= 4096 is at most 19

__device__ inline uint32_t block_scan_1024(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kScanThreads / 64; k++) {
    const uint32_t s = wsum[k];
    if (k < w) pre += s;
    tot += s;
  }
  *total = tot;
  return pre + x - v;
}

// K3, one block per camera: the lists' [start, end) (global over the
// cameras), the render order of the camera's tiles (a counting sort by the
// bit length of the list length, longest first; within a bucket the order
// may vary from call to call), the number of lists of at least 4096 and of
// at least 1024 entries (the front of that order), and from the last
// camera's block the total P for the device and the host (with each
// camera's count of long lists).
__global__ void __launch_bounds__(kScanThreads) bin_scan_kernel(uint2* __restrict__ ranges,
                                                                uint32_t* __restrict__ order, CamTiles ct,
                                                                int n_cams, unsigned long long* __restrict__ sw,
                                                                void* host) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  __shared__ unsigned bcnt[33], bcur[33];
  const int c = blockIdx.x, t = threadIdx.x;
  const int base = ct.base[c], Tc = ct.count[c];
  unsigned long long off = 0;
  for (int k = 0; k < c; k++) off += sw[SmallLayout::cam_pairs / 8 + k];
  if (c == n_cams - 1 && t == 0) {
    const unsigned long long P = off + sw[SmallLayout::cam_pairs / 8 + c];
    sw[SmallLayout::total / 8] = P;
    volatile uint32_t* hp = (volatile uint32_t*)host;
    hp[0] = (uint32_t)P;
    hp[1] = (uint32_t)(P >> 32);
  }
  if (t < 33) bcnt[t] = 0u;
  __syncthreads();
  uint32_t carry = (uint32_t)off;
  for (int p0 = 0; p0 < Tc; p0 += kScanThreads * kScanItems) {
    const int len = min(Tc - p0, kScanThreads * kScanItems);
    const int q = (len + kScanThreads - 1) / kScanThreads;
    const int b0 = p0 + t * q;
    uint32_t v[kScanItems], sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
      const bool in = i < q && b0 + i < p0 + len;
      v[i] = in ? ranges[base + b0 + i].y : 0u;
      if (in) atomicAdd(&bcnt[__clz(v[i])], 1u);
      sum += v[i];
    }
    uint32_t total;
    uint32_t run = carry + block_scan_1024(sum, wsum, &total);
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
      if (i < q && b0 + i < p0 + len) ranges[base + b0 + i] = make_uint2(run, run + v[i]);
      run += v[i];
    }
    carry += total;
    __syncthreads();  // wsum is reused by the next piece
  }
  if (t == 0) {
    unsigned acc = 0, big = 0, mid = 0;
    for (int b = 0; b < 33; b++) {
      bcur[b] = acc;
      acc += bcnt[b];
      if (b <= kBigBucket) big += bcnt[b];
      if (b <= kMidBucket) mid += bcnt[b];
    }
    uint32_t* nb = (uint32_t*)((char*)sw + SmallLayout::nbig);
    uint32_t* nm = (uint32_t*)((char*)sw + SmallLayout::nmid);
    nb[c] = big;
    nm[c] = mid;
    ((volatile uint32_t*)host)[2 + c] = big;  // for the host: whether the long-list sort has work
  }
  __syncthreads();
  for (int j = t; j < Tc; j += kScanThreads) {
    const uint2 r = ranges[base + j];  // written before the barrier above
    const unsigned pos = atomicAdd(&bcur[__clz(r.y - r.x)], 1u);
    order[base + pos] = (uint32_t)j;
  }
}

// ------------------------------------------------------------- list sort

constexpr int kTSItems = 16;      // keys per thread in one LDS chunk
constexpr uint32_t kTieRun = 32;  // longer runs of equal depth take the full sort

// LDS of one sorting block of NT threads: a chunk of NT * 16 keys.
template <int NT>
struct TileSortSmem {
  static constexpr int W = NT / 64;
  unsigned long long stage[NT * kTSItems];
  uint32_t wh[W][256];  // per-wave running digit counts, then wave prefixes
  uint32_t lstart[256];  // start of digit d's run in the chunk
  uint32_t dcnt[256];    // digit d's count in the chunk
  uint32_t dbase[256];   // (lists over one chunk) next output position of digit d
  uint32_t wsum[4];
  unsigned long long wor[W];
  uint32_t flag;
};

// Chunk position of item r of this thread: wave-major, then item, then lane.
__device__ inline int ts_pos(int r) {
  return (int)(threadIdx.x >> 6) * (64 * kTSItems) + r * 64 + (int)(threadIdx.x & 63);
}

__device__ inline uint32_t ts_digit(const uint32_t (&dg)[kTSItems / 4], int r) {
  return (dg[r >> 2] >> (8 * (r & 3))) & 255u;
}

// Per digit: the per-wave counts in S.wh become exclusive prefixes over the
// waves, S.dcnt the chunk's counts and S.lstart their exclusive prefix
// (thread t handles digits [t Q, t Q + Q)).
template <int NT>
__device__ inline void digit_prefix(TileSortSmem<NT>& S) {
  constexpr int W = NT / 64, Q = NT >= 256 ? 1 : 256 / NT, NS = 256 / Q;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  uint32_t cnt[Q], tot = 0;
#pragma unroll
  for (int q = 0; q < Q; q++) cnt[q] = 0u;
  if (t < NS) {
#pragma unroll
    for (int q = 0; q < Q; q++) {
      const int d = t * Q + q;
      uint32_t sum = 0;
#pragma unroll
      for (int k = 0; k < W; k++) {
        const uint32_t v = S.wh[k][d];
        S.wh[k][d] = sum;
        sum += v;
      }
      S.dcnt[d] = sum;
      cnt[q] = sum;
      tot += sum;
    }
  }
  uint32_t x = tot;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (t < NS && lane == 63) S.wsum[w] = x;
  __syncthreads();
  if (t < NS) {
    uint32_t run = x - tot;
    for (int k = 0; k < w; k++) run += S.wsum[k];
#pragma unroll
    for (int q = 0; q < Q; q++) {
      S.lstart[t * Q + q] = run;
      run += cnt[q];
    }
  }
  __syncthreads();
}

// Stable rank of the chunk's valid items by their digits (item r's digit is
// byte r & 3 of dg[r >> 2]): within a wave with ballot peer masks and
// per-wave running digit counts, across waves by the per-digit wave
// prefixes.  Leaves the start and count of each digit's run in S.lstart /
// S.dcnt and returns each item's place in the chunk's digit order.  Item
// rows with no valid item are skipped (the check is uniform per wave).
template <int NT>
__device__ inline void chunk_rank(const uint32_t (&dg)[kTSItems / 4], uint32_t vmask, uint32_t (&lp)[kTSItems],
                                  TileSortSmem<NT>& S) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int d = lane; d < 256; d += 64) S.wh[w][d] = 0u;
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < kTSItems; r++) {
    const bool valid = (vmask >> r) & 1u;
    lp[r] = 0u;
    unsigned long long peers = __ballot(valid);
    if (peers == 0ull) continue;
    const uint32_t d = ts_digit(dg, r);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t before = (uint32_t)__popcll(peers & lt);
    const uint32_t run = valid ? S.wh[w][d] : 0u;
    if (valid && before == 0) S.wh[w][d] = run + (uint32_t)__popcll(peers);
    lp[r] = run + before;  // rank within the wave's items of digit d so far
  }
  __syncthreads();
  digit_prefix<NT>(S);
#pragma unroll
  for (int r = 0; r < kTSItems; r++) {
    if (!((vmask >> r) & 1u)) continue;
    const uint32_t d = ts_digit(dg, r);
    lp[r] += S.lstart[d] + S.wh[w][d];
  }
}

__device__ inline void ts_digits(const unsigned long long (&kk)[kTSItems], int shift,
                                 uint32_t (&dg)[kTSItems / 4]) {
#pragma unroll
  for (int q = 0; q < kTSItems / 4; q++) {
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) v |= ((uint32_t)(kk[4 * q + j] >> shift) & 255u) << (8 * j);
    dg[q] = v;
  }
}

// OR over the block.
template <int NT>
__device__ inline unsigned long long block_or(unsigned long long x, TileSortSmem<NT>& S) {
  for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
  if ((threadIdx.x & 63) == 0) S.wor[threadIdx.x >> 6] = x;
  __syncthreads();
  unsigned long long m = 0;
#pragma unroll
  for (int k = 0; k < TileSortSmem<NT>::W; k++) m |= S.wor[k];
  __syncthreads();
  return m;
}

// One LSD pass over the byte at `shift` of the chunk's keys (registers, in
// chunk positions); leaves them in their new order in kk.
template <int NT>
__device__ inline void lds_pass(unsigned long long (&kk)[kTSItems], uint32_t vmask, int shift,
                                TileSortSmem<NT>& S) {
  uint32_t dg[kTSItems / 4], lp[kTSItems];
  ts_digits(kk, shift, dg);
  chunk_rank<NT>(dg, vmask, lp, S);
#pragma unroll
  for (int r = 0; r < kTSItems; r++)
    if ((vmask >> r) & 1u) S.stage[lp[r]] = kk[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kTSItems; r++)
    if ((vmask >> r) & 1u) kk[r] = S.stage[ts_pos(r)];
  __syncthreads();
}

// Sorts one list of L <= NT * 16 keys in LDS and writes its entry ids.  The
// passes cover only the depth bytes that vary within the list, which orders
// it by depth; runs of equal depth (rare) are then put in entry-id order by
// the thread that owns their first key, or, if a run is longer than
// kTieRun, the list is sorted again over every varying byte.
template <int NT>
__device__ __forceinline__ void sort_list_lds(const unsigned long long* __restrict__ keys, uint32_t L,
                                     uint32_t* __restrict__ ids, TileSortSmem<NT>& S) {
  unsigned long long kk[kTSItems];
  uint32_t vmask = 0;
  const unsigned long long k0 = keys[0];
  unsigned long long orv = 0;
#pragma unroll
  for (int r = 0; r < kTSItems; r++) {
    const int p = ts_pos(r);
    const bool v = (uint32_t)p < L;
    kk[r] = v ? keys[p] : 0ull;
    vmask |= (uint32_t)v << r;
    if (v) orv |= kk[r] ^ k0;
  }
  const unsigned long long mask = block_or<NT>(orv, S);
  for (int shift = 32; shift < 64; shift += 8)
    if ((mask >> shift) & 255ull) lds_pass<NT>(kk, vmask, shift, S);
  // the depth-sorted keys in LDS (also when no pass ran), then the ties
#pragma unroll
  for (int r = 0; r < kTSItems; r++)
    if ((vmask >> r) & 1u) S.stage[ts_pos(r)] = kk[r];
  if (threadIdx.x == 0) S.flag = 0u;
  __syncthreads();
  bool tie = false;
#pragma unroll
  for (int r = 0; r < kTSItems; r++) {
    const uint32_t p = (uint32_t)ts_pos(r);
    if (p + 1 < L && (S.stage[p] >> 32) == (S.stage[p + 1] >> 32)) tie = true;
  }
  if (__syncthreads_or(tie)) {
#pragma unroll
    for (int r = 0; r < kTSItems; r++) {
      const uint32_t p = (uint32_t)ts_pos(r);
      if (p + 1 >= L) continue;
      const unsigned long long d = S.stage[p] >> 32;
      if ((S.stage[p + 1] >> 32) != d || (p > 0 && (S.stage[p - 1] >> 32) == d)) continue;
      uint32_t q = p + 1;  // the run of depth d is [p, q)
      while (q < L && (S.stage[q] >> 32) == d) q++;
      if (q - p > kTieRun) {
        S.flag = 1u;
        continue;
      }
      for (uint32_t i = p + 1; i < q; i++) {  // insertion sort by the whole key (the ids)
        const unsigned long long x = S.stage[i];
        uint32_t j = i;
        while (j > p && S.stage[j - 1] > x) {
          S.stage[j] = S.stage[j - 1];
          j--;
        }
        S.stage[j] = x;
      }
    }
    __syncthreads();
    if (S.flag) {  // long runs of equal depth: sort again over every varying byte
#pragma unroll
      for (int r = 0; r < kTSItems; r++)
        if ((vmask >> r) & 1u) kk[r] = S.stage[ts_pos(r)];
      __syncthreads();
      for (int shift = 0; shift < 64; shift += 8)
        if ((mask >> shift) & 255ull) lds_pass<NT>(kk, vmask, shift, S);
#pragma unroll
      for (int r = 0; r < kTSItems; r++)
        if ((vmask >> r) & 1u) S.stage[ts_pos(r)] = kk[r];
      __syncthreads();
    }
  }
#pragma unroll
  for (int r = 0; r < kTSItems; r++) {
    const int p = ts_pos(r);
    if ((vmask >> r) & 1u) ids[p] = (uint32_t)S.stage[p];
  }
}

// Sorts one list longer than a chunk over every byte that varies within it:
// per byte, a histogram over all its chunks, then the chunks in order, each
// ranked in LDS and written to its digit's next positions (stable across
// chunks), ping-ponging between src and tmp; the last pass writes the entry
// ids.  The chunk's keys wait in LDS while their digits are ranked.
template <int NT>
__device__ __forceinline__ void sort_list_chunked(unsigned long long* __restrict__ src, unsigned long long* __restrict__ tmp,
                                         uint32_t L, uint32_t* __restrict__ ids, TileSortSmem<NT>& S) {
  constexpr uint32_t CH = NT * kTSItems;
  const int t = threadIdx.x;
  const unsigned long long k0 = src[0];
  unsigned long long orv = 0;
  for (uint32_t c0 = 0; c0 < L; c0 += CH)
#pragma unroll
    for (int r = 0; r < kTSItems; r++) {
      const uint32_t p = c0 + (uint32_t)ts_pos(r);
      if (p < L) orv |= src[p] ^ k0;
    }
  const unsigned long long mask = block_or<NT>(orv, S);
  int last = -1;
  for (int shift = 0; shift < 64; shift += 8)
    if ((mask >> shift) & 255ull) last = shift;
  if (last < 0) {  // all keys equal (cannot happen for distinct entries)
    for (uint32_t p = t; p < L; p += NT) ids[p] = (uint32_t)src[p];
    return;
  }
  unsigned long long *a = src, *b = tmp;
  for (int shift = 0; shift <= last; shift += 8) {
    if (!((mask >> shift) & 255ull)) continue;
    if (t < 256) S.dbase[t] = 0u;
    __syncthreads();
    for (uint32_t c0 = 0; c0 < L; c0 += CH)
#pragma unroll
      for (int r = 0; r < kTSItems; r++) {
        const uint32_t p = c0 + (uint32_t)ts_pos(r);
        if (p < L) atomicAdd(&S.dbase[(uint32_t)(a[p] >> shift) & 255u], 1u);
      }
    __syncthreads();
    // exclusive prefix of the histogram (S.wh[0] is free here)
    if (t < 256) S.wh[0][t] = S.dbase[t];
    __syncthreads();
    if (t == 0) {
      uint32_t run = 0;
      for (int d = 0; d < 256; d++) {
        S.dbase[d] = run;
        run += S.wh[0][d];
      }
    }
    __syncthreads();
    const bool final_pass = shift == last;
    for (uint32_t c0 = 0; c0 < L; c0 += CH) {
      uint32_t vmask = 0, lp[kTSItems], dg[kTSItems / 4] = {};
#pragma unroll
      for (int r = 0; r < kTSItems; r++) {
        const uint32_t p = c0 + (uint32_t)ts_pos(r);
        const bool v = p < L;
        const unsigned long long k = v ? a[p] : 0ull;
        S.stage[ts_pos(r)] = k;
        dg[r >> 2] |= ((uint32_t)(k >> shift) & 255u) << (8 * (r & 3));
        vmask |= (uint32_t)v << r;
      }
      chunk_rank<NT>(dg, vmask, lp, S);
#pragma unroll
      for (int r = 0; r < kTSItems; r++) {
        if (!((vmask >> r) & 1u)) continue;
        const uint32_t d = ts_digit(dg, r);
        const unsigned long long k = S.stage[ts_pos(r)];
        const uint32_t pos = S.dbase[d] + (lp[r] - S.lstart[d]);
        if (final_pass) ids[pos] = (uint32_t)k;
        else b[pos] = k;
      }
      __syncthreads();
      if (t < 256) S.dbase[t] += S.dcnt[t];
      __syncthreads();
    }
    unsigned long long* sw = a;
    a = b;
    b = sw;
  }
}

// Bucket sort of one list, the common path.  The keys of a list agree on
// every bit above the highest one that varies within it, so the next db
// bits from there down, taken as a digit, order the keys (coarsely) as the
// keys themselves do.  The keys are counted per digit, moved into their
// digit's bucket in LDS (in any order inside it), and each key's place in
// the list is its bucket's start plus the number of keys of its bucket below
// it: a direct comparison of the whole (depth, id) keys, so equal depths
// need no second step.  db grows with the list: depths inside a tile bunch
// up, so the buckets need to be much finer than L to stay small.  When a
// bucket holds more than kBucketMax keys (the comparisons would cost more
// than a radix sort) the sort gives up before touching ids, and the list
// goes to the radix sort.
constexpr uint32_t kBucketMax = 64;

// A block of NT threads sorts one list of L <= NT ROWS keys with the bucket
// sort above: item r of thread t is list position NT r + t, the rows are
// unrolled and the rank counts run without branches, so that their LDS reads
// overlap.  nb = 2^db buckets, db two bits above the bit length of L, at most
// DBM; thread t owns the q = nb / NT consecutive digits from t q on (in the
// scan), kept at counter j NT + t for its j-th digit so that the scan's
// reads do not collide in the banks.  P16: the counters are 16-bit halves of
// 32-bit words (every count and position is at most L <= 65535), counted and
// claimed with word atomics that add 1 to one half, which halves their LDS.
template <int NT, int ROWS, int DBM, bool P16 = false>
struct BlockSortSmem {
  union {
    unsigned long long keys[NT * ROWS];
    struct {
      uint32_t wsum[NT / 64];
      uint32_t wmax[NT / 64];
      unsigned long long wor[NT / 64];
    } w;  // the waves' partials, read only before the keys move in
  };
  uint32_t cnt[P16 ? (1 << DBM) / 2 : (1 << DBM)];
};

template <bool P16>
__device__ inline uint32_t ctr_get(const uint32_t* c, uint32_t i) {
  return P16 ? (uint32_t)reinterpret_cast<const unsigned short*>(c)[i] : c[i];
}
template <bool P16>
__device__ inline void ctr_set(uint32_t* c, uint32_t i, uint32_t v) {
  if (P16) reinterpret_cast<unsigned short*>(c)[i] = (unsigned short)v;
  else c[i] = v;
}
// Adds 1 to counter i and returns its old value.
template <bool P16>
__device__ inline uint32_t ctr_inc(uint32_t* c, uint32_t i) {
  if (!P16) return atomicAdd(&c[i], 1u);
  const uint32_t sh = 16u * (i & 1u);
  return (atomicAdd(&c[i >> 1], 1u << sh) >> sh) & 0xffffu;
}

template <int NT, int ROWS, int DBM, bool P16>
__device__ __forceinline__ bool block_bucket_sort(const unsigned long long* __restrict__ keys, uint32_t L,
                                         uint32_t* __restrict__ ids, BlockSortSmem<NT, ROWS, DBM, P16>& S,
                                         uint32_t bucket_max = kBucketMax) {
  constexpr int W = NT / 64;
  constexpr int LNT = NT == 64 ? 6 : NT == 128 ? 7 : NT == 256 ? 8 : NT == 512 ? 9 : 10;
  constexpr int QM = (1 << DBM) / NT > 0 ? (1 << DBM) / NT : 1;  // most digits per thread
  static_assert((1 << LNT) == NT, "threads");
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  unsigned long long kk[ROWS];
  bool ok[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; r++) {
    const uint32_t p = (uint32_t)(r * NT + t);
    ok[r] = p < L;
    kk[r] = ok[r] ? keys[p] : 0ull;
  }
  const int db = min(DBM, 34 - __clz(L));  // bit length of L, plus two
  const uint32_t nb = 1u << db;
  const int lq = db > LNT ? db - LNT : 0;
  const uint32_t q = 1u << lq;  // digits per thread
  const bool own = (uint32_t)t < nb;  // thread owns digits (all once nb >= NT)
  // the bits that vary within the list (any of its keys is a reference)
  const unsigned long long k0 = keys[0];
  unsigned long long orv = 0;
#pragma unroll
  for (int r = 0; r < ROWS; r++) orv |= ok[r] ? kk[r] ^ k0 : 0ull;
  for (int o = 32; o > 0; o >>= 1) orv |= __shfl_xor(orv, o, 64);
  if (W > 1 && lane == 0) S.w.wor[w] = orv;
  for (uint32_t i = t; i < (P16 ? (nb + 1) / 2 : nb); i += NT) S.cnt[i] = 0u;
  __syncthreads();
  if (W > 1) {
    orv = 0;
#pragma unroll
    for (int k = 0; k < W; k++) orv |= S.w.wor[k];
  }
  const int hb = orv ? 63 - __clzll((long long)orv) : 0;
  const int shift = hb >= db - 1 ? hb - (db - 1) : 0;
  uint32_t sl[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; r++) {
    const uint32_t d = (uint32_t)(kk[r] >> shift) & (nb - 1);
    sl[r] = ((d & (q - 1)) << LNT) | (d >> lq);
  }
#pragma unroll
  for (int r = 0; r < ROWS; r++)
    if (ok[r]) (void)ctr_inc<P16>(S.cnt, sl[r]);
  __syncthreads();
  uint32_t c[QM], tot = 0, mx = 0;
#pragma unroll
  for (int j = 0; j < QM; j++) {
    c[j] = (uint32_t)j < q && own ? ctr_get<P16>(S.cnt, j * NT + t) : 0u;
    tot += c[j];
    mx = max(mx, c[j]);
  }
  uint32_t x = tot;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, o, 64));
  uint32_t run = x - tot;
  if (W > 1) {
    if (lane == 63) S.w.wsum[w] = x;
    if (lane == 0) S.w.wmax[w] = mx;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < W; k++) {
      if (k < w) run += S.w.wsum[k];
      mx = max(mx, S.w.wmax[k]);
    }
  }
  if (mx > bucket_max) {
    __syncthreads();  // every thread has read S before it is reused
    return false;
  }
#pragma unroll
  for (int j = 0; j < QM; j++) {
    if ((uint32_t)j < q && own) ctr_set<P16>(S.cnt, j * NT + t, run);
    run += c[j];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ROWS; r++)
    if (ok[r]) S.keys[ctr_inc<P16>(S.cnt, sl[r])] = kk[r];
  __syncthreads();
  // The counters now hold each bucket's end, which is the next bucket's
  // start.  The rank counts run over the keys in their bucket order (item r
  // of thread t is the key at place NT r + t of the moved list), so the 64
  // lanes of a wave mostly share a few neighbouring buckets and the count of
  // a row stops at the longest of those, not at the longest bucket that 64
  // keys from anywhere in the list would meet.
#pragma unroll
  for (int r = 0; r < ROWS; r++) kk[r] = ok[r] ? S.keys[r * NT + t] : 0ull;
  uint32_t base[ROWS], len[ROWS], most = 0;
#pragma unroll
  for (int r = 0; r < ROWS; r++) {
    const uint32_t d = (uint32_t)(kk[r] >> shift) & (nb - 1), dp = d ? d - 1 : 0u;
    const uint32_t e = ctr_get<P16>(S.cnt, ((d & (q - 1)) << LNT) | (d >> lq));
    const uint32_t s0 = ctr_get<P16>(S.cnt, ((dp & (q - 1)) << LNT) | (dp >> lq));
    base[r] = d ? s0 : 0u;
    len[r] = ok[r] ? e - base[r] : 0u;
    most = max(most, len[r]);
  }
  uint32_t rank[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; r++) rank[r] = base[r];
  if (ROWS * NT <= 4096) {
    // all rows advance together (their reads overlap), as far as the wave's
    // largest bucket
    for (int o = 32; o > 0; o >>= 1) most = max(most, (uint32_t)__shfl_xor(most, o, 64));
    for (uint32_t j = 0; j < most; j++)
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        const unsigned long long v = S.keys[min(base[r] + j, L - 1)];
        rank[r] += ((j < len[r]) & (v < kk[r])) ? 1u : 0u;  // no short circuit: no branch in the loop
      }
  } else {
    // long lists: a row at a time, as far as the wave's largest bucket in
    // that row
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      uint32_t lm = len[r];
      for (int o = 32; o > 0; o >>= 1) lm = max(lm, (uint32_t)__shfl_xor(lm, o, 64));
      for (uint32_t j = 0; j < lm; j++) {
        const unsigned long long v = S.keys[min(base[r] + j, L - 1)];
        rank[r] += ((j < len[r]) & (v < kk[r])) ? 1u : 0u;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < ROWS; r++)
    if (ok[r]) ids[rank[r]] = (uint32_t)kk[r];
  return true;
}

// K5 for lists of 1 to 1023 entries, one wave per tile, in two launches by
// length (the LDS a wave holds, and so how many waves fit a CU, follows the
// longest list of the launch): ROWS_MAX 4 takes lists below 256 entries,
// ROWS_MAX 16 the others (with 16-bit counters: 12 KB of LDS a wave instead
// of 16, so 13 waves fit a CU instead of 10).  A list whose largest bucket
// is too large goes on the list for tile_sort_fallback_kernel.
template <int ROWS_MAX>
__global__ void __launch_bounds__(64) tile_sort_small_kernel(const uint2* __restrict__ ranges,
                                                            const unsigned long long* __restrict__ keys,
                                                            uint32_t* __restrict__ ids,
                                                            const unsigned long long* __restrict__ P_dev,
                                                            unsigned long long cap, uint32_t* __restrict__ nfall,
                                                            uint32_t* __restrict__ fall) {
  constexpr uint32_t lo = ROWS_MAX == 4 ? 1u : 256u, hi = 64u * ROWS_MAX;
  __shared__ BlockSortSmem<64, ROWS_MAX, ROWS_MAX == 4 ? 9 : 11, ROWS_MAX == 16> S;
  const unsigned long long P = *P_dev;
  const uint2 r = ranges[blockIdx.x];  // written by K3 whatever P is
  if (P > cap) return;                 // the keys were not written
  const uint32_t L = r.y - r.x;
  if (L < lo || L >= hi || (unsigned long long)r.y > cap) return;
  bool done;
  if (L == 1) {
    if (threadIdx.x == 0) ids[r.x] = (uint32_t)keys[r.x];
    done = true;
  } else if (L <= 64u) {
    done = block_bucket_sort<64, 1, 7, false>(keys + r.x, L, ids + r.x, *(BlockSortSmem<64, 1, 7>*)&S);
  } else if (L <= 128u) {
    done = block_bucket_sort<64, 2, 8, false>(keys + r.x, L, ids + r.x, *(BlockSortSmem<64, 2, 8>*)&S);
  } else if (ROWS_MAX == 4 || L <= 256u) {
    done = block_bucket_sort<64, 4, 9, false>(keys + r.x, L, ids + r.x, *(BlockSortSmem<64, 4, 9>*)&S);
  } else if (L <= 512u) {
    done = block_bucket_sort<64, 8, 10, false>(keys + r.x, L, ids + r.x, *(BlockSortSmem<64, 8, 10>*)&S);
  } else {
    done = block_bucket_sort<64, ROWS_MAX, ROWS_MAX == 4 ? 9 : 11, ROWS_MAX == 16>(keys + r.x, L, ids + r.x, S);
  }
  if (!done && threadIdx.x == 0) fall[atomicAdd(nfall, 1u)] = blockIdx.x;
}

// The lists whose buckets came out too large, by the stable LSD radix sort:
// in LDS up to 4096 entries, else in chunks through the ping-pong buffer.
constexpr int kFallThreads = 256, kFallBlocks = 256;
__global__ void __launch_bounds__(kFallThreads) tile_sort_fallback_kernel(const uint2* __restrict__ ranges,
                                                                         unsigned long long* __restrict__ keys,
                                                                         unsigned long long* __restrict__ tmp,
                                                                         uint32_t* __restrict__ ids,
                                                                         const uint32_t* __restrict__ nfall,
                                                                         const uint32_t* __restrict__ fall) {
  __shared__ TileSortSmem<kFallThreads> S;
  const uint32_t m = *nfall;
  for (uint32_t i = blockIdx.x; i < m; i += gridDim.x) {
    const uint2 r = ranges[fall[i]];
    const uint32_t L = r.y - r.x;
    if (L <= (uint32_t)kFallThreads * kTSItems)
      sort_list_lds<kFallThreads>(keys + r.x, L, ids + r.x, S);
    else
      sort_list_chunked<kFallThreads>(keys + r.x, tmp + r.x, L, ids + r.x, S);
    __syncthreads();  // the LDS is reused by the next list
  }
}

// The t-th tile of the positions [n_from[c], n_to[c]) of the cameras' render
// orders (n_from null: from 0), counted across the cameras in turn.
__device__ inline uint32_t order_tile(uint32_t g, const uint32_t* __restrict__ order, const CamTiles& ct,
                                      const uint32_t* __restrict__ n_from, const uint32_t* __restrict__ n_to) {
  int c = 0;
  for (;;) {
    const uint32_t lo = n_from ? n_from[c] : 0u, cnt = n_to[c] - lo;
    if (g < cnt) return (uint32_t)ct.base[c] + order[ct.base[c] + lo + g];
    g -= cnt;
    c++;
  }
}

__device__ inline uint32_t order_count(int n_cams, const uint32_t* __restrict__ n_from,
                                       const uint32_t* __restrict__ n_to) {
  uint32_t total = 0;
  for (int c = 0; c < n_cams; c++) total += n_to[c] - (n_from ? n_from[c] : 0u);
  return total;
}

// K5 for lists of 1024 to 4095 entries (the positions [nbig, nmid) of each
// camera's render order): a fixed grid of 256-thread blocks, block b taking
// the b-th, (b + grid)-th, ... of them, by the bucket sort (16-bit counters
// and the waves' partials inside the key array: 40 KB of LDS and 128 VGPRs,
// four blocks a CU instead of three); a list whose
// largest bucket holds more than 128 entries goes on the list for
// tile_sort_fallback_kernel.
constexpr int kMidThreads = 256, kMidBlocks = 1024;
constexpr uint32_t kMidBucketMax = 128;
__global__ void __launch_bounds__(kMidThreads, 4) tile_sort_mid_kernel(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ order, CamTiles ct, int n_cams,
    const uint32_t* __restrict__ nbig, const uint32_t* __restrict__ nmid, const unsigned long long* __restrict__ keys,
    uint32_t* __restrict__ ids, const unsigned long long* __restrict__ P_dev, unsigned long long cap,
    uint32_t* __restrict__ nfall, uint32_t* __restrict__ fall) {
  __shared__ BlockSortSmem<kMidThreads, kTSItems, 12, true> S;
  if (*P_dev > cap) return;
  const uint32_t total = order_count(n_cams, nbig, nmid);
  for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {
    const uint32_t tile = order_tile(g, order, ct, nbig, nmid);
    const uint2 r = ranges[tile];
    if (!block_bucket_sort<kMidThreads, kTSItems, 12, true>(keys + r.x, r.y - r.x, ids + r.x, S, kMidBucketMax)) {
      if (threadIdx.x == 0) fall[atomicAdd(nfall, 1u)] = tile;
    }
    __syncthreads();  // the LDS is reused by the next list
  }
}

// K5 for lists of 4096 entries and more (the positions [0, nbig)): a fixed
// grid of 1024-thread blocks, one per CU, by the bucket sort with up to 8192
// buckets (16-bit counters) for lists of up to 16384 entries.  A longer list
// is first cut into runs of at most 16384 by the 8 bits below its highest
// varying bit (runs of whole digit values, so every key of a run is below
// every key of the next), moved run by run into the ping-pong buffer, and
// each run is bucket-sorted there.  A list with a run or bucket of more than
// 128 entries, or a digit value of more than 16384, goes on the list for
// tile_sort_fallback_kernel.
constexpr int kBigThreads = 1024, kBigBlocks = 256, kBigRows = 16;
constexpr uint32_t kBigMax = kBigThreads * kBigRows;
constexpr uint32_t kBigBucketMax = 128;
constexpr int kMaxRuns = 256;
struct SplitSmem {
  uint32_t hist[256];
  uint32_t run_of[256];  // the run of each digit value
  uint32_t fill[kMaxRuns];
  unsigned long long wor[kBigThreads / 64];
  uint32_t ok;
};
union BigSortSmem {
  BlockSortSmem<kBigThreads, kBigRows, 13, true> bucket;
  SplitSmem split;
};

// Cuts the L > kBigMax keys of src into runs of at most kBigMax (see above)
// and moves them to dst; the runs' bounds go to bounds[0 .. *nrun].  Returns
// false (and moves nothing) when one digit value holds more than kBigMax.
__device__ inline bool split_list(const unsigned long long* __restrict__ src, uint32_t L,
                                  unsigned long long* __restrict__ dst, SplitSmem& S, uint32_t* bounds,
                                  uint32_t* nrun) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  constexpr int U = 8;  // loads in flight per thread
  const unsigned long long k0 = src[0];
  unsigned long long orv = 0;
  for (uint32_t p0 = t; p0 < L; p0 += U * kBigThreads) {
    unsigned long long k[U];
#pragma unroll
    for (int j = 0; j < U; j++) k[j] = p0 + j * kBigThreads < L ? src[p0 + j * kBigThreads] : k0;
#pragma unroll
    for (int j = 0; j < U; j++) orv |= k[j] ^ k0;
  }
  for (int o = 32; o > 0; o >>= 1) orv |= __shfl_xor(orv, o, 64);
  if (lane == 0) S.wor[w] = orv;
  if (t < 256) S.hist[t] = 0u;
  __syncthreads();
  orv = 0;
#pragma unroll
  for (int k = 0; k < kBigThreads / 64; k++) orv |= S.wor[k];
  const int hb = orv ? 63 - __clzll((long long)orv) : 0;
  const int shift = hb >= 7 ? hb - 7 : 0;
  for (uint32_t p0 = t; p0 < L; p0 += U * kBigThreads) {
    unsigned long long k[U];
#pragma unroll
    for (int j = 0; j < U; j++) k[j] = p0 + j * kBigThreads < L ? src[p0 + j * kBigThreads] : 0ull;
#pragma unroll
    for (int j = 0; j < U; j++)
      if (p0 + j * kBigThreads < L) atomicAdd(&S.hist[(uint32_t)(k[j] >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (t == 0) {  // greedy cut at digit boundaries
    uint32_t run = 0, acc = 0, start = 0, ok = 1;
    bounds[0] = 0;
    for (int d = 0; d < 256; d++) {
      const uint32_t c = S.hist[d];
      if (c > kBigMax) ok = 0;
      if (acc + c > kBigMax) {
        run++;
        bounds[run] = start;
        acc = 0;
      }
      S.run_of[d] = run;
      acc += c;
      start += c;
    }
    *nrun = run + 1;
    bounds[run + 1] = L;
    S.ok = ok;
  }
  __syncthreads();
  if (!S.ok) {
    __syncthreads();
    return false;
  }
  if ((uint32_t)t < *nrun) S.fill[t] = bounds[t];
  __syncthreads();
  for (uint32_t p0 = t; p0 < L; p0 += U * kBigThreads) {
    unsigned long long k[U];
#pragma unroll
    for (int j = 0; j < U; j++) k[j] = p0 + j * kBigThreads < L ? src[p0 + j * kBigThreads] : 0ull;
#pragma unroll
    for (int j = 0; j < U; j++)
      if (p0 + j * kBigThreads < L) dst[atomicAdd(&S.fill[S.run_of[(uint32_t)(k[j] >> shift) & 255u]], 1u)] = k[j];
  }
  __syncthreads();  // the runs are in dst for the whole block
  return true;
}

__global__ void __launch_bounds__(kBigThreads) tile_sort_big_kernel(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ order, CamTiles ct, int n_cams,
    const uint32_t* __restrict__ nbig, const unsigned long long* __restrict__ keys,
    unsigned long long* __restrict__ tmp, uint32_t* __restrict__ ids, const unsigned long long* __restrict__ P_dev,
    unsigned long long cap, uint32_t* __restrict__ nfall, uint32_t* __restrict__ fall) {
  __shared__ BigSortSmem S;
  __shared__ uint32_t bounds[kMaxRuns + 1];
  __shared__ uint32_t nrun;
  if (*P_dev > cap) return;
  const uint32_t total = order_count(n_cams, nullptr, nbig);
  for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {
    const uint32_t tile = order_tile(g, order, ct, nullptr, nbig);
    const uint2 r = ranges[tile];
    const uint32_t L = r.y - r.x;
    bool done = false;
    if (L <= kBigMax) {
      done = block_bucket_sort<kBigThreads, kBigRows, 13, true>(keys + r.x, L, ids + r.x, S.bucket, kBigBucketMax);
    } else if (L <= kBigMax * (kMaxRuns / 2) && split_list(keys + r.x, L, tmp + r.x, S.split, bounds, &nrun)) {
      const uint32_t m = nrun;
      done = true;
      for (uint32_t k = 0; k < m && done; k++) {
        const uint32_t a = bounds[k], n = bounds[k + 1] - a;
        if (n > 0)
          done = block_bucket_sort<kBigThreads, kBigRows, 13, true>(tmp + r.x + a, n, ids + r.x + a, S.bucket,
                                                                    kBigBucketMax);
        __syncthreads();
      }
    }
    // the list's keys are still whole in keys: the radix sort takes it over
    if (!done && threadIdx.x == 0) fall[atomicAdd(nfall, 1u)] = tile;
    __syncthreads();  // the LDS is reused by the next list
  }
}

// ------------------------------------------------------------------ host

// Pinned host slot for the pair-count read-back and the event that marks
// it, one per host thread.
struct ReadbackSlot {
  void* p = nullptr;   // host address: P (2 words), then each camera's long lists
  void* dp = nullptr;  // the same memory as the device sees it
  hipEvent_t ev = nullptr;
  int n_cams = 0;      // cameras of the last count phase
  ~ReadbackSlot() {
    if (p) (void)hipHostFree(p);
    if (ev) (void)hipEventDestroy(ev);
  }
};
static thread_local ReadbackSlot g_readback;

static inline unsigned grid_for(int64_t m, int threads) { return (unsigned)((m + threads - 1) / threads); }

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, int64_t m, uint32_t v) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) p[j] = v;
}

gut_status fill_u32(uint32_t* p, int64_t m, uint32_t v, hipStream_t st) {
  if (m <= 0) return GUT_OK;
  fill_u32_kernel<<<grid_for(m, 256), 256, 0, st>>>(p, m, v);
  GUT_LAUNCH_CHECK();
  return GUT_OK;
}

static CamTiles cam_tiles(const DevCam* dc, int n_cams) {
  CamTiles ct;
  for (int c = 0; c < n_cams; c++) {
    ct.base[c] = dc[c].tile_base;
    ct.tx[c] = dc[c].tiles_x;
    ct.count[c] = dc[c].tiles_x * dc[c].tiles_y;
  }
  return ct;
}

static BinArgs bin_args(const gut_projected* proj, int n, const DevCam* dc, int n_cams, bool cull,
                        size_t* lds_bytes) {
  BinArgs a;
  a.rect = (const short4*)proj->rect;
  a.tiles = proj->tiles;
  a.depth = proj->depth;
  a.mean2d = (const float2*)proj->mean2d;
  a.extent = (const float4*)proj->extent;
  a.n = n;
  a.bpc = (int)blocks_per_cam(n);
  a.cull = cull ? 1 : 0;
  a.n_cams = n_cams;
  a.ct = cam_tiles(dc, n_cams);
  int w = 0;  // LDS words of the largest window (with the count kernel's spare column)
  for (int c = 0; c < n_cams; c++) {
    const int txc = a.ct.tx[c], tyc = a.ct.count[c] / txc;
    w = std::max(w, window_rows(txc, tyc) * (txc + 1));
  }
  *lds_bytes = (size_t)w * 4;
  return a;
}

gut_status bin_count_launch(const gut_projected* proj, int n, const DevCam* dc, int n_cams, int64_t T,
                            bool cull, char* cws, uint32_t* tile_ranges, hipStream_t s) {
  if (!g_readback.p) {
    GUT_HIP(hipHostMalloc(&g_readback.p, 4 * (2 + kMaxCams), hipHostMallocMapped | hipHostMallocCoherent));
    GUT_HIP(hipHostGetDevicePointer(&g_readback.dp, g_readback.p, 0));
  }
  if (!g_readback.ev) GUT_HIP(hipEventCreateWithFlags(&g_readback.ev, hipEventDisableTiming));
  std::memset(g_readback.p, 0xff, 8);  // a sentinel no total can equal
  g_readback.n_cams = n_cams;
  size_t lds = 0;
  const BinArgs a = bin_args(proj, n, dc, n_cams, cull, &lds);
  uint32_t* M = (uint32_t*)cws;
  unsigned long long* sw = (unsigned long long*)(cws + al((size_t)((int64_t)a.bpc * T) * 4));
  bin_init_kernel<<<1, 64, 0, s>>>(sw);
  GUT_LAUNCH_CHECK();
  if (n > 0) {
    bin_count_kernel<<<(unsigned)(a.bpc * n_cams), kBinThreads, lds, s>>>(a, M);
    GUT_LAUNCH_CHECK();
    bin_colscan_kernel<<<grid_for(T, kColTiles), kColThreads, 0, s>>>(
        M, a.ct, n_cams, a.bpc, T, (uint2*)tile_ranges, sw + SmallLayout::cam_pairs / 8);
    GUT_LAUNCH_CHECK();
  } else {  // no entries: every count is zero
    gut_status st = fill_u32(tile_ranges, 2 * T, 0u, s);
    if (st != GUT_OK) return st;
  }
  bin_scan_kernel<<<n_cams, kScanThreads, 0, s>>>((uint2*)tile_ranges, tile_ranges + 2 * T, a.ct, n_cams, sw,
                                                  g_readback.dp);
  GUT_LAUNCH_CHECK();
  GUT_HIP(hipEventRecord(g_readback.ev, s));
  return GUT_OK;
}

gut_status bin_count_wait(uint64_t* P, uint32_t* n_long) {
  GUT_HIP(hipEventSynchronize(g_readback.ev));
  uint32_t w[2 + kMaxCams];
  std::memcpy(w, g_readback.p, 4 * (2 + g_readback.n_cams));
  const uint64_t v = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
  if (v == ~0ull) {
    set_error("binning: the pair count did not reach the host");
    return GUT_E_HIP;
  }
  *P = v;
  if (n_long) {
    uint32_t m = 0;
    for (int c = 0; c < g_readback.n_cams; c++) m += w[2 + c];
    *n_long = m;
  }
  return GUT_OK;
}

gut_status bin_sort_launch(const gut_projected* proj, int n, const DevCam* dc, int n_cams, int64_t T, bool cull,
                           char* cws, int64_t cap, char* pws, uint32_t* tile_ranges, uint32_t* sorted_ids,
                           hipStream_t s, int phases) {
  size_t lds = 0;
  const BinArgs a = bin_args(proj, n, dc, n_cams, cull, &lds);
  const uint32_t* M = (const uint32_t*)cws;
  char* swb = cws + al((size_t)((int64_t)a.bpc * T) * 4);
  const unsigned long long* P_dev = (const unsigned long long*)(swb + SmallLayout::total);
  const uint32_t* nbig = (const uint32_t*)(swb + SmallLayout::nbig);
  const uint32_t* nmid = (const uint32_t*)(swb + SmallLayout::nmid);
  unsigned long long* keys = (unsigned long long*)pws;
  unsigned long long* tmp = (unsigned long long*)(pws + al((size_t)(cap > 0 ? cap : 1) * 8));
  const unsigned long long ucap = (unsigned long long)cap;
  uint32_t* nfall = (uint32_t*)(swb + SmallLayout::nfall);
  uint32_t* fall = (uint32_t*)(swb + kSmallBytes);
  if (phases & kSortLists) {
    if (n > 0) {
      bin_scatter_kernel<<<(unsigned)(a.bpc * n_cams), kBinThreads, lds, s>>>(a, M, (const uint2*)tile_ranges,
                                                                               P_dev, ucap, keys);
      GUT_LAUNCH_CHECK();
    }
    tile_sort_small_kernel<4><<<(unsigned)T, 64, 0, s>>>((const uint2*)tile_ranges, keys, sorted_ids, P_dev, ucap,
                                                         nfall, fall);
    GUT_LAUNCH_CHECK();
    tile_sort_small_kernel<16><<<(unsigned)T, 64, 0, s>>>((const uint2*)tile_ranges, keys, sorted_ids, P_dev, ucap,
                                                          nfall, fall);
    GUT_LAUNCH_CHECK();
    tile_sort_mid_kernel<<<kMidBlocks, kMidThreads, 0, s>>>((const uint2*)tile_ranges, tile_ranges + 2 * T, a.ct,
                                                            n_cams, nbig, nmid, keys, sorted_ids, P_dev, ucap, nfall,
                                                            fall);
    GUT_LAUNCH_CHECK();
  }
  if (phases & kSortLong) {
    tile_sort_big_kernel<<<kBigBlocks, kBigThreads, 0, s>>>((const uint2*)tile_ranges, tile_ranges + 2 * T, a.ct,
                                                            n_cams, nbig, keys, tmp, sorted_ids, P_dev, ucap, nfall,
                                                            fall);
    GUT_LAUNCH_CHECK();
  }
  if (phases & kSortFallback) {
    tile_sort_fallback_kernel<<<kFallBlocks, kFallThreads, 0, s>>>((const uint2*)tile_ranges, keys, tmp, sorted_ids,
                                                                   nfall, fall);
    GUT_LAUNCH_CHECK();
  }
  return GUT_OK;
}

}  // namespace gut

using namespace gut;

extern "C" size_t gut_bin_workspace_bytes(int64_t n, const gut_camera* cams, int32_t n_cams,
                                          int64_t pair_capacity) {
  if (n < 0 || !cams || n_cams <= 0 || n_cams > kMaxCams || pair_capacity < 0) return 0;
  int64_t T = 0;
  for (int c = 0; c < n_cams; c++) {
    if (cams[c].width <= 0 || cams[c].height <= 0) return 0;
    T += (int64_t)((cams[c].width + kTile - 1) / kTile) * ((cams[c].height + kTile - 1) / kTile);
  }
  return bin_count_bytes(n, T) + bin_pair_bytes(pair_capacity);
}

extern "C" gut_status gut_bin(const gut_projected* proj, int64_t n, const gut_camera* cams,
                              int32_t n_cams, const gut_params* p, void* ws, size_t ws_bytes,
                              int64_t pair_capacity, uint32_t* tile_ranges, uint32_t* sorted_ids,
                              int64_t* n_pairs, void* stream) {
  gut_status st = check_params(p);
  if (st != GUT_OK) return st;
  if (!proj || (n > 0 && (!proj->rect || !proj->tiles || !proj->depth))) {
    set_error("projected rect, tiles and depth are required");
    return GUT_E_INVALID;
  }
  const bool cull = p->tile_cull != 0;
  if (cull && n > 0 && (!proj->mean2d || !proj->extent)) {
    set_error("tile culling needs the projected mean2d and extent");
    return GUT_E_INVALID;
  }
  if (((uintptr_t)proj->rect & 7) || ((uintptr_t)tile_ranges & 7) || ((uintptr_t)proj->mean2d & 7) ||
      ((uintptr_t)proj->extent & 15)) {
    set_error("rect, mean2d and tile_ranges must be 8-byte, extent 16-byte aligned");
    return GUT_E_INVALID;
  }
  if (n < 0 || pair_capacity < 0 || !tile_ranges || (pair_capacity > 0 && !sorted_ids)) {
    set_error("bad sizes or NULL outputs");
    return GUT_E_INVALID;
  }
  if (pair_capacity >= (int64_t(1) << 32)) {
    set_error("pair_capacity must be below 2^32");
    return GUT_E_INVALID;
  }
  DevCam dc[kMaxCams];
  int64_t T = 0;
  if ((st = prepare_cams(cams, n_cams, *p, dc, &T, nullptr)) != GUT_OK) return st;
  const int64_t E = n * n_cams;
  if (E >= (int64_t(1) << 31)) { set_error("n * n_cams must be below 2^31"); return GUT_E_INVALID; }
  const size_t cb = bin_count_bytes(n, T), need = cb + bin_pair_bytes(pair_capacity);
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) {
    set_error("workspace must be 256-byte aligned and hold %zu bytes (got %zu)", need, ws_bytes);
    return GUT_E_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  char* cws = (char*)ws;
  char* pws = cws + cb;
  if ((st = bin_count_launch(proj, (int)n, dc, n_cams, T, cull, cws, tile_ranges, s)) != GUT_OK) return st;
  // The scatter and the sorts up to 4095 entries are queued before the one
  // wait (they check the capacity on the device); the long lists' sort is
  // queued after it, only if there are long lists, and the fallback last.
  if ((st = bin_sort_launch(proj, (int)n, dc, n_cams, T, cull, cws, pair_capacity, pws, tile_ranges, sorted_ids, s,
                            kSortLists)) != GUT_OK)
    return st;
  uint64_t P = 0;
  uint32_t n_long = 0;
  if ((st = bin_count_wait(&P, &n_long)) != GUT_OK) return st;
  if ((st = bin_sort_launch(proj, (int)n, dc, n_cams, T, cull, cws, pair_capacity, pws, tile_ranges, sorted_ids, s,
                            (n_long ? kSortLong : 0) | kSortFallback)) != GUT_OK)
    return st;
  if (n_pairs) *n_pairs = (int64_t)P;
  if ((int64_t)P > pair_capacity) {
    (void)fill_u32(tile_ranges, 2 * T, 0u, s);  // every tile empty
    set_error("pair capacity %lld < required %llu", (long long)pair_capacity, (unsigned long long)P);
    return GUT_E_CAPACITY;
  }
  return GUT_OK;
}
