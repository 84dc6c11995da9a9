// Tile binning: the global per-tile depth sort of Sec. 4.3.
//
// Order of work (E = n_cams * n entries, P = pairs):
//   1. stable LSD radix sort of the visible entries by depth (32 bits); its
//      first pass reads every entry and places only the visible ones, so the
//      compaction costs no pass of its own; its histogram also leaves
//      per-block totals of N_vis and P, which go to the host while the rest
//      of the sort runs; its last pass writes, instead of the depth keys, what
//      the duplication reads: each entry's tile count and tile geometry
//   2. scan of the tile counts in depth order -> pair offsets
//   3. duplicate: each entry writes (global tile id, entry id) for every tile
//      of its rectangle at its offset
//   4. stable LSD radix sort of the P pairs by tile id (ceil(log2 T) bits);
//      its last pass also writes the per-tile [start, end) ranges
// Sorting entries by depth first and then pairs by tile only gives exactly the
// (tile, depth, id) order of a full-key sort while moving far fewer bytes:
// the tile sort carries 4-byte keys over ceil(log2 T)/8 passes instead of
// 8-byte keys over (32 + log2 T)/8 passes.
#include <cstring>

#include "radix.h"

namespace gut {

struct CamTiles {
  int base[kMaxCams];
  int tx[kMaxCams];
  int count[kMaxCams];
};

static size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace of the entry phase (sized by E = n_cams * n) and of the pair
// phase (sized by the pair capacity).
struct EntryLayout {
  size_t scalars, part_n, part_p, dkA, dvA, dkB, dvB, pA, pB, geo, offs, offs_tmp, radix_tmp, total;
};
struct PairLayout {
  size_t pkA, pkB, pvB, radix_tmp, total;
};

static EntryLayout entry_layout(int64_t E) {
  EntryLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += al(bytes); return r; };
  const int64_t nb = radix_blocks(E);
  L.scalars = take(64);
  L.part_n = take(nb * 4);
  L.part_p = take(nb * 8);
  L.dkA = take(E * 4);
  L.dvA = take(E * 4);
  L.dkB = take(E * 4);
  L.dvB = take(E * 4);
  L.pA = take(E * 4);
  L.pB = take(E * 4);
  L.geo = take(E * 8);
  L.offs = take(E * 4);
  L.offs_tmp = take(scan_temp_bytes(E));
  L.radix_tmp = take(radix_temp_bytes(E));
  L.total = o;
  return L;
}

static PairLayout pair_layout(int64_t cap) {
  PairLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += al(bytes); return r; };
  L.pkA = take(cap * 4);
  L.pkB = take(cap * 4);
  L.pvB = take(cap * 4);
  L.radix_tmp = take(radix_temp_bytes(cap));
  L.total = o;
  return L;
}

size_t bin_entry_bytes(int64_t E) { return entry_layout(E).total; }
size_t bin_pair_bytes(int64_t cap) { return pair_layout(cap).total; }

// Packed tile rectangle: x0 | y0 << 8 | (x1 - x0) << 16 | (y1 - y0) << 24,
// exact when every camera has at most 256 tiles per axis.
__device__ inline uint32_t pack_rect(short4 r) {
  return ((uint32_t)r.x & 255u) | (((uint32_t)r.y & 255u) << 8) | (((uint32_t)(r.z - r.x) & 255u) << 16) |
         (((uint32_t)(r.w - r.y) & 255u) << 24);
}

// The entries of chunk `chunk` as depth-sort items: key = depth bits, value =
// entry id, valid = the entry touches a tile.  *pairs (if given) receives the
// sum of the items' tile counts; rect (if given) fills pp with the packed
// rectangles.
__device__ inline uint32_t load_entry_chunk(const uint32_t* __restrict__ tiles,
                                            const float* __restrict__ depth, int64_t E,
                                            uint32_t (&kk)[kRItems], uint32_t (&vv)[kRItems],
                                            unsigned long long* pairs, const short4* __restrict__ rect,
                                            uint32_t (&pp)[kRItems], int64_t chunk) {
  const int lane = threadIdx.x & (kRWave - 1), w = threadIdx.x / kRWave;
  const int64_t base = chunk * kRChunk + (int64_t)w * (kRChunk / kRWaves);
  uint32_t vmask = 0;
  unsigned long long sum = 0;
#pragma unroll
  for (int r = 0; r < kRItems; r++) {
    const int64_t g = base + r * kRWave + lane;
    const uint32_t tl = g < E ? tiles[g] : 0u;
    kk[r] = g < E ? __float_as_uint(depth[g]) : 0u;
    vv[r] = (uint32_t)g;
    if (rect) pp[r] = tl > 0 ? pack_rect(rect[g]) : 0u;
    vmask |= (uint32_t)(tl > 0) << r;
    sum += tl;
  }
  if (pairs) *pairs = sum;
  return vmask;
}

// First depth pass, histogram: digit counts of the visible entries, and the
// block's visible-entry and pair totals.  The blocks also set the tile ranges
// to (~0u, 0), which the last tile pass lowers / raises with atomics.
__global__ void __launch_bounds__(kRThreadsSort) entry_hist_kernel(
    const uint32_t* __restrict__ tiles, const float* __restrict__ depth, int64_t E,
    uint32_t* __restrict__ counts, int64_t nblocks, uint32_t* __restrict__ part_n,
    unsigned long long* __restrict__ part_p, uint2* __restrict__ ranges, int64_t T) {
  __shared__ uint32_t h[kRadix];
  __shared__ unsigned long long wp[kRWaves];
  __shared__ uint32_t wv[kRWaves];
  for (int64_t i = (int64_t)blockIdx.x * kRThreadsSort + threadIdx.x; i < T;
       i += nblocks * kRThreadsSort)
    ranges[i] = make_uint2(~0u, 0u);
  uint32_t kk[kRItems], vv[kRItems], pp[kRItems];
  unsigned long long pairs;
  const uint32_t vmask = load_entry_chunk(tiles, depth, E, kk, vv, &pairs, nullptr, pp, blockIdx.x);
  uint32_t nv = (uint32_t)__popc(vmask);
  for (int o = 32; o > 0; o >>= 1) {
    pairs += __shfl_xor(pairs, o, 64);
    nv += __shfl_xor(nv, o, 64);
  }
  if ((threadIdx.x & 63) == 0) { wp[threadIdx.x >> 6] = pairs; wv[threadIdx.x >> 6] = nv; }
  radix_hist_store(kk, vmask, 0, kRadix - 1, h, counts, nblocks);  // synchronises the block
  if (threadIdx.x == 0) {
    unsigned long long sp = 0;
    uint32_t sv = 0;
    for (int k = 0; k < kRWaves; k++) { sp += wp[k]; sv += wv[k]; }
    part_n[blockIdx.x] = sv;
    part_p[blockIdx.x] = sp;
  }
}

// First depth pass, scatter: places the visible entries only; with PACKED,
// the packed rectangle travels with each entry.
template <bool PACKED>
__global__ void __launch_bounds__(kRThreadsSort) entry_scatter_kernel(
    const uint32_t* __restrict__ tiles, const float* __restrict__ depth, const short4* __restrict__ rect,
    int64_t E, KVSink sink, const uint32_t* __restrict__ offs, const uint32_t* __restrict__ totals,
    int64_t nblocks) {
  __shared__ RadixRankSmem S;
  __shared__ uint32_t sk[kRChunk];
  uint32_t kk[kRItems], vv[kRItems], pp[kRItems];
  const int64_t chunk = radix_xcd_chunk(nblocks);
  const uint32_t vmask =
      load_entry_chunk(tiles, depth, E, kk, vv, nullptr, PACKED ? rect : nullptr, pp, chunk);
  radix_scatter_chunk<PACKED>(kk, vv, pp, vmask, 0, kRadixBits, offs, totals, nblocks, chunk, sink, S, sk);
}

// Output of the last depth pass when the rectangles travel packed: the
// entry ids, the packed rectangles and the tile counts, in depth order.
struct EntryFinalSink {
  uint32_t* ent;
  uint32_t* rectp;
  uint32_t* cnt;
  __device__ uint2* bounds() const { return nullptr; }
  __device__ void key(uint32_t, uint32_t) const {}
  __device__ void vals(const uint32_t (&pos)[kRItems], const uint32_t (&v)[kRItems], int t,
                       uint32_t count) const {
#pragma unroll
    for (int i = 0; i < kRItems; i++)
      if (t + i * kRThreadsSort < (int)count) ent[pos[i]] = v[i];
  }
  __device__ void pays(const uint32_t (&pos)[kRItems], const uint32_t (&p)[kRItems], int t,
                       uint32_t count) const {
#pragma unroll
    for (int i = 0; i < kRItems; i++) {
      if (t + i * kRThreadsSort >= (int)count) continue;
      rectp[pos[i]] = p[i];
      cnt[pos[i]] = (((p[i] >> 16) & 255u) + 1u) * ((p[i] >> 24) + 1u);
    }
  }
};

__global__ void __launch_bounds__(kRThreadsSort) entry_final_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, const uint32_t* __restrict__ pin,
    const uint32_t* n_dev, EntryFinalSink sink, int shift, int nbits, const uint32_t* __restrict__ offs,
    const uint32_t* __restrict__ totals, int64_t nblocks) {
  __shared__ RadixRankSmem S;
  __shared__ uint32_t sk[kRChunk];
  const int64_t n = *n_dev;
  const int64_t chunk = radix_xcd_chunk((n + kRChunk - 1) / kRChunk);
  if (chunk < 0) return;
  uint32_t kk[kRItems], vv[kRItems], pp[kRItems];
  const uint32_t vmask = radix_load_kv(kin, vin, pin, n, chunk, kk, vv, pp);
  radix_scatter_chunk<true>(kk, vv, pp, vmask, shift, nbits, offs, totals, nblocks, chunk, sink, S, sk);
}

// The depth-sorted entries' tile counts and geometry, gathered once by a
// kernel with many waves in flight (the reads are random in the entry id):
// cnt[j] = tiles[e], geo[j] = (first tile id, rectangle width | camera tiles
// per row << 16) for e = ent[j]; each block also leaves the sum of its
// 4096 counts for the offsets scan.
__global__ void __launch_bounds__(kRThreadsSort) entry_gather_kernel(
    const uint32_t* __restrict__ ent, int64_t m, const uint32_t* __restrict__ tiles,
    const short4* __restrict__ rect, int n, CamTiles ct, uint32_t* __restrict__ cnt,
    uint2* __restrict__ geo, uint32_t* __restrict__ sums) {
  __shared__ uint32_t wsum[kRWaves];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kRChunk;
  uint32_t e[kRItems], tl[kRItems];
  short4 r[kRItems];
#pragma unroll
  for (int j = 0; j < kRItems; j++) {
    const int64_t g = base + j * kRThreadsSort + t;
    e[j] = g < m ? ent[g] : 0u;
  }
#pragma unroll
  for (int j = 0; j < kRItems; j++) {
    const int64_t g = base + j * kRThreadsSort + t;
    tl[j] = g < m ? tiles[e[j]] : 0u;
    r[j] = g < m ? rect[e[j]] : make_short4(0, 0, 0, 0);
  }
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < kRItems; j++) {
    const int64_t g = base + j * kRThreadsSort + t;
    if (g >= m) continue;
    const int cam = (int)(e[j] / (uint32_t)n);
    const uint32_t tx = (uint32_t)ct.tx[cam];
    cnt[g] = tl[j];
    geo[g] = make_uint2((uint32_t)ct.base[cam] + (uint32_t)r[j].y * tx + (uint32_t)r[j].x,
                        (uint32_t)(r[j].z - r[j].x + 1) | (tx << 16));
    acc += tl[j];
  }
  uint32_t total;
  radix_block_scan(acc, wsum, &total);
  if (t == 0) sums[blockIdx.x] = total;
}

// Expands each visible entry (in depth order) into one (tile, entry) pair per
// tile of its rectangle, row-major.  A block takes 256 consecutive entries
// and spreads their contiguous output range evenly over its threads (each
// output finds its entry by binary search of the block's offsets in LDS), so
// the writes are coalesced whatever the rectangle sizes.  The rectangles come
// packed (PACKED) or as gathered geometry.  Outputs stay below P and tile ids
// below T whatever the inputs.
constexpr int kDupThreads = 256;
template <bool PACKED>
__global__ void __launch_bounds__(kDupThreads) duplicate_kernel(
    const uint32_t* __restrict__ ent, const uint32_t* __restrict__ offs, const uint32_t* __restrict__ rectp,
    const uint2* __restrict__ geo, int n, CamTiles ct, int64_t m, uint64_t P, uint32_t T,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  __shared__ uint32_t so[kDupThreads + 1];
  __shared__ uint32_t se[kDupThreads];
  __shared__ uint32_t st0[kDupThreads];  // first tile
  __shared__ uint32_t sw[kDupThreads];   // rectangle width
  __shared__ uint32_t stx[kDupThreads];  // camera tiles per row
  __shared__ float sinv[kDupThreads];    // 1 / width
  const int t = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * kDupThreads;
  const int cnt = (int)min((int64_t)kDupThreads, m - j0);
  if (t < cnt) {
    const uint32_t e = ent[j0 + t];
    uint32_t t0, w, tx;
    if (PACKED) {
      const uint32_t p = rectp[j0 + t];
      const int cam = (int)(e / (uint32_t)n);
      tx = (uint32_t)ct.tx[cam];
      t0 = (uint32_t)ct.base[cam] + ((p >> 8) & 255u) * tx + (p & 255u);
      w = ((p >> 16) & 255u) + 1u;
    } else {
      const uint2 g = geo[j0 + t];
      t0 = g.x;
      w = g.y & 0xffffu;
      tx = g.y >> 16;
    }
    so[t] = offs[j0 + t];
    se[t] = e;
    st0[t] = t0;
    sw[t] = w;
    stx[t] = tx;
    sinv[t] = 1.0f / (float)w;
  }
  if (t == 0) so[cnt] = j0 + cnt < m ? offs[j0 + cnt] : (uint32_t)P;
  __syncthreads();
  const uint32_t p1 = min(so[cnt], (uint32_t)P);
  for (uint32_t p = so[0] + t; p < p1; p += kDupThreads) {
    int lo = 0, hi = cnt - 1;  // last entry whose output starts at or before p
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (so[mid] <= p) lo = mid; else hi = mid - 1;
    }
    const uint32_t k = p - so[lo], w = sw[lo];
    // k / w through the float reciprocal (k < 2^24), corrected by one step
    uint32_t y = (uint32_t)((float)k * sinv[lo]);
    int32_t x = (int32_t)(k - y * w);
    if (x < 0) { y--; x += (int32_t)w; } else if (x >= (int32_t)w) { y++; x -= (int32_t)w; }
    keys[p] = min(st0[lo] + y * stx[lo] + (uint32_t)x, T - 1u);
    vals[p] = se[lo];
  }
}

// Render order of one camera's tiles (one block per camera): a counting sort
// of the tiles by bucket = bit length of the list length, longest first.
// Only the schedule depends on it (every tile is rendered independently), so
// the order within a bucket may vary from call to call.  Tiles that no pair
// reached still hold (~0u, 0) from the initialisation and are set to [0, 0).
constexpr int kOrderThreads = 1024;
__global__ void __launch_bounds__(kOrderThreads) order_kernel(uint2* __restrict__ ranges, CamTiles ct,
                                                             uint32_t* __restrict__ order) {
  __shared__ unsigned cnt[33], cur[33];
  const int c = blockIdx.x, base = ct.base[c], nt = ct.count[c];
  for (int b = threadIdx.x; b < 33; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  for (int t = threadIdx.x; t < nt; t += blockDim.x) {
    uint2 r = ranges[base + t];
    if (r.x > r.y) {
      r = make_uint2(0u, 0u);
      ranges[base + t] = r;
    }
    const int key = __clz(r.y - r.x);  // 32 - bit length: 0 for the longest lists
    atomicAdd(&cnt[key], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned acc = 0;
    for (int b = 0; b < 33; b++) { cur[b] = acc; acc += cnt[b]; }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nt; t += blockDim.x) {
    const uint2 r = ranges[base + t];  // as this thread left it above
    const unsigned pos = atomicAdd(&cur[__clz(r.y - r.x)], 1u);
    order[base + pos] = (uint32_t)t;
  }
}

// Pinned host slot for the count read-back and the event that marks it, one
// per host thread.
struct ReadbackSlot {
  void* p = nullptr;   // host address
  void* dp = nullptr;  // the same memory as the device sees it
  hipEvent_t ev = nullptr;
  ~ReadbackSlot() {
    if (p) (void)hipHostFree(p);
    if (ev) (void)hipEventDestroy(ev);
  }
};
static thread_local ReadbackSlot g_readback;

static inline unsigned grid_for(int64_t m, int threads) {
  return (unsigned)((m + threads - 1) / threads);
}

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

// The depth sort's passes: the first writes (dkB, dvB[, pB]) and the others
// ping-pong from B, so the sorted entry ids end in dvA; with packed
// rectangles the last pass is entry_final_kernel, which also leaves the
// packed rectangles in pA and the tile counts in dkA.
static int depth_passes() { return radix_passes(32); }

// The rectangles travel packed in 32 bits when every camera has at most 256
// tiles per axis (4096 px); otherwise they are gathered after the sort.
static bool rects_pack(const DevCam* dc, int n_cams) {
  for (int c = 0; c < n_cams; c++)
    if (dc[c].tiles_x > 256 || dc[c].tiles_y > 256) return false;
  return true;
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

gut_status bin_count(const gut_projected* proj, int n, const DevCam* dc, int n_cams, int64_t T, char* ews,
                     uint32_t* tile_ranges, uint32_t* nvis_out, uint64_t* P_out, hipStream_t s) {
  const int64_t E = (int64_t)n * n_cams;
  EntryLayout L = entry_layout(E);
  auto E32 = [&](size_t off) { return (uint32_t*)(ews + off); };
  uint32_t* scal = E32(L.scalars);
  *nvis_out = 0;
  *P_out = 0;
  gut_status st;
  if (E == 0) return fill_u32(tile_ranges, 2 * T, 0u, s);
  if (!g_readback.p) {
    GUT_HIP(hipHostMalloc(&g_readback.p, 64, hipHostMallocMapped | hipHostMallocCoherent));
    GUT_HIP(hipHostGetDevicePointer(&g_readback.dp, g_readback.p, 0));
  }
  if (!g_readback.ev) GUT_HIP(hipEventCreateWithFlags(&g_readback.ev, hipEventDisableTiming));
  const int64_t nb = radix_blocks(E);
  const RadixTemp rt = radix_temp(ews + L.radix_tmp, E);
  entry_hist_kernel<<<(unsigned)nb, kRThreadsSort, 0, s>>>(
      proj->tiles, proj->depth, E, rt.counts, nb, E32(L.part_n),
      (unsigned long long*)(ews + L.part_p), (uint2*)tile_ranges, T);
  GUT_LAUNCH_CHECK();
  // the rowscan's extra block totals N_vis and P into scal and the pinned
  // slot; the slot starts as a sentinel no total can equal
  std::memset(g_readback.p, 0xff, 16);
  const RowscanTail tail = {E32(L.part_n), (const unsigned long long*)(ews + L.part_p), nb, scal,
                            g_readback.dp};
  if ((st = radix_rowscan(rt.counts, rt.offs, rt.totals, nb, s, &tail)) != GUT_OK) return st;
  GUT_HIP(hipEventRecord(g_readback.ev, s));
  const bool packed = rects_pack(dc, n_cams);
  const KVSink sink0 = {E32(L.dkB), E32(L.dvB), nullptr, E32(L.pB)};
  if (packed)
    entry_scatter_kernel<true><<<(unsigned)nb, kRThreadsSort, 0, s>>>(
        proj->tiles, proj->depth, (const short4*)proj->rect, E, sink0, rt.offs, rt.totals, nb);
  else
    entry_scatter_kernel<false><<<(unsigned)nb, kRThreadsSort, 0, s>>>(
        proj->tiles, proj->depth, nullptr, E, sink0, rt.offs, rt.totals, nb);
  GUT_LAUNCH_CHECK();
  // the remaining passes take N_vis from the device
  const int passes = depth_passes(), per = radix_per_pass(32);
  int inB = 0;
  if (!packed) {
    if ((st = radix_sort_passes(E32(L.dkB), E32(L.dvB), E32(L.dkA), E32(L.dvA), E, scal, 32, 1, passes,
                                ews + L.radix_tmp, s, &inB, nullptr)) != GUT_OK)
      return st;
  } else {
    if ((st = radix_sort_passes(E32(L.dkB), E32(L.dvB), E32(L.dkA), E32(L.dvA), E, scal, 32, 1,
                                passes - 1, ews + L.radix_tmp, s, &inB, nullptr, E32(L.pB), E32(L.pA))) !=
        GUT_OK)
      return st;
    if (inB) {  // the middle passes are even in number: the last reads B
      set_error("binning: depth sort ended in the wrong buffer");
      return GUT_E_HIP;
    }
    const int shift = (passes - 1) * per, nbits = 32 - shift;
    if ((st = radix_hist(E32(L.dkB), E, scal, shift, (1u << nbits) - 1u, rt.counts, nb, s)) != GUT_OK)
      return st;
    if ((st = radix_rowscan(rt.counts, rt.offs, rt.totals, nb, s)) != GUT_OK) return st;
    const EntryFinalSink fin = {E32(L.dvA), E32(L.pA), E32(L.dkA)};
    entry_final_kernel<<<(unsigned)nb, kRThreadsSort, 0, s>>>(E32(L.dkB), E32(L.dvB), E32(L.pB), scal, fin,
                                                              shift, nbits, rt.offs, rt.totals, nb);
    GUT_LAUNCH_CHECK();
    inB = 1;
  }
  if (!inB) {
    set_error("binning: depth sort ended in the wrong buffer");
    return GUT_E_HIP;
  }
  // the one wait of the binning: for the totals, while the sort runs on
  GUT_HIP(hipEventSynchronize(g_readback.ev));
  uint32_t nvis;
  unsigned long long P;
  std::memcpy(&nvis, g_readback.p, 4);
  std::memcpy(&P, (char*)g_readback.p + 8, 8);
  if ((int64_t)nvis > E) {
    set_error("binning: the visible-entry count did not reach the host");
    return GUT_E_HIP;
  }
  *nvis_out = nvis;
  *P_out = P;
  return GUT_OK;
}

gut_status bin_sort(const gut_projected* proj, int n, const DevCam* dc, int n_cams, int64_t T,
                    int64_t E, char* ews, uint32_t nvis, uint64_t P, char* pws,
                    uint32_t* tile_ranges, uint32_t* sorted_ids, hipStream_t s) {
  if (nvis == 0 || P == 0) return GUT_OK;
  EntryLayout L = entry_layout(E);
  PairLayout Lp = pair_layout((int64_t)P);
  auto E32 = [&](size_t off) { return (uint32_t*)(ews + off); };
  auto Q32 = [&](size_t off) { return (uint32_t*)(pws + off); };
  gut_status st;
  const CamTiles ct = cam_tiles(dc, n_cams);
  const bool packed = rects_pack(dc, n_cams);
  if (packed) {  // the depth sort left the tile counts in dkA
    if ((st = exclusive_scan_u32(E32(L.dkA), E32(L.offs), nvis, ews + L.offs_tmp, s)) != GUT_OK) return st;
  } else {
    // tile counts (into dkA, free after the depth sort) and geometry, with
    // the scan's block sums, then the rest of the offsets scan
    entry_gather_kernel<<<(unsigned)radix_blocks(nvis), kRThreadsSort, 0, s>>>(
        E32(L.dvA), nvis, proj->tiles, (const short4*)proj->rect, n, ct, E32(L.dkA),
        (uint2*)(ews + L.geo), (uint32_t*)(ews + L.offs_tmp));
    GUT_LAUNCH_CHECK();
    if ((st = exclusive_scan_u32(E32(L.dkA), E32(L.offs), nvis, ews + L.offs_tmp, s, true)) != GUT_OK)
      return st;
  }
  int bits = 1;
  while ((int64_t(1) << bits) < T) bits++;
  const int passes = radix_passes(bits);
  // the duplication lands so that the last pass writes (pkA, sorted_ids)
  uint32_t *k0 = Q32(Lp.pkA), *v0 = sorted_ids, *k1 = Q32(Lp.pkB), *v1 = Q32(Lp.pvB);
  if (passes % 2 == 1) { std::swap(k0, k1); std::swap(v0, v1); }
  if (packed)
    duplicate_kernel<true><<<grid_for(nvis, kDupThreads), kDupThreads, 0, s>>>(
        E32(L.dvA), E32(L.offs), E32(L.pA), nullptr, n, ct, nvis, P, (uint32_t)T, k0, v0);
  else
    duplicate_kernel<false><<<grid_for(nvis, kDupThreads), kDupThreads, 0, s>>>(
        E32(L.dvA), E32(L.offs), nullptr, (const uint2*)(ews + L.geo), n, ct, nvis, P, (uint32_t)T, k0, v0);
  GUT_LAUNCH_CHECK();
  int inB = 0;
  return radix_sort_passes(k0, v0, k1, v1, (int64_t)P, nullptr, bits, 0, passes, pws + Lp.radix_tmp, s,
                           &inB, (uint2*)tile_ranges);
}

gut_status bin_order(const DevCam* dc, int n_cams, int64_t T, uint32_t* tile_ranges, hipStream_t s) {
  const CamTiles ct = cam_tiles(dc, n_cams);
  order_kernel<<<n_cams, kOrderThreads, 0, s>>>((uint2*)tile_ranges, ct, tile_ranges + 2 * T);
  GUT_LAUNCH_CHECK();
  return GUT_OK;
}

}  // namespace gut

using namespace gut;

extern "C" size_t gut_bin_workspace_bytes(int64_t n, int32_t n_cams, int64_t pair_capacity) {
  if (n < 0 || n_cams <= 0 || pair_capacity < 0) return 0;
  return bin_entry_bytes(n * n_cams) + bin_pair_bytes(pair_capacity);
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
  if (((uintptr_t)proj->rect & 7) || ((uintptr_t)tile_ranges & 7)) {
    set_error("rect and tile_ranges must be 8-byte aligned");
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
  const size_t eb = bin_entry_bytes(E), need = eb + bin_pair_bytes(pair_capacity);
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) {
    set_error("workspace must be 256-byte aligned and hold %zu bytes (got %zu)", need, ws_bytes);
    return GUT_E_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  char* ews = (char*)ws;
  char* pws = ews + eb;
  uint32_t nvis = 0;
  uint64_t P = 0;
  if ((st = bin_count(proj, (int)n, dc, n_cams, T, ews, tile_ranges, &nvis, &P, s)) != GUT_OK) return st;
  if (n_pairs) *n_pairs = (int64_t)P;
  if ((int64_t)P > pair_capacity) {
    (void)bin_order(dc, n_cams, T, tile_ranges, s);  // leaves every tile empty
    set_error("pair capacity %lld < required %llu", (long long)pair_capacity, (unsigned long long)P);
    return GUT_E_CAPACITY;
  }
  if ((st = bin_sort(proj, (int)n, dc, n_cams, T, E, ews, nvis, P, pws, tile_ranges, sorted_ids,
                     s)) != GUT_OK)
    return st;
  return bin_order(dc, n_cams, T, tile_ranges, s);
}
