// Tile binning: the global per-tile depth sort of Sec. 4.3.
//
// Order of work (E = n_cams * n entries, P = pairs):
//   1. compact the visible entries into (depth bits, entry id), in id order,
//      and total the pairs P                       (reduce + scan + emit)
//   2. read back (N_vis, P): the one host synchronisation of the path
//   3. stable LSD radix sort of the N_vis entries by depth (32 bits)
//   4. scan of tiles touched in depth order -> pair offsets
//   5. duplicate: each entry writes (global tile id, entry id) for every
//      tile of its rectangle at its offset
//   6. stable LSD radix sort of the P pairs by tile id (ceil(log2 T) bits)
//   7. per-tile [start, end) ranges
// Sorting entries by depth first and then pairs by tile only gives exactly the
// (tile, depth, id) order of a full-key sort while moving far fewer bytes:
// the tile sort carries 4-byte keys over ceil(log2 T)/8 passes instead of
// 8-byte keys over (32 + log2 T)/8 passes.
#include <cstring>

#include "common.h"

namespace gut {

constexpr int kBThreads = 256;
constexpr int kBItems = 16;
constexpr int kBChunk = kBThreads * kBItems;

struct CamTiles {
  int base[kMaxCams];
  int tx[kMaxCams];
  int count[kMaxCams];
};

static size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace of the entry phase (sized by E = n_cams * n) and of the pair
// phase (sized by the pair capacity).
struct EntryLayout {
  size_t vis_part, vis_scan, vis_tmp, scalars, dkA, dvA, dkB, dvB, cnt, offs, offs_tmp, radix_tmp,
      total;
};
struct PairLayout {
  size_t pkA, pkB, pvB, radix_tmp, total;
};

static EntryLayout entry_layout(int64_t E) {
  EntryLayout L;
  int64_t nb = (E + kBChunk - 1) / kBChunk;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += al(bytes); return r; };
  L.vis_part = take(nb * 4);
  L.vis_scan = take(nb * 4);
  L.vis_tmp = take(scan_temp_bytes(nb));
  L.scalars = take(64);
  L.dkA = take(E * 4);
  L.dvA = take(E * 4);
  L.dkB = take(E * 4);
  L.dvB = take(E * 4);
  L.cnt = take(E * 4);
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

__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kBThreads / 64; k++) {
    uint32_t s = wsum[k];
    if (k < w) pre += s;
    tot += s;
  }
  *total = tot;
  return pre + x - v;
}

__global__ void __launch_bounds__(kBThreads) vis_reduce_kernel(const uint32_t* __restrict__ tiles,
                                                               int64_t E, uint32_t* __restrict__ part,
                                                               unsigned long long* __restrict__ ptotal) {
  __shared__ uint32_t wsum[kBThreads / 64];
  __shared__ unsigned long long wp[kBThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kBChunk;
  uint32_t cnt = 0;
  unsigned long long pairs = 0;
#pragma unroll
  for (int j = 0; j < kBItems; j++) {
    int64_t g = base + j * kBThreads + threadIdx.x;
    uint32_t t = g < E ? tiles[g] : 0u;
    cnt += t > 0;
    pairs += t;
  }
  for (int o = 32; o > 0; o >>= 1) pairs += __shfl_xor(pairs, o, 64);
  if ((threadIdx.x & 63) == 0) wp[threadIdx.x >> 6] = pairs;
  uint32_t total;
  block_excl_scan(cnt, wsum, &total);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = total;
    unsigned long long s = 0;
    for (int k = 0; k < kBThreads / 64; k++) s += wp[k];
    atomicAdd(ptotal, s);
  }
}

__global__ void __launch_bounds__(kBThreads) vis_emit_kernel(
    const uint32_t* __restrict__ tiles, const float* __restrict__ depth, int64_t E,
    const uint32_t* __restrict__ offs, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
    uint32_t* __restrict__ nvis, int64_t nblocks) {
  __shared__ uint32_t sm[kBChunk + kBChunk / 32];
  __shared__ uint32_t wsum[kBThreads / 64];
  const int t = threadIdx.x;
  int64_t base = (int64_t)blockIdx.x * kBChunk;
  auto pad = [](int i) { return i + (i >> 5); };
#pragma unroll
  for (int j = 0; j < kBItems; j++) {
    int idx = j * kBThreads + t;
    int64_t g = base + idx;
    sm[pad(idx)] = (g < E && tiles[g] > 0) ? 1u : 0u;
  }
  __syncthreads();
  uint32_t v[kBItems], s = 0;
#pragma unroll
  for (int j = 0; j < kBItems; j++) { v[j] = sm[pad(t * kBItems + j)]; s += v[j]; }
  uint32_t total;
  uint32_t run = block_excl_scan(s, wsum, &total) + offs[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kBItems; j++) { sm[pad(t * kBItems + j)] = run; run += v[j]; }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kBItems; j++) {
    int idx = j * kBThreads + t;
    int64_t g = base + idx;
    if (g < E && tiles[g] > 0) {
      uint32_t pos = sm[pad(idx)];
      keys[pos] = __float_as_uint(depth[g]);
      vals[pos] = (uint32_t)g;
    }
  }
  if (blockIdx.x == nblocks - 1 && t == 0) *nvis = offs[blockIdx.x] + total;
}

__global__ void gather_tiles_kernel(const uint32_t* __restrict__ ent, const uint32_t* __restrict__ tiles,
                                    int64_t m, uint32_t* __restrict__ out) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) out[j] = tiles[ent[j]];
}

// Expands each visible entry (in depth order) into one (tile, entry) pair per
// tile of its rectangle, row-major.  A block takes 256 consecutive entries
// and spreads their contiguous output range evenly over its threads (each
// output finds its entry by binary search of the block's offsets in LDS), so
// the writes are coalesced whatever the rectangle sizes.
constexpr int kDupThreads = 256;
__global__ void __launch_bounds__(kDupThreads) duplicate_kernel(
    const uint32_t* __restrict__ ent, const uint32_t* __restrict__ offs,
    const short4* __restrict__ rect, int n, CamTiles ct, int64_t m, uint64_t P,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  __shared__ uint32_t so[kDupThreads + 1];
  __shared__ uint32_t se[kDupThreads];
  __shared__ int4 sr[kDupThreads];  // x0, y0, width, camera tile base
  __shared__ int stx[kDupThreads];
  const int t = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * kDupThreads;
  const int cnt = (int)min((int64_t)kDupThreads, m - j0);
  if (t < cnt) {
    const uint32_t e = ent[j0 + t];
    const int cam = (int)(e / (uint32_t)n);
    const short4 r = rect[e];
    so[t] = offs[j0 + t];
    se[t] = e;
    sr[t] = make_int4(r.x, r.y, r.z - r.x + 1, ct.base[cam]);
    stx[t] = ct.tx[cam];
  }
  if (t == 0) so[cnt] = j0 + cnt < m ? offs[j0 + cnt] : (uint32_t)P;
  __syncthreads();
  const uint32_t p1 = so[cnt];
  for (uint32_t p = so[0] + t; p < p1; p += kDupThreads) {
    int lo = 0, hi = cnt - 1;  // last entry whose output starts at or before p
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (so[mid] <= p) lo = mid; else hi = mid - 1;
    }
    const int4 r = sr[lo];
    const uint32_t k = p - so[lo];
    const uint32_t y = k / (uint32_t)r.z, x = k - y * (uint32_t)r.z;
    keys[p] = (uint32_t)(r.w + (r.y + (int)y) * stx[lo] + r.x + (int)x);
    vals[p] = se[lo];
  }
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, int64_t m, uint32_t v) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) p[j] = v;
}

__global__ void ranges_kernel(const uint32_t* __restrict__ keys, int64_t m, uint2* __restrict__ ranges) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  uint32_t k = keys[i];
  if (i == 0 || keys[i - 1] != k) ranges[k].x = (uint32_t)i;
  if (i == m - 1 || keys[i + 1] != k) ranges[k].y = (uint32_t)(i + 1);
}

// Render order of one camera's tiles (one block per camera): a counting sort
// of the tiles by bucket = bit length of the list length, longest first.
// Only the schedule depends on it (every tile is rendered independently), so
// the order within a bucket may vary from call to call.
constexpr int kOrderThreads = 1024;
__global__ void __launch_bounds__(kOrderThreads) order_kernel(const uint2* __restrict__ ranges,
                                                             CamTiles ct, uint32_t* __restrict__ order) {
  __shared__ unsigned cnt[33], cur[33];
  const int c = blockIdx.x, base = ct.base[c], nt = ct.count[c];
  for (int b = threadIdx.x; b < 33; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  for (int t = threadIdx.x; t < nt; t += blockDim.x) {
    const uint2 r = ranges[base + t];
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
    const uint2 r = ranges[base + t];
    const unsigned pos = atomicAdd(&cur[__clz(r.y - r.x)], 1u);
    order[base + pos] = (uint32_t)t;
  }
}

// Pinned host slot for the count read-back, one per host thread.
struct PinnedSlot {
  void* p = nullptr;
  ~PinnedSlot() {
    if (p) (void)hipHostFree(p);
  }
};
static thread_local PinnedSlot g_pinned;

static inline unsigned grid_for(int64_t m, int threads) {
  return (unsigned)((m + threads - 1) / threads);
}

gut_status fill_u32(uint32_t* p, int64_t m, uint32_t v, hipStream_t st) {
  if (m <= 0) return GUT_OK;
  fill_u32_kernel<<<grid_for(m, 256), 256, 0, st>>>(p, m, v);
  GUT_LAUNCH_CHECK();
  return GUT_OK;
}

// Phase 1: compaction of the visible entries into (depth bits, id) and the
// pair total; reads back (N_vis, P) -- the one host synchronisation.
gut_status bin_count(const gut_projected* proj, int64_t E, char* ews, uint32_t* nvis_out,
                     uint64_t* P_out, hipStream_t s) {
  EntryLayout L = entry_layout(E);
  auto P32 = [&](size_t off) { return (uint32_t*)(ews + off); };
  uint32_t* scal = P32(L.scalars);
  unsigned long long* ptotal = (unsigned long long*)(scal + 2);
  *nvis_out = 0;
  *P_out = 0;
  if (E == 0) return GUT_OK;
  gut_status st;
  if ((st = fill_u32(scal, 16, 0u, s)) != GUT_OK) return st;
  int64_t nb = (E + kBChunk - 1) / kBChunk;
  vis_reduce_kernel<<<(unsigned)nb, kBThreads, 0, s>>>(proj->tiles, E, P32(L.vis_part), ptotal);
  GUT_LAUNCH_CHECK();
  if ((st = exclusive_scan_u32(P32(L.vis_part), P32(L.vis_scan), nb, ews + L.vis_tmp, s)) != GUT_OK)
    return st;
  vis_emit_kernel<<<(unsigned)nb, kBThreads, 0, s>>>(proj->tiles, proj->depth, E, P32(L.vis_scan),
                                                      P32(L.dkA), P32(L.dvA), scal, nb);
  GUT_LAUNCH_CHECK();
  if (!g_pinned.p) GUT_HIP(hipHostMalloc(&g_pinned.p, 64, hipHostMallocDefault));
  GUT_HIP(hipMemcpyAsync(g_pinned.p, scal, 16, hipMemcpyDeviceToHost, s));
  GUT_HIP(hipStreamSynchronize(s));
  uint32_t nvis;
  unsigned long long P;
  std::memcpy(&nvis, g_pinned.p, 4);
  std::memcpy(&P, (char*)g_pinned.p + 8, 8);
  *nvis_out = nvis;
  *P_out = P;
  return GUT_OK;
}

// Phase 2: depth sort, duplicate, tile sort, ranges.  tile_ranges must
// already be zero; sorted_ids and the pair workspace hold at least P pairs.
gut_status bin_sort(const gut_projected* proj, int n, const DevCam* dc, int n_cams, int64_t T,
                    int64_t E, char* ews, uint32_t nvis, uint64_t P, char* pws,
                    uint32_t* tile_ranges, uint32_t* sorted_ids, hipStream_t s) {
  if (nvis == 0 || P == 0) return GUT_OK;
  EntryLayout L = entry_layout(E);
  PairLayout Lp = pair_layout((int64_t)P);
  auto E32 = [&](size_t off) { return (uint32_t*)(ews + off); };
  auto Q32 = [&](size_t off) { return (uint32_t*)(pws + off); };
  gut_status st;
  int inB = 0;
  if ((st = radix_sort_pairs_pp(E32(L.dkA), E32(L.dvA), E32(L.dkB), E32(L.dvB), nvis, 32,
                                ews + L.radix_tmp, s, &inB)) != GUT_OK)
    return st;
  uint32_t* ent = inB ? E32(L.dvB) : E32(L.dvA);
  gather_tiles_kernel<<<grid_for(nvis, 256), 256, 0, s>>>(ent, proj->tiles, nvis, E32(L.cnt));
  GUT_LAUNCH_CHECK();
  if ((st = exclusive_scan_u32(E32(L.cnt), E32(L.offs), nvis, ews + L.offs_tmp, s)) != GUT_OK)
    return st;
  CamTiles ct;
  for (int c = 0; c < n_cams; c++) { ct.base[c] = dc[c].tile_base; ct.tx[c] = dc[c].tiles_x; }
  duplicate_kernel<<<grid_for(nvis, kDupThreads), kDupThreads, 0, s>>>(
      ent, E32(L.offs), (const short4*)proj->rect, n, ct, nvis, P, Q32(Lp.pkA), sorted_ids);
  GUT_LAUNCH_CHECK();
  int bits = 1;
  while ((int64_t(1) << bits) < T) bits++;
  if ((st = radix_sort_pairs_pp(Q32(Lp.pkA), sorted_ids, Q32(Lp.pkB), Q32(Lp.pvB), (int64_t)P,
                                bits, pws + Lp.radix_tmp, s, &inB)) != GUT_OK)
    return st;
  uint32_t* keys = inB ? Q32(Lp.pkB) : Q32(Lp.pkA);
  if (inB) GUT_HIP(hipMemcpyAsync(sorted_ids, Q32(Lp.pvB), P * 4, hipMemcpyDeviceToDevice, s));
  ranges_kernel<<<grid_for((int64_t)P, 256), 256, 0, s>>>(keys, (int64_t)P, (uint2*)tile_ranges);
  GUT_LAUNCH_CHECK();
  return GUT_OK;
}

// Render order after the ranges (tile_ranges[2T .. 3T)).
gut_status bin_order(const DevCam* dc, int n_cams, int64_t T, uint32_t* tile_ranges, hipStream_t s) {
  CamTiles ct;
  for (int c = 0; c < n_cams; c++) {
    ct.base[c] = dc[c].tile_base;
    ct.tx[c] = dc[c].tiles_x;
    ct.count[c] = dc[c].tiles_x * dc[c].tiles_y;
  }
  order_kernel<<<n_cams, kOrderThreads, 0, s>>>((const uint2*)tile_ranges, ct, tile_ranges + 2 * T);
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
  if ((st = fill_u32(tile_ranges, 2 * T, 0u, s)) != GUT_OK) return st;
  uint32_t nvis = 0;
  uint64_t P = 0;
  if ((st = bin_count(proj, E, ews, &nvis, &P, s)) != GUT_OK) return st;
  if (n_pairs) *n_pairs = (int64_t)P;
  if ((int64_t)P > pair_capacity) {
    set_error("pair capacity %lld < required %llu", (long long)pair_capacity, (unsigned long long)P);
    return GUT_E_CAPACITY;
  }
  if ((st = bin_sort(proj, (int)n, dc, n_cams, T, E, ews, nvis, P, pws, tile_ranges, sorted_ids,
                     s)) != GUT_OK)
    return st;
  return bin_order(dc, n_cams, T, tile_ranges, s);
}
