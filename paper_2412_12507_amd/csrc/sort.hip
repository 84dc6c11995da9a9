// Device-wide exclusive scan and stable LSD radix sort of (key, value) pairs.
//
// Both process 4096-element chunks per 256-thread block (4 wave64s x 16
// items).  The scan is reduce -> (recursive) scan of chunk sums -> downsweep.
// Each radix pass (8-bit digits) is histogram -> per-digit scan of the
// digit-major count matrix (one block per digit) -> scatter.  The scatter
// ranks keys inside each wave with ballot-based peer masks (a key's rank
// among equal digits is the popcount of the lower peer lanes), keeps
// per-wave running digit counts in LDS, combines waves with one barrier
// (so the sort is stable without a block-wide sort), and reorders the chunk
// by digit in LDS before writing, so each digit's run is one coalesced write.
#include "common.h"

namespace gut {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kChunk = kThreads * kItems;  // 4096
constexpr int kWave = 64;

__device__ inline int lds_pad(int i) { return i + (i >> 5); }

// Exclusive scan of one value per thread across the block; returns the
// exclusive prefix and writes the block total.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) wsum[w] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kThreads / kWave; k++) {
    uint32_t s = wsum[k];
    if (k < w) pre += s;
    tot += s;
  }
  *total = tot;
  return pre + x - v;
}

__global__ void __launch_bounds__(kThreads) scan_reduce_kernel(const uint32_t* __restrict__ in,
                                                               int64_t n, uint32_t* __restrict__ sums) {
  __shared__ uint32_t wsum[kThreads / kWave];
  int64_t base = (int64_t)blockIdx.x * kChunk;
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < kItems; j++) {
    int64_t g = base + j * kThreads + threadIdx.x;
    if (g < n) acc += in[g];
  }
  uint32_t total;
  block_exclusive_scan(acc, wsum, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kThreads) scan_down_kernel(const uint32_t* __restrict__ in,
                                                             uint32_t* __restrict__ out, int64_t n,
                                                             const uint32_t* __restrict__ offs) {
  __shared__ uint32_t sm[kChunk + kChunk / 32];
  __shared__ uint32_t wsum[kThreads / kWave];
  int64_t base = (int64_t)blockIdx.x * kChunk;
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < kItems; j++) {
    int idx = j * kThreads + t;
    int64_t g = base + idx;
    sm[lds_pad(idx)] = g < n ? in[g] : 0u;
  }
  __syncthreads();
  uint32_t v[kItems], s = 0;
#pragma unroll
  for (int j = 0; j < kItems; j++) { v[j] = sm[lds_pad(t * kItems + j)]; s += v[j]; }
  uint32_t total;
  uint32_t run = block_exclusive_scan(s, wsum, &total) + (offs ? offs[blockIdx.x] : 0u);
#pragma unroll
  for (int j = 0; j < kItems; j++) { sm[lds_pad(t * kItems + j)] = run; run += v[j]; }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kItems; j++) {
    int idx = j * kThreads + t;
    int64_t g = base + idx;
    if (g < n) out[g] = sm[lds_pad(idx)];
  }
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t scan_temp_bytes(int64_t n) {
  size_t bytes = 0;
  while (n > kChunk) {
    int64_t nb = ceil_div(n, kChunk);
    bytes += 2 * align256(nb * sizeof(uint32_t));
    n = nb;
  }
  return bytes + 256;
}

gut_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* temp,
                              hipStream_t st) {
  if (n <= 0) return GUT_OK;
  if (n <= kChunk) {
    scan_down_kernel<<<1, kThreads, 0, st>>>(in, out, n, nullptr);
    GUT_LAUNCH_CHECK();
    return GUT_OK;
  }
  int64_t nb = ceil_div(n, kChunk);
  char* tp = (char*)temp;
  uint32_t* sums = (uint32_t*)tp;
  uint32_t* scanned = (uint32_t*)(tp + align256(nb * sizeof(uint32_t)));
  char* rest = tp + 2 * align256(nb * sizeof(uint32_t));
  scan_reduce_kernel<<<(unsigned)nb, kThreads, 0, st>>>(in, n, sums);
  GUT_LAUNCH_CHECK();
  gut_status s = exclusive_scan_u32(sums, scanned, nb, rest, st);
  if (s != GUT_OK) return s;
  scan_down_kernel<<<(unsigned)nb, kThreads, 0, st>>>(in, out, n, scanned);
  GUT_LAUNCH_CHECK();
  return GUT_OK;
}

// ------------------------------------------------------------------ radix sort

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

__global__ void __launch_bounds__(kThreads) radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                              int64_t n, int shift, uint32_t mask,
                                                              uint32_t* __restrict__ counts,
                                                              int64_t nblocks) {
  __shared__ uint32_t h[kRadix];
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kChunk;
  uint32_t kk[kItems];  // all loads first, then the LDS atomics
#pragma unroll
  for (int j = 0; j < kItems; j++) {
    int64_t g = base + j * kThreads + t;
    kk[j] = g < n ? keys[g] : 0xffffffffu;
  }
#pragma unroll
  for (int j = 0; j < kItems; j++) {
    int64_t g = base + j * kThreads + t;
    if (g < n) atomicAdd(&h[(kk[j] >> shift) & mask], 1u);
  }
  __syncthreads();
  counts[(int64_t)t * nblocks + blockIdx.x] = h[t];
}

// Per digit (one block each): exclusive scan of that digit's per-block
// counts in place of the count row, and the digit's total.
__global__ void __launch_bounds__(kThreads) radix_rowscan_kernel(const uint32_t* __restrict__ counts,
                                                                 uint32_t* __restrict__ offs,
                                                                 uint32_t* __restrict__ totals,
                                                                 int64_t nblocks) {
  __shared__ uint32_t wsum[kThreads / kWave];
  const int d = blockIdx.x;
  const uint32_t* row = counts + (int64_t)d * nblocks;
  uint32_t* orow = offs + (int64_t)d * nblocks;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nblocks; b0 += kThreads) {
    const int64_t b = b0 + threadIdx.x;
    const uint32_t v = b < nblocks ? row[b] : 0u;
    uint32_t total;
    const uint32_t pre = block_exclusive_scan(v, wsum, &total);
    if (b < nblocks) orow[b] = carry + pre;
    carry += total;
    __syncthreads();  // wsum is reused by the next chunk
  }
  if (threadIdx.x == 0) totals[d] = carry;
}

// Stable scatter of one 4096-key chunk.  Keys are ranked inside each wave
// with ballot peer masks (rank = popcount of lower lanes holding the same
// digit), waves are combined through per-wave digit counts, and the chunk is
// first reordered by digit in LDS so that each digit's run leaves the block
// as one contiguous, coalesced write.
__global__ void __launch_bounds__(kThreads) radix_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t n, int shift, int nbits, const uint32_t* __restrict__ offs,
    const uint32_t* __restrict__ totals, int64_t nblocks) {
  __shared__ uint32_t wh[kThreads / kWave][kRadix];
  __shared__ uint32_t goff[kRadix];    // global start of this block's run of digit d
  __shared__ uint32_t lstart[kRadix];  // start of digit d's run inside the chunk
  __shared__ uint32_t sk[kChunk];     // the chunk reordered by digit: keys, then values
  __shared__ uint32_t wsum[kThreads / kWave];
  const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
  const uint32_t mask = (1u << nbits) - 1u;
#pragma unroll
  for (int k = 0; k < kThreads / kWave; k++) wh[k][t] = 0;
  {  // digit bases: exclusive scan of the digit totals
    uint32_t tot;
    const uint32_t base = block_exclusive_scan(totals[t], wsum, &tot);
    goff[t] = base + offs[(int64_t)t * nblocks + blockIdx.x];
  }
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)w * (kChunk / 4);
  uint32_t kk[kItems], vv[kItems], rk[kItems];
#pragma unroll
  for (int r = 0; r < kItems; r++) {  // all loads first
    int64_t g = base + r * kWave + lane;
    kk[r] = g < n ? kin[g] : 0u;
    vv[r] = g < n ? vin[g] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kItems; r++) {
    int64_t g = base + r * kWave + lane;
    bool valid = g < n;
    uint32_t k = kk[r];
    uint32_t d = (k >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < nbits; b++) {
      bool bit = (d >> b) & 1u;
      uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    uint32_t before = (uint32_t)__popcll(peers & lt);
    uint32_t run = valid ? wh[w][d] : 0u;
    if (valid && before == 0) wh[w][d] = run + (uint32_t)__popcll(peers);
    rk[r] = valid ? run + before : 0xffffffffu;
  }
  __syncthreads();
  {  // per digit t: exclusive prefix over the waves, and the chunk's digit total
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kThreads / kWave; k++) {
      uint32_t c = wh[k][t];
      wh[k][t] = sum;
      sum += c;
    }
    uint32_t tot;
    lstart[t] = block_exclusive_scan(sum, wsum, &tot);
  }
  __syncthreads();
  uint32_t lp[kItems];  // each key's place in the chunk's digit order
#pragma unroll
  for (int r = 0; r < kItems; r++) {
    if (rk[r] == 0xffffffffu) { lp[r] = 0xffffffffu; continue; }
    const uint32_t d = (kk[r] >> shift) & mask;
    lp[r] = lstart[d] + wh[w][d] + rk[r];
    sk[lp[r]] = kk[r];
  }
  __syncthreads();
  const int cnt = (int)min((int64_t)kChunk, n - (int64_t)blockIdx.x * kChunk);
  uint32_t pos[kItems];  // output position of the chunk's j-th key, j = t + 256 i
#pragma unroll
  for (int i = 0; i < kItems; i++) {
    const int j = t + i * kThreads;
    if (j >= cnt) continue;
    const uint32_t k = sk[j];
    const uint32_t d = (k >> shift) & mask;
    pos[i] = goff[d] + (uint32_t)j - lstart[d];
    kout[pos[i]] = k;
  }
  __syncthreads();  // the same LDS now stages the values
#pragma unroll
  for (int r = 0; r < kItems; r++)
    if (lp[r] != 0xffffffffu) sk[lp[r]] = vv[r];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kItems; i++) {
    const int j = t + i * kThreads;
    if (j < cnt) vout[pos[i]] = sk[j];
  }
}

int64_t radix_blocks(int64_t n) { return ceil_div(n > 0 ? n : 1, kChunk); }

size_t radix_temp_bytes(int64_t n) {
  int64_t nb = radix_blocks(n);
  size_t cnt = align256((size_t)kRadix * nb * sizeof(uint32_t));
  return 2 * cnt + align256(kRadix * sizeof(uint32_t));
}

gut_status radix_sort_pairs_pp(uint32_t* kA, uint32_t* vA, uint32_t* kB, uint32_t* vB, int64_t n,
                               int bits, void* temp, hipStream_t st, int* result_in_b) {
  *result_in_b = 0;
  if (n <= 0) return GUT_OK;
  int passes = (bits + kRadixBits - 1) / kRadixBits;
  if (passes < 1) passes = 1;
  // spread the bits evenly over the passes (14 bits: 7 + 7, not 8 + 6), so
  // no pass scatters into more digit runs than it must
  const int per = (bits + passes - 1) / passes;
  int64_t nb = radix_blocks(n);
  size_t cnt_bytes = align256((size_t)kRadix * nb * sizeof(uint32_t));
  uint32_t* counts = (uint32_t*)temp;
  uint32_t* offs = (uint32_t*)((char*)temp + cnt_bytes);
  uint32_t* totals = (uint32_t*)((char*)temp + 2 * cnt_bytes);
  uint32_t *ks = kA, *vs = vA;
  for (int p = 0; p < passes; p++) {
    uint32_t* kd = ks == kA ? kB : kA;
    uint32_t* vd = ks == kA ? vB : vA;
    int shift = p * per;
    int nbits = bits - shift < per ? bits - shift : per;
    radix_hist_kernel<<<(unsigned)nb, kThreads, 0, st>>>(ks, n, shift, (1u << nbits) - 1u, counts, nb);
    GUT_LAUNCH_CHECK();
    radix_rowscan_kernel<<<kRadix, kThreads, 0, st>>>(counts, offs, totals, nb);
    GUT_LAUNCH_CHECK();
    radix_scatter_kernel<<<(unsigned)nb, kThreads, 0, st>>>(ks, vs, kd, vd, n, shift, nbits, offs,
                                                            totals, nb);
    GUT_LAUNCH_CHECK();
    ks = kd;
    vs = vd;
  }
  *result_in_b = ks == kB;
  return GUT_OK;
}

}  // namespace gut
