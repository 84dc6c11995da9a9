// Building blocks of the stable LSD radix sort, shared by the plain sort
// (sort.hip) and the binning kernels that generate their keys on the fly
// (bin.hip).  Not part of the ABI.
//
// A pass works on 4096-item chunks, one per 256-thread block (4 wave64s x 16
// items): item r of wave w, lane l of chunk c is item c*4096 + w*1024 + r*64 + l.
// Each pass is histogram -> per-digit scan of the digit-major count matrix
// (one block per digit) -> scatter.  The scatter ranks keys inside each wave
// with ballot peer masks (a key's rank among equal digits is the popcount of
// the lower peer lanes), keeps per-wave running digit counts in LDS, combines
// the waves with one barrier (so the sort is stable without a block-wide
// sort), and reorders the chunk by digit in LDS before writing, so that each
// digit's run leaves the block as one contiguous, coalesced write.
#pragma once

#include "common.h"

namespace gut {

constexpr int kRThreadsSort = 256;
constexpr int kRItems = 16;
constexpr int kRChunk = kRThreadsSort * kRItems;  // 4096
constexpr int kRWave = 64;
constexpr int kRWaves = kRThreadsSort / kRWave;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

// Exclusive scan of one value per thread across a 256-thread block; returns
// the thread's exclusive prefix and the block total.
__device__ inline uint32_t radix_block_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const int lane = threadIdx.x & (kRWave - 1), w = threadIdx.x / kRWave;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < kRWave; o <<= 1) {
    uint32_t y = __shfl_up(x, o, kRWave);
    if (lane >= o) x += y;
  }
  if (lane == kRWave - 1) wsum[w] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kRWaves; k++) {
    uint32_t s = wsum[k];
    if (k < w) pre += s;
    tot += s;
  }
  *total = tot;
  return pre + x - v;
}

// Per-block digit histogram of the valid keys (bit r of vmask marks item r),
// written to counts[digit * nblocks + block].  h: kRadix words of LDS.
__device__ inline void radix_hist_store(const uint32_t (&kk)[kRItems], uint32_t vmask, int shift,
                                        uint32_t mask, uint32_t* h, uint32_t* __restrict__ counts,
                                        int64_t nblocks) {
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRItems; r++)
    if ((vmask >> r) & 1u) atomicAdd(&h[(kk[r] >> shift) & mask], 1u);
  __syncthreads();
  counts[(int64_t)t * nblocks + blockIdx.x] = h[t];
}

// The chunk a scatter block takes.  Blocks are dealt to the 8 XCDs in turn
// (block b to XCD b % 8), so chunk = b would give neighbouring chunks, whose
// runs of a digit are neighbours in the output, to different L2s, and each
// would write its runs back as partial lines.  Instead XCD x takes the
// contiguous chunks [x q + min(x, r), ...) of the nact = 8 q + r chunks that
// hold items, in order (a bijection on blocks 0 .. nact-1: XCD x receives
// exactly q + (x < r) of them); blocks from nact on get -1 and stay idle.
__device__ inline int64_t radix_xcd_chunk(int64_t nact) {
  const int64_t b = blockIdx.x, x = b & 7, k = b >> 3;
  if (b >= nact) return -1;
  const int64_t q = nact >> 3, r = nact & 7;
  return x * q + (x < r ? x : r) + k;
}

// LDS of one scatter block's ranking; the chunk is reordered by digit through
// a separate kRChunk-word staging array (keys, then values).
struct RadixRankSmem {
  uint32_t wh[kRWaves][kRadix];  // per-wave running digit counts, then wave prefixes
  uint32_t goff[kRadix];         // global start of this block's run of digit d
  uint32_t lstart[kRadix];       // start of digit d's run inside the chunk
  uint32_t wsum[kRWaves];
};

// Where a pass's sorted keys and values go.  The plain sink writes them to
// kout / vout (kout may be null: keys not kept); with ranges (the last pass,
// where the sorted key is the whole key) it also records each key's
// [start, end) in the output through atomicMin / atomicMax on ranges[key],
// initialised by the caller to (~0u, 0).
struct KVSink {
  uint32_t* kout;
  uint32_t* vout;
  uint2* ranges;
  uint32_t* pout;  // payload (sorts that carry one)
  __device__ uint2* bounds() const { return ranges; }
  __device__ void key(uint32_t pos, uint32_t k) const {
    if (kout) kout[pos] = k;
  }
  // values of the chunk's items j = t + 256 i (valid for j < cnt) at pos[i]
  __device__ void vals(const uint32_t (&pos)[kRItems], const uint32_t (&v)[kRItems], int t,
                       uint32_t cnt) const {
#pragma unroll
    for (int i = 0; i < kRItems; i++)
      if (t + i * kRThreadsSort < (int)cnt) vout[pos[i]] = v[i];
  }
  __device__ void pays(const uint32_t (&pos)[kRItems], const uint32_t (&p)[kRItems], int t,
                       uint32_t cnt) const {
#pragma unroll
    for (int i = 0; i < kRItems; i++)
      if (t + i * kRThreadsSort < (int)cnt) pout[pos[i]] = p[i];
  }
};

// Stable scatter of one chunk held in registers (item r of this thread is
// chunk item w*1024 + r*64 + lane; bit r of vmask marks it valid).  offs and
// totals come from the per-digit scan of the pass's count matrix; sk is a
// kRChunk-word LDS staging array.  With PAY, a 32-bit payload pp travels
// with each key (sink.pays) through one more staging round.
template <bool PAY, class Sink>
__device__ inline void radix_scatter_chunk(const uint32_t (&kk)[kRItems], const uint32_t (&vv)[kRItems],
                                           const uint32_t (&pp)[kRItems], uint32_t vmask, int shift,
                                           int nbits,
                                           const uint32_t* __restrict__ offs,
                                           const uint32_t* __restrict__ totals, int64_t nblocks,
                                           int64_t chunk, const Sink& sink, RadixRankSmem& S,
                                           uint32_t* __restrict__ sk) {
  const int t = threadIdx.x, lane = t & (kRWave - 1), w = t / kRWave;
  const uint32_t mask = (1u << nbits) - 1u;
#pragma unroll
  for (int k = 0; k < kRWaves; k++) S.wh[k][t] = 0;
  {  // digit bases: exclusive scan of the digit totals
    uint32_t tot;
    const uint32_t base = radix_block_scan(totals[t], S.wsum, &tot);
    S.goff[t] = base + offs[(int64_t)t * nblocks + chunk];
  }
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kRWave - lane));
  uint32_t rk[kRItems];
#pragma unroll
  for (int r = 0; r < kRItems; r++) {
    const bool valid = (vmask >> r) & 1u;
    const uint32_t d = (kk[r] >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < nbits; b++) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t before = (uint32_t)__popcll(peers & lt);
    const uint32_t run = valid ? S.wh[w][d] : 0u;
    if (valid && before == 0) S.wh[w][d] = run + (uint32_t)__popcll(peers);
    rk[r] = run + before;
  }
  __syncthreads();
  uint32_t cnt;  // valid keys in the chunk
  {  // per digit t: exclusive prefix over the waves, and the chunk's digit total
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kRWaves; k++) {
      const uint32_t c = S.wh[k][t];
      S.wh[k][t] = sum;
      sum += c;
    }
    S.lstart[t] = radix_block_scan(sum, S.wsum, &cnt);
  }
  __syncthreads();
  uint32_t lp[kRItems];  // each key's place in the chunk's digit order
#pragma unroll
  for (int r = 0; r < kRItems; r++) {
    if (!((vmask >> r) & 1u)) continue;
    const uint32_t d = (kk[r] >> shift) & mask;
    lp[r] = S.lstart[d] + S.wh[w][d] + rk[r];
    sk[lp[r]] = kk[r];
  }
  __syncthreads();
  uint2* const ranges = sink.bounds();
  uint32_t pos[kRItems];  // output position of the chunk's j-th key, j = t + 256 i
#pragma unroll
  for (int i = 0; i < kRItems; i++) {
    const int j = t + i * kRThreadsSort;
    if (j >= (int)cnt) continue;
    const uint32_t k = sk[j];
    const uint32_t d = (k >> shift) & mask;
    pos[i] = S.goff[d] + (uint32_t)j - S.lstart[d];
    sink.key(pos[i], k);
    if (ranges) {
      // in the last pass the keys of a digit's run are ascending, so a key's
      // first and last places in the chunk bound its run in the output
      if (j == 0 || sk[j - 1] != k) atomicMin(&ranges[k].x, pos[i]);
      if (j == (int)cnt - 1 || sk[j + 1] != k) atomicMax(&ranges[k].y, pos[i] + 1u);
    }
  }
  __syncthreads();  // the same LDS now stages the values
#pragma unroll
  for (int r = 0; r < kRItems; r++)
    if ((vmask >> r) & 1u) sk[lp[r]] = vv[r];
  __syncthreads();
  uint32_t vj[kRItems];
#pragma unroll
  for (int i = 0; i < kRItems; i++) {
    const int j = t + i * kRThreadsSort;
    vj[i] = j < (int)cnt ? sk[j] : 0u;
  }
  sink.vals(pos, vj, t, cnt);
  if constexpr (PAY) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRItems; r++)
      if ((vmask >> r) & 1u) sk[lp[r]] = pp[r];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRItems; i++) {
      const int j = t + i * kRThreadsSort;
      vj[i] = j < (int)cnt ? sk[j] : 0u;
    }
    sink.pays(pos, vj, t, cnt);
  }
}

// Items of this block's chunk: (key, value[, payload]) below the count n
// (vin / pin may be null when not wanted).
__device__ inline uint32_t radix_load_kv(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                         const uint32_t* __restrict__ pin, int64_t n, int64_t chunk,
                                         uint32_t (&kk)[kRItems], uint32_t (&vv)[kRItems],
                                         uint32_t (&pp)[kRItems]) {
  const int lane = threadIdx.x & (kRWave - 1), w = threadIdx.x / kRWave;
  const int64_t base = chunk * kRChunk + (int64_t)w * (kRChunk / kRWaves);
  uint32_t vmask = 0;
#pragma unroll
  for (int r = 0; r < kRItems; r++) {
    const int64_t g = base + r * kRWave + lane;
    const bool valid = g < n;
    kk[r] = valid ? kin[g] : 0u;
    if (vin) vv[r] = valid ? vin[g] : 0u;
    if (pin) pp[r] = valid ? pin[g] : 0u;
    vmask |= (uint32_t)valid << r;
  }
  return vmask;
}

// Histogram of one pass over keys[0, n) (n = *n_dev when given, else n_max).
gut_status radix_hist(const uint32_t* keys, int64_t n_max, const uint32_t* n_dev, int shift,
                      uint32_t mask, uint32_t* counts, int64_t nblocks, hipStream_t st);

// Per-block totals that the first pass's histogram leaves for the host: the
// rowscan reduces them in one extra block to (sum of n, sum of p) and writes
// them to dev (uint32 n at dev[0], uint64 p at dev[2..3]) and to the host
// buffer (same layout), which the host may read once the launch is done.
struct RowscanTail {
  const uint32_t* part_n;
  const unsigned long long* part_p;
  int64_t count;
  uint32_t* dev;
  void* host;
};

// Per digit (one block each, kRadix blocks): exclusive scan of that digit's
// per-block counts into offs, and the digit's total.
gut_status radix_rowscan(const uint32_t* counts, uint32_t* offs, uint32_t* totals, int64_t nblocks,
                         hipStream_t st, const RowscanTail* tail = nullptr);

// The count matrix, its scan and the digit totals of one pass over up to
// n_max items, carved from one workspace of radix_temp_bytes(n_max).
struct RadixTemp {
  uint32_t *counts, *offs, *totals;
};
RadixTemp radix_temp(void* temp, int64_t n_max);

// Bits per pass when `bits` key bits are sorted in ceil(bits / 8) passes:
// spread evenly (14 bits: 7 + 7, not 8 + 6), so no pass scatters into more
// digit runs than it must.
inline int radix_passes(int bits) { return bits <= kRadixBits ? 1 : (bits + kRadixBits - 1) / kRadixBits; }
inline int radix_per_pass(int bits) {
  const int p = radix_passes(bits);
  return (bits + p - 1) / p;
}

}  // namespace gut
