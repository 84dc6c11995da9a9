// Device-wide exclusive scan and stable LSD radix sort of (key, value) pairs.
//
// Both process 4096-element chunks per 256-thread block (4 wave64s x 16
// items).  The scan is reduce -> (recursive) scan of chunk sums -> downsweep.
// The radix passes (histogram -> per-digit scan -> scatter) are built from
// the blocks in radix.h; a pass may take its item count from device memory,
// so a sort can be queued before the host knows how many items it will see
// (the grid covers the upper bound and the blocks past the count stay idle).
#include "radix.h"

namespace gut {

__device__ inline int lds_pad(int i) { return i + (i >> 5); }

__global__ void __launch_bounds__(kRThreadsSort) scan_reduce_kernel(const uint32_t* __restrict__ in,
                                                                    int64_t n, uint32_t* __restrict__ sums) {
  __shared__ uint32_t wsum[kRWaves];
  int64_t base = (int64_t)blockIdx.x * kRChunk;
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < kRItems; j++) {
    int64_t g = base + j * kRThreadsSort + threadIdx.x;
    if (g < n) acc += in[g];
  }
  uint32_t total;
  radix_block_scan(acc, wsum, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kRThreadsSort) scan_down_kernel(const uint32_t* __restrict__ in,
                                                                  uint32_t* __restrict__ out, int64_t n,
                                                                  const uint32_t* __restrict__ offs) {
  __shared__ uint32_t sm[kRChunk + kRChunk / 32];
  __shared__ uint32_t wsum[kRWaves];
  int64_t base = (int64_t)blockIdx.x * kRChunk;
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < kRItems; j++) {
    int idx = j * kRThreadsSort + t;
    int64_t g = base + idx;
    sm[lds_pad(idx)] = g < n ? in[g] : 0u;
  }
  __syncthreads();
  uint32_t v[kRItems], s = 0;
#pragma unroll
  for (int j = 0; j < kRItems; j++) { v[j] = sm[lds_pad(t * kRItems + j)]; s += v[j]; }
  uint32_t total;
  uint32_t run = radix_block_scan(s, wsum, &total) + (offs ? offs[blockIdx.x] : 0u);
#pragma unroll
  for (int j = 0; j < kRItems; j++) { sm[lds_pad(t * kRItems + j)] = run; run += v[j]; }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kRItems; j++) {
    int idx = j * kRThreadsSort + t;
    int64_t g = base + idx;
    if (g < n) out[g] = sm[lds_pad(idx)];
  }
}

// Downsweep for up to kRChunk chunks whose sums are not yet scanned: each
// block first reduces the sums of the chunks before it (a few hundred words
// at the sizes here), so the scan of the sums needs no launch of its own.
__global__ void __launch_bounds__(kRThreadsSort) scan_down_sums_kernel(const uint32_t* __restrict__ in,
                                                                       uint32_t* __restrict__ out, int64_t n,
                                                                       const uint32_t* __restrict__ sums) {
  __shared__ uint32_t sm[kRChunk + kRChunk / 32];
  __shared__ uint32_t wsum[kRWaves];
  const int t = threadIdx.x;
  uint32_t pre = 0;
  for (int k = t; k < (int)blockIdx.x; k += kRThreadsSort) pre += sums[k];
  uint32_t offset;
  radix_block_scan(pre, wsum, &offset);  // offset = the block total of pre
  __syncthreads();                        // wsum is reused below
  int64_t base = (int64_t)blockIdx.x * kRChunk;
#pragma unroll
  for (int j = 0; j < kRItems; j++) {
    int idx = j * kRThreadsSort + t;
    int64_t g = base + idx;
    sm[lds_pad(idx)] = g < n ? in[g] : 0u;
  }
  __syncthreads();
  uint32_t v[kRItems], s = 0;
#pragma unroll
  for (int j = 0; j < kRItems; j++) { v[j] = sm[lds_pad(t * kRItems + j)]; s += v[j]; }
  uint32_t total;
  uint32_t run = radix_block_scan(s, wsum, &total) + offset;
#pragma unroll
  for (int j = 0; j < kRItems; j++) { sm[lds_pad(t * kRItems + j)] = run; run += v[j]; }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kRItems; j++) {
    int idx = j * kRThreadsSort + t;
    int64_t g = base + idx;
    if (g < n) out[g] = sm[lds_pad(idx)];
  }
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t scan_temp_bytes(int64_t n) {
  size_t bytes = 0;
  while (n > kRChunk) {
    int64_t nb = ceil_div(n, kRChunk);
    bytes += 2 * align256(nb * sizeof(uint32_t));
    n = nb;
  }
  return bytes + 256;
}

gut_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* temp, hipStream_t st,
                              bool have_sums) {
  if (n <= 0) return GUT_OK;
  if (n <= kRChunk) {
    scan_down_kernel<<<1, kRThreadsSort, 0, st>>>(in, out, n, nullptr);
    GUT_LAUNCH_CHECK();
    return GUT_OK;
  }
  int64_t nb = ceil_div(n, kRChunk);
  char* tp = (char*)temp;
  uint32_t* sums = (uint32_t*)tp;
  uint32_t* scanned = (uint32_t*)(tp + align256(nb * sizeof(uint32_t)));
  char* rest = tp + 2 * align256(nb * sizeof(uint32_t));
  if (!have_sums) {
    scan_reduce_kernel<<<(unsigned)nb, kRThreadsSort, 0, st>>>(in, n, sums);
    GUT_LAUNCH_CHECK();
  }
  if (nb <= kRChunk) {  // one level: the downsweep reduces the sums before each chunk itself
    scan_down_sums_kernel<<<(unsigned)nb, kRThreadsSort, 0, st>>>(in, out, n, sums);
    GUT_LAUNCH_CHECK();
    return GUT_OK;
  }
  gut_status s = exclusive_scan_u32(sums, scanned, nb, rest, st, false);
  if (s != GUT_OK) return s;
  scan_down_kernel<<<(unsigned)nb, kRThreadsSort, 0, st>>>(in, out, n, scanned);
  GUT_LAUNCH_CHECK();
  return GUT_OK;
}

// ------------------------------------------------------------------ radix sort

__global__ void __launch_bounds__(kRThreadsSort) radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                                   int64_t n_max, const uint32_t* n_dev,
                                                                   int shift, uint32_t mask,
                                                                   uint32_t* __restrict__ counts,
                                                                   int64_t nblocks) {
  __shared__ uint32_t h[kRadix];
  const int64_t n = n_dev ? (int64_t)*n_dev : n_max;
  uint32_t kk[kRItems], vv[kRItems], pp[kRItems];
  const uint32_t vmask = radix_load_kv(keys, nullptr, nullptr, n, blockIdx.x, kk, vv, pp);
  radix_hist_store(kk, vmask, shift, mask, h, counts, nblocks);
}

constexpr int kRowItems = 16;  // counts per thread held in registers

// Blocks 0 .. kRadix-1: one digit each.  Each thread takes a run of up to
// kRowItems consecutive per-block counts, loaded before any arithmetic so the
// row costs one memory round trip (longer rows loop over 4096-count pieces).
// Block kRadix (launched with a tail only) reduces the per-block totals.
__global__ void __launch_bounds__(kRThreadsSort) radix_rowscan_kernel(const uint32_t* __restrict__ counts,
                                                                      uint32_t* __restrict__ offs,
                                                                      uint32_t* __restrict__ totals,
                                                                      int64_t nblocks, RowscanTail tail) {
  __shared__ uint32_t wsum[kRWaves];
  __shared__ unsigned long long wp[kRWaves];
  const int d = blockIdx.x, t = threadIdx.x;
  if (d == kRadix) {
    uint32_t sn = 0;
    unsigned long long sp = 0;
    for (int64_t b = t; b < tail.count; b += kRThreadsSort) {
      sn += tail.part_n[b];
      sp += tail.part_p[b];
    }
    for (int o = 32; o > 0; o >>= 1) {
      sn += __shfl_xor(sn, o, 64);
      sp += __shfl_xor(sp, o, 64);
    }
    if ((t & 63) == 0) { wsum[t >> 6] = sn; wp[t >> 6] = sp; }
    __syncthreads();
    if (t == 0) {
      sn = 0;
      sp = 0;
      for (int k = 0; k < kRWaves; k++) { sn += wsum[k]; sp += wp[k]; }
      tail.dev[0] = sn;
      *(unsigned long long*)(tail.dev + 2) = sp;
      volatile uint32_t* h = (volatile uint32_t*)tail.host;
      h[0] = sn;
      h[2] = (uint32_t)sp;
      h[3] = (uint32_t)(sp >> 32);
    }
    return;
  }
  const uint32_t* row = counts + (int64_t)d * nblocks;
  uint32_t* orow = offs + (int64_t)d * nblocks;
  uint32_t carry = 0;
  for (int64_t p0 = 0; p0 < nblocks; p0 += (int64_t)kRThreadsSort * kRowItems) {
    const int64_t len = nblocks - p0 < (int64_t)kRThreadsSort * kRowItems
                            ? nblocks - p0 : (int64_t)kRThreadsSort * kRowItems;
    const int q = (int)((len + kRThreadsSort - 1) / kRThreadsSort);  // counts per thread
    const int64_t b0 = p0 + (int64_t)t * q;
    uint32_t v[kRowItems], sum = 0;
#pragma unroll
    for (int i = 0; i < kRowItems; i++) {
      v[i] = (i < q && b0 + i < p0 + len) ? row[b0 + i] : 0u;
      sum += v[i];
    }
    uint32_t total;
    uint32_t run = carry + radix_block_scan(sum, wsum, &total);
#pragma unroll
    for (int i = 0; i < kRowItems; i++) {
      if (i < q && b0 + i < p0 + len) orow[b0 + i] = run;
      run += v[i];
    }
    carry += total;
    __syncthreads();  // wsum is reused by the next piece
  }
  if (t == 0) totals[d] = carry;
}

template <bool PAY>
__global__ void __launch_bounds__(kRThreadsSort) radix_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, const uint32_t* __restrict__ pin,
    int64_t n_max, const uint32_t* n_dev, KVSink sink, int shift, int nbits,
    const uint32_t* __restrict__ offs, const uint32_t* __restrict__ totals, int64_t nblocks) {
  __shared__ RadixRankSmem S;
  __shared__ uint32_t sk[kRChunk];
  const int64_t n = n_dev ? (int64_t)*n_dev : n_max;
  const int64_t chunk = radix_xcd_chunk((n + kRChunk - 1) / kRChunk);
  if (chunk < 0) return;  // past the count: nothing to place
  uint32_t kk[kRItems], vv[kRItems], pp[kRItems];
  const uint32_t vmask = radix_load_kv(kin, vin, PAY ? pin : nullptr, n, chunk, kk, vv, pp);
  radix_scatter_chunk<PAY>(kk, vv, pp, vmask, shift, nbits, offs, totals, nblocks, chunk, sink, S, sk);
}

gut_status radix_hist(const uint32_t* keys, int64_t n_max, const uint32_t* n_dev, int shift,
                      uint32_t mask, uint32_t* counts, int64_t nblocks, hipStream_t st) {
  radix_hist_kernel<<<(unsigned)nblocks, kRThreadsSort, 0, st>>>(keys, n_max, n_dev, shift, mask, counts,
                                                                 nblocks);
  GUT_LAUNCH_CHECK();
  return GUT_OK;
}

gut_status radix_rowscan(const uint32_t* counts, uint32_t* offs, uint32_t* totals, int64_t nblocks,
                         hipStream_t st, const RowscanTail* tail) {
  RowscanTail tl = {};
  if (tail) tl = *tail;
  radix_rowscan_kernel<<<kRadix + (tail ? 1 : 0), kRThreadsSort, 0, st>>>(counts, offs, totals, nblocks,
                                                                          tl);
  GUT_LAUNCH_CHECK();
  return GUT_OK;
}

int64_t radix_blocks(int64_t n) { return ceil_div(n > 0 ? n : 1, kRChunk); }

size_t radix_temp_bytes(int64_t n) {
  int64_t nb = radix_blocks(n);
  size_t cnt = align256((size_t)kRadix * nb * sizeof(uint32_t));
  return 2 * cnt + align256(kRadix * sizeof(uint32_t));
}

RadixTemp radix_temp(void* temp, int64_t n_max) {
  const size_t cnt_bytes = align256((size_t)kRadix * radix_blocks(n_max) * sizeof(uint32_t));
  RadixTemp r;
  r.counts = (uint32_t*)temp;
  r.offs = (uint32_t*)((char*)temp + cnt_bytes);
  r.totals = (uint32_t*)((char*)temp + 2 * cnt_bytes);
  return r;
}

gut_status radix_sort_passes(uint32_t* kA, uint32_t* vA, uint32_t* kB, uint32_t* vB, int64_t n_max,
                             const uint32_t* n_dev, int bits, int pass0, int pass_end, void* temp,
                             hipStream_t st, int* result_in_b, uint2* ranges, uint32_t* pA,
                             uint32_t* pB) {
  *result_in_b = 0;
  if (n_max <= 0) return GUT_OK;
  const int passes = radix_passes(bits), per = radix_per_pass(bits);
  if (pass_end > passes) pass_end = passes;
  const int64_t nb = radix_blocks(n_max);
  const RadixTemp rt = radix_temp(temp, n_max);
  uint32_t *ks = kA, *vs = vA, *ps = pA;
  for (int p = pass0; p < pass_end; p++) {
    uint32_t* kd = ks == kA ? kB : kA;
    uint32_t* vd = ks == kA ? vB : vA;
    uint32_t* pd = ks == kA ? pB : pA;
    const int shift = p * per;
    const int nbits = bits - shift < per ? bits - shift : per;
    gut_status s = radix_hist(ks, n_max, n_dev, shift, (1u << nbits) - 1u, rt.counts, nb, st);
    if (s != GUT_OK) return s;
    if ((s = radix_rowscan(rt.counts, rt.offs, rt.totals, nb, st)) != GUT_OK) return s;
    // with ranges, the last pass keeps no keys: the ranges imply them
    const bool last_ranges = p == passes - 1 && ranges;
    const KVSink sink = {last_ranges ? nullptr : kd, vd, last_ranges ? ranges : nullptr, pd};
    if (pA)
      radix_scatter_kernel<true><<<(unsigned)nb, kRThreadsSort, 0, st>>>(
          ks, vs, ps, n_max, n_dev, sink, shift, nbits, rt.offs, rt.totals, nb);
    else
      radix_scatter_kernel<false><<<(unsigned)nb, kRThreadsSort, 0, st>>>(
          ks, vs, nullptr, n_max, n_dev, sink, shift, nbits, rt.offs, rt.totals, nb);
    GUT_LAUNCH_CHECK();
    ks = kd;
    vs = vd;
    ps = pd;
  }
  *result_in_b = ks == kB;
  return GUT_OK;
}

}  // namespace gut
