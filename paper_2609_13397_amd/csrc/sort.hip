// Device exclusive scan (uint32) and stable LSD radix sort of (uint32 key, uint32
// value) pairs, 8 bits per pass.
//
// Radix pass = histogram kernel (per-block digit counts, LDS atomics) + row scan (one
// workgroup per digit: the exclusive prefix of the digit's counts over the blocks, and
// the digit's total) + scatter kernel, which adds the exclusive prefix of the 256 digit
// totals that it forms itself: three launches per pass.  The scatter is stable: each
// wavefront owns a contiguous run of 1024 items, walks it in rounds of 64, and ranks
// items of equal digit with 8 ballots (a wave-wide digit match); per-wave digit
// counters in LDS carry the running offsets between rounds and are prefixed across
// the block's four wavefronts before the writes.
#include "cg_common.hpp"

namespace cg {

// ------------------------------------------------------------------------------ scan

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;  // 2048

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

// Exclusive scan of one 2048-item tile per block; block totals to `partials`.
__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                           int64_t n, uint32_t* __restrict__ partials) {
  __shared__ uint32_t wsum[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t local = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    local += v[k];
  }
  const uint32_t incl = wave_incl_scan(local);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t woff = 0;
  for (int k = 0; k < w; ++k) woff += wsum[k];
  uint32_t run = woff + incl - local;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kScanBlock - 1 && partials) partials[blockIdx.x] = woff + incl;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_add(uint32_t* __restrict__ out, int64_t n,
                                                         const uint32_t* __restrict__ partials) {
  const uint32_t add = partials[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) out[base + k] += add;
}

// Two-launch scan for up to kScanTile tiles (reduce, then scan): the first launch sums
// each tile, the second has every block add the sums of the tiles before its own (at
// most kScanTile of them, eight per thread) to its tile's local scan.
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                            uint32_t* __restrict__ partials) {
  __shared__ uint32_t wsum[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t local = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) local += (base + k < n) ? in[base + k] : 0u;
  for (int o = 32; o > 0; o >>= 1) local += __shfl_xor(local, o);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ __launch_bounds__(kScanBlock) void k_scan_final(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                           int64_t n, const uint32_t* __restrict__ partials) {
  __shared__ uint32_t wsum[4], psum[4];
  // the sum of the tiles before this one
  uint32_t before = 0;
  for (int t = (int)threadIdx.x; t < (int)blockIdx.x; t += kScanBlock) before += partials[t];
  for (int o = 32; o > 0; o >>= 1) before += __shfl_xor(before, o);
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t local = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    local += v[k];
  }
  const uint32_t incl = wave_incl_scan(local);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) wsum[w] = incl;
  if ((threadIdx.x & 63) == 0) psum[w] = before;
  __syncthreads();
  uint32_t run = psum[0] + psum[1] + psum[2] + psum[3] + incl - local;
  for (int k = 0; k < w; ++k) run += wsum[k];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
}

// The same two launches for a scan in a permuted order, scattered back: the first
// gathers vals[perm[k]] (kept in vals_perm), sums each tile and adds the tile's sum to
// *total (64 bits); the second scans vals_perm and writes each prefix to out[perm[k]].
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce_perm(const uint32_t* __restrict__ vals,
                                                                 const uint32_t* __restrict__ perm, int64_t n,
                                                                 uint32_t* __restrict__ vals_perm,
                                                                 uint32_t* __restrict__ partials,
                                                                 unsigned long long* __restrict__ total) {
  __shared__ unsigned long long wsum[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < n) ? vals[perm[base + k]] : 0u;
  unsigned long long local = 0;  // the exact total in 64 bits: 32-bit sums may wrap
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) vals_perm[base + k] = v[k];
    local += v[k];
  }
  for (int o = 32; o > 0; o >>= 1) local += __shfl_xor(local, o);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    partials[blockIdx.x] = (uint32_t)t;  // wraps only where the 64-bit total rejects the call
    atomicAdd(total, t);
  }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_final_perm(const uint32_t* __restrict__ vals_perm,
                                                                const uint32_t* __restrict__ perm, int64_t n,
                                                                const uint32_t* __restrict__ partials,
                                                                uint32_t* __restrict__ out) {
  __shared__ uint32_t wsum[4], psum[4];
  uint32_t before = 0;
  for (int t = (int)threadIdx.x; t < (int)blockIdx.x; t += kScanBlock) before += partials[t];
  for (int o = 32; o > 0; o >>= 1) before += __shfl_xor(before, o);
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t local = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? vals_perm[base + k] : 0u;
    local += v[k];
  }
  const uint32_t incl = wave_incl_scan(local);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) wsum[w] = incl;
  if ((threadIdx.x & 63) == 0) psum[w] = before;
  __syncthreads();
  uint32_t run = psum[0] + psum[1] + psum[2] + psum[3] + incl - local;
  for (int k = 0; k < w; ++k) run += wsum[k];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[perm[base + k]] = run;
    run += v[k];
  }
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

size_t scan_temp_bytes(int64_t n) {
  size_t total = 0;
  int64_t m = n;
  while (m > kScanTile) {
    m = ceil_div(m, kScanTile);
    total += (size_t)m * sizeof(uint32_t) * 2;
  }
  return total + 256;
}

static hipError_t scan_rec(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* temp, hipStream_t s) {
  const int64_t blocks = ceil_div(n, kScanTile);
  if (blocks <= 1) {
    k_scan_tiles<<<dim3(1), dim3(kScanBlock), 0, s>>>(in, out, n, nullptr);
    return hipGetLastError();
  }
  uint32_t* part = temp;
  uint32_t* part_scan = temp + blocks;
  k_scan_tiles<<<dim3((unsigned)blocks), dim3(kScanBlock), 0, s>>>(in, out, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_rec(part, part_scan, blocks, temp + 2 * blocks, s);
  if (e != hipSuccess) return e;
  k_scan_add<<<dim3((unsigned)blocks), dim3(kScanBlock), 0, s>>>(out, n, part_scan);
  return hipGetLastError();
}

hipError_t launch_permuted_scan(const uint32_t* vals, const uint32_t* perm, int64_t n, uint32_t* vals_perm,
                                uint32_t* vals_perm_scan, uint32_t* out, unsigned long long* total, void* temp,
                                hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = ceil_div(n, kScanTile);
  if (blocks <= kScanTile) {
    uint32_t* part = static_cast<uint32_t*>(temp);
    k_scan_reduce_perm<<<dim3((unsigned)blocks), dim3(kScanBlock), 0, s>>>(vals, perm, n, vals_perm, part, total);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_scan_final_perm<<<dim3((unsigned)blocks), dim3(kScanBlock), 0, s>>>(vals_perm, perm, n, part, out);
    return hipGetLastError();
  }
  hipError_t e = launch_gather_total(vals, perm, n, vals_perm, total, s);
  if (e != hipSuccess) return e;
  e = launch_exclusive_scan(vals_perm, vals_perm_scan, n, temp, s);
  if (e != hipSuccess) return e;
  return launch_scatter_u32(vals_perm_scan, perm, n, out, s);
}

hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, void* temp, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = ceil_div(n, kScanTile);
  if (blocks > 1 && blocks <= kScanTile) {  // reduce, then scan: two launches
    uint32_t* part = static_cast<uint32_t*>(temp);
    k_scan_reduce<<<dim3((unsigned)blocks), dim3(kScanBlock), 0, s>>>(in, n, part);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_scan_final<<<dim3((unsigned)blocks), dim3(kScanBlock), 0, s>>>(in, out, n, part);
    return hipGetLastError();
  }
  return scan_rec(in, out, n, static_cast<uint32_t*>(temp), s);
}

// ------------------------------------------------------------------------------ radix sort

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortBlock = 256;
constexpr int kSortRounds = 16;                                 // rounds of 64 items per wave
constexpr int kSortTile = kSortBlock * kSortRounds;             // 4096 items per block
constexpr int kWaveItems = 64 * kSortRounds;                    // 1024 items per wave

template <class K>
__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const K* __restrict__ keys, int64_t n, int shift, uint32_t dmask,
                                                           uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint32_t cnt[kRadix];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int k = 0; k < kSortRounds; ++k) {
    const int64_t idx = base + (int64_t)k * kSortBlock + threadIdx.x;
    if (idx < n) atomicAdd(&cnt[(uint32_t)(keys[idx] >> shift) & dmask], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// One workgroup per digit d: hist[d * nblocks + b] becomes the exclusive prefix of the
// digit's counts over blocks b' < b (in place), and totals[d] the digit's count.
__global__ __launch_bounds__(kScanBlock) void k_radix_rowscan(uint32_t* __restrict__ hist, int nblocks,
                                                              uint32_t* __restrict__ totals) {
  __shared__ uint32_t wsum[4];
  uint32_t* __restrict__ row = hist + (int64_t)blockIdx.x * nblocks;
  const int w = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (int base = 0; base < nblocks; base += kScanTile) {
    const int b0 = base + (int)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t local = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      v[k] = b0 + k < nblocks ? row[b0 + k] : 0u;
      local += v[k];
    }
    const uint32_t incl = wave_incl_scan(local);
    if ((threadIdx.x & 63) == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t woff = 0, tile = 0;
    for (int k = 0; k < 4; ++k) {
      woff += k < w ? wsum[k] : 0u;
      tile += wsum[k];
    }
    uint32_t run = carry + woff + incl - local;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (b0 + k < nblocks) row[b0 + k] = run;
      run += v[k];
    }
    carry += tile;
    __syncthreads();  // wsum is rewritten by the next tile
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Scatter of one pass.  The block first ranks its 4096 items by digit (stable) into
// LDS, in digit order, then writes them out linearly: consecutive threads write
// consecutive positions of a digit's run, so the global writes come in contiguous
// runs (about 16 items per digit per block) instead of isolated 4-byte stores.
template <class K>
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(const K* __restrict__ kin,
                                                              const uint32_t* __restrict__ vin,
                                                              K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                              int64_t n, int shift, uint32_t dmask,
                                                              const uint32_t* __restrict__ offsets,
                                                              const uint32_t* __restrict__ totals, int nblocks) {
  __shared__ uint32_t wcnt[4][kRadix];
  __shared__ int64_t gdelta[kRadix];  // global position of a digit's run minus its LDS start
  __shared__ uint32_t wsum[4], tsum[4];
  __shared__ K skey[kSortTile];
  __shared__ uint32_t sval[kSortTile];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int w = 0; w < 4; ++w) wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  const int64_t bbase = (int64_t)blockIdx.x * kSortTile;
  const int64_t wbase = bbase + (int64_t)wave * kWaveItems;
  const uint64_t lt = __lanemask_lt();
  K key[kSortRounds];
  uint32_t val[kSortRounds];
  uint32_t rank[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t idx = wbase + (int64_t)r * 64 + lane;
    const bool ok = idx < n;
    key[r] = ok ? kin[idx] : K(0);
    val[r] = ok ? vin[idx] : 0u;
    const uint32_t d = (uint32_t)(key[r] >> shift) & dmask;
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t before = (uint32_t)__popcll(peers & lt);
    uint32_t base = 0;
    if (ok) base = wcnt[wave][d];
    if (ok && before == 0) wcnt[wave][d] = base + (uint32_t)__popcll(peers);
    rank[r] = ok ? base + before : 0xffffffffu;
  }
  __syncthreads();
  {  // per digit: exclusive prefix over the block's waves, then over the digits; the
     // digit's global start is the exclusive prefix of the digit totals plus the counts
     // of the digit in the blocks before this one (the row scan)
    const int d = threadIdx.x;
    uint32_t run = 0;
    for (int w = 0; w < 4; ++w) {
      const uint32_t t = wcnt[w][d];
      wcnt[w][d] = run;
      run += t;
    }
    const uint32_t tot = totals[d];
    const uint32_t incl = wave_incl_scan(run);
    const uint32_t tincl = wave_incl_scan(tot);
    if (lane == 63) {
      wsum[wave] = incl;
      tsum[wave] = tincl;
    }
    __syncthreads();
    uint32_t start = incl - run, dstart = tincl - tot;
    for (int w = 0; w < wave; ++w) {
      start += wsum[w];
      dstart += tsum[w];
    }
    for (int w = 0; w < 4; ++w) wcnt[w][d] += start;
    gdelta[d] = (int64_t)dstart + (int64_t)offsets[(int64_t)d * nblocks + blockIdx.x] - (int64_t)start;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    if (rank[r] == 0xffffffffu) continue;
    const uint32_t d = (uint32_t)(key[r] >> shift) & dmask;
    const uint32_t lpos = wcnt[wave][d] + rank[r];
    skey[lpos] = key[r];
    sval[lpos] = val[r];
  }
  __syncthreads();
  const int cnt = (int)min((int64_t)kSortTile, n - bbase);
  for (int i = threadIdx.x; i < cnt; i += kSortBlock) {
    const K k = skey[i];
    const uint32_t d = (uint32_t)(k >> shift) & dmask;
    const int64_t pos = gdelta[d] + i;
    kout[pos] = k;
    vout[pos] = sval[i];
  }
}

size_t radix_temp_bytes(int64_t n) {
  const int64_t nblocks = ceil_div(n > 0 ? n : 1, kSortTile);
  const int64_t m = nblocks * kRadix;
  return (size_t)(m + kRadix) * sizeof(uint32_t) + 256;
}

template <class K>
static hipError_t radix_sort_t(K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt, int64_t n, int end_bit,
                               void* temp, int* result_in_alt, hipStream_t s) {
  *result_in_alt = 0;
  if (n <= 1) return hipSuccess;
  const int nblocks = (int)ceil_div(n, kSortTile);
  const int64_t m = (int64_t)nblocks * kRadix;
  uint32_t* hist = static_cast<uint32_t*>(temp);  // becomes the row-scanned offsets
  uint32_t* totals = hist + m;
  K* kin = keys;
  uint32_t* vin = vals;
  K* kout = keys_alt;
  uint32_t* vout = vals_alt;
  int alt = 0;
  for (int shift = 0; shift < end_bit; shift += kRadixBits) {
    // the last pass's digit stops at end_bit: bits above it may hold other data
    const uint32_t dmask = end_bit - shift >= kRadixBits ? (uint32_t)(kRadix - 1) : (1u << (end_bit - shift)) - 1u;
    k_radix_hist<K><<<dim3(nblocks), dim3(kSortBlock), 0, s>>>(kin, n, shift, dmask, hist, nblocks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_radix_rowscan<<<dim3(kRadix), dim3(kScanBlock), 0, s>>>(hist, nblocks, totals);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_radix_scatter<K><<<dim3(nblocks), dim3(kSortBlock), 0, s>>>(kin, vin, kout, vout, n, shift, dmask, hist, totals,
                                                                    nblocks);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    K* tk = kin; kin = kout; kout = tk;
    uint32_t* tv = vin; vin = vout; vout = tv;
    alt ^= 1;
  }
  *result_in_alt = alt;
  return hipSuccess;
}

hipError_t launch_radix_sort32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, int64_t n,
                               int end_bit, void* temp, int* result_in_alt, hipStream_t s) {
  return radix_sort_t<uint32_t>(keys, vals, keys_alt, vals_alt, n, end_bit, temp, result_in_alt, s);
}

}  // namespace cg
