// Angular-cone tile binning.  A (tile, Gaussian) pair is emitted when the tile's cone
// of pixel-centre rays can overlap the Gaussian's influence cone; no projection is
// involved, so the same code serves every central camera.  Both cones are in chord
// form (axis, chord radius), tested by the triangle inequality of the chord distance
// (chords_overlap), which accepts every pair the exact angular test accepts.
//
// Layout of the work: a wavefront owns 64 Gaussians of one view.  Phase 1: each lane
// tests its Gaussian against every 8x8 tile group of the view (a loop that is uniform
// across the wave, reading the group cones through the scalar cache) and records the
// groups it overlaps.  Phase 2: the wave walks the lanes' hit groups together, one
// lane per member tile, reading the group-major member copy (one coalesced 1 KiB
// load per group, several groups ahead), so the 64 tile tests of a group run as one
// vector step and their ballot gives both the count and, in the emit pass, each
// pair's position.
#include "camera_dev.hpp"

namespace cg {

constexpr int kMaxGroupHits = kBinHitList;
constexpr int kPhase1Unroll = 8;
constexpr int kPhase2Depth = 2;

__device__ __forceinline__ float readlane_f(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ uint32_t readlane_u(uint32_t x, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}

template <bool EMIT>
__global__ __launch_bounds__(256) void k_bin(int64_t n, const DevCamera* __restrict__ cams,
                                             const float4* __restrict__ cone, const float4* __restrict__ groups,
                                             const float4* __restrict__ members, uint32_t* __restrict__ counts,
                                             const uint32_t* __restrict__ offsets,
                                             const uint32_t* __restrict__ slot_offs, uint32_t* __restrict__ keys,
                                             uint32_t* __restrict__ vals, uint32_t* __restrict__ slot_gid,
                                             uint8_t* __restrict__ hit_n, uint16_t* __restrict__ hit_list,
                                             uint2* __restrict__ clear_ranges, int64_t n_ranges, uint32_t cap) {
  __shared__ __align__(16) uint16_t hitbuf[4][64 * kMaxGroupHits];  // per wave: the lanes' hit groups
  __shared__ uint32_t flat[4][64 * kMaxGroupHits];
  const int v = blockIdx.y;
  const DevCamera& c = cams[v];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint16_t* __restrict__ hits = hitbuf[wave] + lane * kMaxGroupHits;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < n;
  const int64_t gv = (int64_t)v * n + i;
  const float4 cn = in ? cone[gv] : make_float4(0.f, 0.f, 1.f, kChordNever);
  const int ng = c.groups_x * c.groups_y;
  const float4* __restrict__ vgroups = groups + c.group_offset;
  const float4* __restrict__ vmem = members + (int64_t)c.group_offset * kGroupTiles + lane;
  const uint32_t my_base = (EMIT && in) ? offsets[gv] : 0u;
  const uint32_t my_slot = (EMIT && in && slot_gid) ? slot_offs[gv] : 0u;
  const float inv_gx = 1.f / (float)c.groups_x;
  uint32_t my_count = 0;
  if (EMIT) {  // the tile ranges that k_tile_ranges fills start at (0, 0): zeroed here
    const int64_t nthreads = (int64_t)gridDim.x * gridDim.y * blockDim.x;
    for (int64_t k = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x; k < n_ranges;
         k += nthreads)
      clear_ranges[k] = make_uint2(0u, 0u);
  }

  // phase 1: overlapping groups of this lane's Gaussian.  The count pass tests them and
  // keeps each Gaussian's list (up to kMaxGroupHits groups, ascending, and their number)
  // for the emit pass, which reads it back instead of testing again.
  int nh = 0;
  if (EMIT) {
    if (in) {
      nh = (int)hit_n[gv];
      const uint4* src = reinterpret_cast<const uint4*>(hit_list + gv * kMaxGroupHits);
      uint4* dst = reinterpret_cast<uint4*>(hits);
      dst[0] = src[0];
      dst[1] = src[1];
    }
  } else {
    if (__ballot(cn.w >= 0.f) != 0) {
      int gi = 0;
      for (; gi + kPhase1Unroll <= ng; gi += kPhase1Unroll) {
        float4 G[kPhase1Unroll];
#pragma unroll
        for (int u = 0; u < kPhase1Unroll; ++u) G[u] = vgroups[gi + u];
        bool h[kPhase1Unroll];
#pragma unroll
        for (int u = 0; u < kPhase1Unroll; ++u) h[u] = chords_overlap(G[u], cn.x, cn.y, cn.z, cn.w);
#pragma unroll
        for (int u = 0; u < kPhase1Unroll; ++u) {
          if (h[u]) {
            if (nh < kMaxGroupHits) hits[nh] = (uint16_t)(gi + u);
            ++nh;
          }
        }
      }
      for (; gi < ng; ++gi) {
        if (chords_overlap(vgroups[gi], cn.x, cn.y, cn.z, cn.w)) {
          if (nh < kMaxGroupHits) hits[nh] = (uint16_t)gi;
          ++nh;
        }
      }
    }
    if (in) {
      hit_n[gv] = (uint8_t)min(nh, 255);
      const uint4* src = reinterpret_cast<const uint4*>(hits);
      uint4* dst = reinterpret_cast<uint4*>(hit_list + gv * kMaxGroupHits);
      dst[0] = src[0];
      dst[1] = src[1];
    }
  }

  // phase 2: tile tests, one lane per member tile of a hit group.
  // One hit group of lane l's Gaussian: m holds the member tiles it overlaps.  Groups
  // of one lane come one after the other, in ascending order; cur, cnt and the cone /
  // base registers follow the lane being walked.
  int cur = -1;
  float cx = 0.f, cy = 0.f, cz = 0.f, cw = 0.f;
  uint32_t base = 0u, slot0 = 0u, cnt = 0u;
  auto take_lane = [&](int l) {
    if (l == cur) return;
    if (lane == cur) my_count = cnt;
    cur = l;
    cnt = 0u;
    cx = readlane_f(cn.x, l);
    cy = readlane_f(cn.y, l);
    cz = readlane_f(cn.z, l);
    cw = readlane_f(cn.w, l);
    if (EMIT) {
      base = readlane_u(my_base, l);
      if (slot_gid) slot0 = readlane_u(my_slot, l);
    }
  };
  auto group_hits = [&](int l, int gi, uint64_t m) {
    if (EMIT && ((m >> lane) & 1ull)) {
      const uint32_t j = cnt + (uint32_t)__popcll(m & __lanemask_lt());
      const uint32_t pos = base + j;
      // gi / groups_x in float32: exact for gi < 2^16 (the quotient is at least
      // 0.5 / groups_x from an integer, the rounding error below 2^16 * 2^-23 / groups_x)
      const int gy = (int)(((float)gi + 0.5f) * inv_gx), gx = gi - gy * c.groups_x;
      const int tx = gx * kGroup + (lane % kGroup), ty = gy * kGroup + lane / kGroup;
      const uint32_t gid = (uint32_t)(blockIdx.x * blockDim.x + (threadIdx.x & ~63) + l);
      // pairs at or past cap are dropped (buffers sized before the pair count was known
      // and found too small: the host emits again)
      if (pos < cap) {
        keys[pos] = (uint32_t)(c.tile_offset + ty * c.tiles_x + tx);
        vals[pos] = slot_gid ? slot0 + j : gid;
      }
      if (slot_gid && slot0 + j < cap) slot_gid[slot0 + j] = gid;
    }
    cnt += (uint32_t)__popcll(m);
  };

  // The wave's hit groups (lane by lane, each lane's in ascending group order) are
  // laid out as one list in LDS, and the member cones of the next kPhase2Depth entries
  // load while the current one is tested: the walk waits on one round trip per
  // kPhase2Depth groups, not per group.  Lanes with more than kMaxGroupHits groups are
  // walked afterwards.
  const uint64_t ovf = __ballot(nh > kMaxGroupHits);
  {
    // exclusive prefix of the listed counts over the wave (lanes below this one)
    const int listed = nh > kMaxGroupHits ? 0 : nh;
    int incl = listed;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    const int total = __builtin_amdgcn_readfirstlane(__shfl(incl, 63, 64));
    const int start = incl - listed;
    for (int h = 0; h < listed; ++h) flat[wave][start + h] = (uint32_t)(lane << 16) | hits[h];
    // the list is read by the whole wave below (LDS writes and reads of one wave are in order)
    __builtin_amdgcn_wave_barrier();
    float4 T[kPhase2Depth];
    uint32_t E[kPhase2Depth];  // list entries (lane << 16 | group)
    // entries past the end of the list repeat its last one (loaded, never tested), so
    // that every load is unconditional and each test waits for its own load only
    auto fetch = [&](int u, int f) {
      E[u] = (uint32_t)__builtin_amdgcn_readfirstlane((int)flat[wave][min(f, total - 1)]);
      T[u] = vmem[(int)(E[u] & 0xffffu) * kGroupTiles];
    };
    if (total > 0) {
#pragma unroll
      for (int u = 0; u < kPhase2Depth; ++u) fetch(u, u);
      for (int f0 = 0; f0 < total; f0 += kPhase2Depth) {
#pragma unroll
        for (int u = 0; u < kPhase2Depth; ++u) {
          const int f = f0 + u;
          const int l = (int)(E[u] >> 16);
          const bool live = f < total;
          if (live) take_lane(l);
          const uint64_t m = __ballot(live && chords_overlap(T[u], cx, cy, cz, cw));
          if (live) group_hits(l, (int)(E[u] & 0xffffu), m);
          fetch(u, f + kPhase2Depth);  // this slot's entry kPhase2Depth ahead
        }
      }
    }
  }
  // lanes whose hit groups overflowed the list: every group tested again, one lane at a time
  for (uint64_t om = ovf; om; om &= om - 1) {
    const int l = (int)__builtin_ctzll(om);
    take_lane(l);
    for (int gi = 0; gi < ng; ++gi) {
      if (!chords_overlap(vgroups[gi], cx, cy, cz, cw)) continue;
      group_hits(l, gi, __ballot(chords_overlap(vmem[gi * kGroupTiles], cx, cy, cz, cw)));
    }
  }
  if (lane == cur) my_count = cnt;
  if (!EMIT && in) counts[gv] = my_count;
}

hipError_t launch_bin_count(int64_t n, int n_views, const DevCamera* cams, const float4* cone, const float4* groups,
                            const float4* members, uint32_t* counts, uint8_t* hit_n, uint16_t* hit_list,
                            hipStream_t s) {
  if (n == 0 || n_views == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)n_views);
  k_bin<false><<<grid, dim3(256), 0, s>>>(n, cams, cone, groups, members, counts, nullptr, nullptr, nullptr, nullptr,
                                          nullptr, hit_n, hit_list, nullptr, 0, 0u);
  return hipGetLastError();
}

hipError_t launch_bin_emit(int64_t n, int n_views, const DevCamera* cams, const float4* cone, const float4* groups,
                           const float4* members, const uint32_t* offsets, const uint32_t* slot_offs,
                           uint32_t* keys, uint32_t* vals, uint32_t* slot_gid, uint8_t* hit_n,
                           uint16_t* hit_list, uint2* ranges, int64_t total_tiles, int64_t cap, hipStream_t s) {
  if (n == 0 || n_views == 0) return launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, 2 * total_tiles, s);
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)n_views);
  k_bin<true><<<grid, dim3(256), 0, s>>>(n, cams, cone, groups, members, nullptr, offsets, slot_offs, keys, vals,
                                         slot_gid, hit_n, hit_list, ranges, total_tiles,
                                         (uint32_t)std::min<int64_t>(cap, 0xffffffffll));
  return hipGetLastError();
}

// counts in compositing order, and their scanned offsets back in item order
__global__ void k_gather_u32(const uint32_t* __restrict__ src, const uint32_t* __restrict__ idx, int64_t m,
                             uint32_t* __restrict__ dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) dst[k] = src[idx[k]];
}

__global__ void k_scatter_u32(const uint32_t* __restrict__ src, const uint32_t* __restrict__ idx, int64_t m,
                              uint32_t* __restrict__ dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) dst[idx[k]] = src[k];
}

// dst[k] = src[idx[k]], and *total += sum of the gathered values in 64 bits (one
// atomic per workgroup).  The grid strides over m with at most kGatherBlocks groups.
constexpr int kGatherBlocks = 1024;

__global__ __launch_bounds__(256) void k_gather_total(const uint32_t* __restrict__ src,
                                                      const uint32_t* __restrict__ idx, int64_t m,
                                                      uint32_t* __restrict__ dst,
                                                      unsigned long long* __restrict__ total) {
  __shared__ unsigned long long wsum[4];
  unsigned long long acc = 0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < m; k += (int64_t)gridDim.x * 256) {
    const uint32_t v = src[idx[k]];
    dst[k] = v;
    acc += v;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(total, wsum[0] + wsum[1] + wsum[2] + wsum[3]);
}

hipError_t launch_gather_total(const uint32_t* src, const uint32_t* idx, int64_t m, uint32_t* dst,
                               unsigned long long* total, hipStream_t s) {
  if (m == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((m + 255) / 256, kGatherBlocks);
  k_gather_total<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(src, idx, m, dst, total);
  return hipGetLastError();
}

hipError_t launch_gather_u32(const uint32_t* src, const uint32_t* idx, int64_t m, uint32_t* dst, hipStream_t s) {
  if (m == 0) return hipSuccess;
  k_gather_u32<<<dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s>>>(src, idx, m, dst);
  return hipGetLastError();
}

hipError_t launch_scatter_u32(const uint32_t* src, const uint32_t* idx, int64_t m, uint32_t* dst, hipStream_t s) {
  if (m == 0) return hipSuccess;
  k_scatter_u32<<<dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s>>>(src, idx, m, dst);
  return hipGetLastError();
}

// Per-tile [start, end) ranges of the tile-sorted pair list.  `ranges` must be zeroed
// beforehand (empty tiles keep (0, 0)).
__global__ void k_tile_ranges(const uint32_t* __restrict__ keys, int64_t n, uint2* __restrict__ ranges) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t tile = keys[i];
  if (i == 0 || keys[i - 1] != tile) ranges[tile].x = (uint32_t)i;
  if (i == n - 1 || keys[i + 1] != tile) ranges[tile].y = (uint32_t)(i + 1);
}

hipError_t launch_tile_ranges(const uint32_t* keys, int64_t n, uint2* ranges, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_tile_ranges<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(keys, n, ranges);
  return hipGetLastError();
}

// Heaviest-first tile order for the render launches: tiles bucketed by the bit length
// of their pair count, buckets taken from the largest down, so the long tiles start
// first and the short ones fill the end of the launch.  One workgroup.  The order
// within a bucket follows the LDS atomics; it changes no result, since tiles are
// rendered independently.
constexpr int kOrderBuckets = 33;

__global__ __launch_bounds__(1024) void k_tile_order(const uint2* __restrict__ ranges, int total_tiles,
                                                     uint32_t* __restrict__ order) {
  __shared__ uint32_t cnt[kOrderBuckets];
  if (threadIdx.x < kOrderBuckets) cnt[threadIdx.x] = 0u;
  __syncthreads();
  for (int t = threadIdx.x; t < total_tiles; t += blockDim.x) {
    const uint2 r = ranges[t];
    atomicAdd(&cnt[32 - __clz(r.y - r.x)], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int k = kOrderBuckets - 1; k >= 0; --k) {
      const uint32_t c = cnt[k];
      cnt[k] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < total_tiles; t += blockDim.x) {
    const uint2 r = ranges[t];
    order[atomicAdd(&cnt[32 - __clz(r.y - r.x)], 1u)] = (uint32_t)t;
  }
}

hipError_t launch_tile_order(const uint2* ranges, int total_tiles, uint32_t* order, hipStream_t s) {
  if (total_tiles == 0) return hipSuccess;
  k_tile_order<<<dim3(1), dim3(1024), 0, s>>>(ranges, total_tiles, order);
  return hipGetLastError();
}

// One workgroup per view: the longest of its tile lists and its pair count, for views
// with fewer than max_tiles tiles (the ones the split tile render may take).
__global__ __launch_bounds__(256) void k_view_stats(const DevCamera* __restrict__ cams, const uint2* __restrict__ ranges,
                                                    int64_t max_tiles, uint32_t* __restrict__ stats) {
  __shared__ uint32_t s_long, s_pairs;
  const DevCamera& c = cams[blockIdx.x];
  const int tiles = c.tiles_x * c.tiles_y;
  if (threadIdx.x == 0) {
    s_long = 0u;
    s_pairs = 0u;
  }
  __syncthreads();
  if (tiles < max_tiles) {
    uint32_t lng = 0u, sum = 0u;
    for (int k = threadIdx.x; k < tiles; k += blockDim.x) {
      const uint2 r = ranges[c.tile_offset + k];
      lng = max(lng, r.y - r.x);
      sum += r.y - r.x;
    }
    atomicMax(&s_long, lng);
    atomicAdd(&s_pairs, sum);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    stats[2 * blockIdx.x] = s_long;
    stats[2 * blockIdx.x + 1] = s_pairs;
  }
}

hipError_t launch_view_stats(const DevCamera* cams, int n_views, const uint2* ranges, int64_t max_tiles,
                             uint32_t* stats, hipStream_t s) {
  k_view_stats<<<dim3((unsigned)n_views), dim3(256), 0, s>>>(cams, ranges, max_tiles, stats);
  return hipGetLastError();
}

}  // namespace cg
