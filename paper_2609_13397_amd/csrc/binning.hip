// Angular-cone tile binning.  A (tile, Gaussian) pair is emitted when the tile's cone
// of pixel-centre rays overlaps the Gaussian's influence cone; no projection is
// involved, so the same test serves every central camera.
//
// Layout of the work: a wavefront owns 64 Gaussians of one view.  Phase 1: each lane
// tests its Gaussian against every 8x8 tile group of the view (a loop that is uniform
// across the wave, reading the group cones through the scalar cache) and records the
// groups it overlaps.  Phase 2: the wave walks the lanes' hit groups together, one
// lane per tile of the group, so the 64 tile tests of a group run as one vector step
// and their ballot gives both the count and, in the emit pass, each pair's position.
#include "camera_dev.hpp"

namespace cg {

constexpr int kMaxGroupHits = 16;

__device__ __forceinline__ float readlane_f(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ uint32_t readlane_u(uint32_t x, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}

template <bool EMIT>
__global__ __launch_bounds__(256) void k_bin(int64_t n, const DevCamera* __restrict__ cams,
                                             const float4* __restrict__ cone, const TileCone* __restrict__ tiles,
                                             const TileCone* __restrict__ groups, uint32_t* __restrict__ counts,
                                             const uint32_t* __restrict__ offsets,
                                             const uint32_t* __restrict__ depth_key, uint64_t* __restrict__ keys,
                                             uint32_t* __restrict__ slots, uint32_t* __restrict__ slot_gid) {
  __shared__ uint16_t hits[4][64][kMaxGroupHits];
  const int v = blockIdx.y;
  const DevCamera& c = cams[v];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < n;
  const int64_t gv = (int64_t)v * n + i;
  const float4 cn = in ? cone[gv] : make_float4(0.f, 0.f, 1.f, -1.f);
  const float sg = sinf(0.5f * cn.w), cg = cosf(0.5f * cn.w);
  const int ng = c.groups_x * c.groups_y;

  // phase 1: overlapping groups of this lane's Gaussian
  int nh = 0;
  if (__ballot(cn.w >= 0.f) != 0) {
    for (int gi = 0; gi < ng; ++gi) {
      const TileCone G = groups[c.group_offset + gi];
      if (cones_overlap(G.ax, G.ay, G.az, G.beta, G.sb, G.cb, cn.x, cn.y, cn.z, cn.w, sg, cg)) {
        if (nh < kMaxGroupHits) hits[wave][lane][nh] = (uint16_t)gi;
        ++nh;
      }
    }
  }

  // phase 2: tile tests, one lane per tile of a hit group
  uint32_t my_count = 0;
  const uint32_t my_base = (EMIT && in) ? offsets[gv] : 0u;
  const uint32_t my_depth = (EMIT && in) ? depth_key[gv] : 0u;
  const int tl_x = lane % kGroup, tl_y = lane / kGroup;
  for (int l = 0; l < 64; ++l) {
    const int nh_l = __builtin_amdgcn_readlane(nh, l);
    if (nh_l == 0) continue;
    const float cx = readlane_f(cn.x, l), cy = readlane_f(cn.y, l), cz = readlane_f(cn.z, l);
    const float cw = readlane_f(cn.w, l), csg = readlane_f(sg, l), ccg = readlane_f(cg, l);
    const uint32_t base = EMIT ? readlane_u(my_base, l) : 0u;
    const uint32_t depth = EMIT ? readlane_u(my_depth, l) : 0u;
    const bool ovf = nh_l > kMaxGroupHits;
    const int n_iter = ovf ? ng : nh_l;
    uint32_t cnt = 0;
    for (int h = 0; h < n_iter; ++h) {
      const int gi = ovf ? h : (int)hits[wave][l][h];
      if (ovf) {
        const TileCone G = groups[c.group_offset + gi];
        if (!cones_overlap(G.ax, G.ay, G.az, G.beta, G.sb, G.cb, cx, cy, cz, cw, csg, ccg)) continue;
      }
      const int gx = gi % c.groups_x, gy = gi / c.groups_x;
      const int tx = gx * kGroup + tl_x, ty = gy * kGroup + tl_y;
      bool hit = false;
      int tile = 0;
      if (tx < c.tiles_x && ty < c.tiles_y) {
        tile = c.tile_offset + ty * c.tiles_x + tx;
        const TileCone T = tiles[tile];
        hit = cones_overlap(T.ax, T.ay, T.az, T.beta, T.sb, T.cb, cx, cy, cz, cw, csg, ccg);
      }
      const uint64_t m = __ballot(hit);
      if (EMIT && hit) {
        const uint32_t pos = base + cnt + (uint32_t)__popcll(m & __lanemask_lt());
        keys[pos] = ((uint64_t)(uint32_t)tile << 31) | (uint64_t)depth;
        slots[pos] = pos;
        slot_gid[pos] = (uint32_t)(blockIdx.x * blockDim.x + (threadIdx.x & ~63) + l);
      }
      cnt += (uint32_t)__popcll(m);
    }
    if (lane == l) my_count = cnt;
  }
  if (!EMIT && in) counts[gv] = my_count;
}

hipError_t launch_bin_count(int64_t n, int n_views, const DevCamera* cams, const float4* cone,
                            const TileCone* tiles, const TileCone* groups, uint32_t* counts, hipStream_t s) {
  if (n == 0 || n_views == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)n_views);
  k_bin<false><<<grid, dim3(256), 0, s>>>(n, cams, cone, tiles, groups, counts, nullptr, nullptr, nullptr, nullptr,
                                          nullptr);
  return hipGetLastError();
}

hipError_t launch_bin_emit(int64_t n, int n_views, const DevCamera* cams, const float4* cone, const TileCone* tiles,
                           const TileCone* groups, const uint32_t* offsets, const uint32_t* depth_key,
                           uint64_t* keys, uint32_t* slots, uint32_t* slot_gid, hipStream_t s) {
  if (n == 0 || n_views == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)n_views);
  k_bin<true><<<grid, dim3(256), 0, s>>>(n, cams, cone, tiles, groups, nullptr, offsets, depth_key, keys, slots,
                                         slot_gid);
  return hipGetLastError();
}

// Per-tile [start, end) ranges of the sorted pair list, and the Gaussian index of each
// sorted pair.  `ranges` must be zeroed beforehand (empty tiles keep (0, 0)).
__global__ void k_tile_ranges(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ slots,
                              const uint32_t* __restrict__ slot_gid, int64_t n, int shift, uint2* __restrict__ ranges,
                              uint32_t* __restrict__ sorted_gid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t tile = (uint32_t)(keys[i] >> shift);
  sorted_gid[i] = slot_gid[slots[i]];
  if (i == 0 || (uint32_t)(keys[i - 1] >> shift) != tile) ranges[tile].x = (uint32_t)i;
  if (i == n - 1 || (uint32_t)(keys[i + 1] >> shift) != tile) ranges[tile].y = (uint32_t)(i + 1);
}

hipError_t launch_tile_ranges(const uint64_t* keys, const uint32_t* slots, const uint32_t* slot_gid, int64_t n,
                              int key_shift, uint2* ranges, uint32_t* sorted_gid, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_tile_ranges<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(keys, slots, slot_gid, n, key_shift, ranges,
                                                                         sorted_gid);
  return hipGetLastError();
}

}  // namespace cg
