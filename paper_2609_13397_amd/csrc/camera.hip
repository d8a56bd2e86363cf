// Camera kernels: Pi^{-1} for a list of coordinates, and the per-tile / per-group
// ray cones used by the angular binning (camera-agnostic: only unit ray directions
// are compared, so the same code serves fields of view beyond 180 degrees).
#include "pixel_buf.hpp"

namespace cg {

__global__ void k_unproject(const DevCamera* cam, int64_t n, const float* __restrict__ pix_xy,
                            float* __restrict__ dirs, uint8_t* __restrict__ valid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d[3];
  const bool ok = cam_unproject(*cam, (double)pix_xy[i], (double)pix_xy[n + i], d);
  for (int k = 0; k < 3; ++k) dirs[k * n + i] = ok ? (float)d[k] : 0.f;
  valid[i] = ok ? 1 : 0;
}

hipError_t launch_unproject(const DevCamera* cam, int64_t n, const float* pix_xy, float* dirs, uint8_t* valid,
                            hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  k_unproject<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(cam, n, pix_xy, dirs, valid);
  return hipGetLastError();
}

// Block-wide maximum over 256 threads (4 waves) through LDS.
__device__ __forceinline__ float block_max(float v, float* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  const float r = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
  __syncthreads();
  return r;
}

// One workgroup per 16x16 tile: the cone around the tile's pixel-centre rays (axis =
// normalised mean direction, half-angle = largest angle to a pixel ray plus a small
// margin) and the tile's largest footprint coefficient (|d_x-d|^2 + |d_y-d|^2) / 3,
// whose per-view maximum (taken by k_group_cones) bounds every pixel's footprint in
// the Gaussian cones.  Each thread also stores its pixel's rays in the pixel buffer (pixel_buf.hpp), in the
// slot of the render thread that shades that pixel.  The first workgroup also zeroes
// the two small arrays of `clr` (accumulators of later kernels), which saves their
// fill launches.
__global__ __launch_bounds__(256) void k_tile_cones(const DevCamera* __restrict__ cams, int n_views, float fs,
                                                    int64_t n_slots, TileCone* __restrict__ tiles,
                                                    float4* __restrict__ pix, ClearPair clr) {
  __shared__ float sh[4];
  const int t = blockIdx.x;
  if (t == 0) {
    for (int k = threadIdx.x; k < clr.n[0]; k += blockDim.x) clr.p[0][k] = 0u;
    for (int k = threadIdx.x; k < clr.n[1]; k += blockDim.x) clr.p[1][k] = 0u;
  }
  const int v = view_of_tile(cams, n_views, t);
  const DevCamera& c = cams[v];
  int i, j;
  tile_pixel(c, t - c.tile_offset, threadIdx.x, i, j);
  PixelRay r;
  r.valid = false;
  if (i < c.crop_w && j < c.crop_h) r = pixel_ray(c, i, j, fs);
  PairPixel pp{};
  if (r.valid) pp = make_pair_pixel(r);
  store_pair_pixel(pix, n_slots, (int64_t)t * kTilePx + threadIdx.x, pp);
  // the tile's ray sums, valid-pixel count and largest footprint coefficient in one
  // reduction (one barrier instead of three per value)
  float v5[5] = {r.valid ? r.df[0] : 0.f, r.valid ? r.df[1] : 0.f, r.valid ? r.df[2] : 0.f, r.valid ? 1.f : 0.f,
                 r.valid ? r.cpix : 0.f};
  for (int o2 = 32; o2 > 0; o2 >>= 1) {
    for (int q = 0; q < 4; ++q) v5[q] += __shfl_xor(v5[q], o2);
    v5[4] = fmaxf(v5[4], __shfl_xor(v5[4], o2));
  }
  __shared__ float sh5[5][4];
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < 5; ++q) sh5[q][threadIdx.x >> 6] = v5[q];
  __syncthreads();
  const float sx = sh5[0][0] + sh5[0][1] + sh5[0][2] + sh5[0][3];
  const float sy = sh5[1][0] + sh5[1][1] + sh5[1][2] + sh5[1][3];
  const float sz = sh5[2][0] + sh5[2][1] + sh5[2][2] + sh5[2][3];
  const float cnt = sh5[3][0] + sh5[3][1] + sh5[3][2] + sh5[3][3];
  const float cm = fmaxf(fmaxf(sh5[4][0], sh5[4][1]), fmaxf(sh5[4][2], sh5[4][3]));
  TileCone tc;
  if (cnt == 0.f) {
    tc = TileCone{0.f, 0.f, 1.f, -1.f, 0.f, 1.f, 0.f, 0.f};
  } else {
    const float nrm = sqrtf(sx * sx + sy * sy + sz * sz);
    const float ax = sx / nrm, ay = sy / nrm, az = sz / nrm;
    float ang = 0.f;
    if (r.valid) {
      const float dx = ax - r.df[0], dy = ay - r.df[1], dz = az - r.df[2];
      ang = 2.f * asinf(fminf(1.f, 0.5f * sqrtf(dx * dx + dy * dy + dz * dz)));
    }
    float beta = block_max(ang, sh) * 1.0001f + 2e-6f;
    if (nrm < 0.5f * cnt) beta = kPiF;  // rays spread too widely for a mean axis
    tc = TileCone{ax, ay, az, beta, sinf(0.5f * beta), cosf(0.5f * beta), cm, 0.f};
  }
  if (threadIdx.x == 0) tiles[t] = tc;
}

hipError_t launch_tile_cones(const DevCamera* cams, int n_views, int total_tiles, float fs, TileCone* tiles,
                             float4* pix, const ClearPair& clr, hipStream_t s) {
  if (total_tiles == 0) {
    for (int k = 0; k < 2; ++k) {
      const hipError_t e = launch_fill_u32(clr.p[k], 0u, clr.n[k], s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  k_tile_cones<<<dim3(total_tiles), dim3(kTilePx), 0, s>>>(cams, n_views, fs, (int64_t)total_tiles * kTilePx, tiles,
                                                          pix, clr);
  return hipGetLastError();
}

// One wave per 8x8 group of tiles: a cone containing every member tile's cone, the
// group-major copy of the member tiles' chord cones and tile indices that the binning
// reads one group at a time, and the group's share of the per-view maximum footprint
// coefficient (one atomic per group: same-address atomics from every tile would
// contend across the XCDs).
__global__ __launch_bounds__(64) void k_group_cones(const DevCamera* __restrict__ cams, int n_views,
                                                   const TileCone* __restrict__ tiles, float4* __restrict__ groups,
                                                   float4* __restrict__ members, float* __restrict__ view_cmax) {
  const int g = blockIdx.x;
  const int v = view_of_group(cams, n_views, g);
  const DevCamera& c = cams[v];
  const int lg = g - c.group_offset;
  const int gx = lg % c.groups_x, gy = lg / c.groups_x;
  const int tx = gx * kGroup + (threadIdx.x % kGroup), ty = gy * kGroup + (threadIdx.x / kGroup);
  TileCone tc{0.f, 0.f, 1.f, -1.f, 0.f, 1.f, 0.f, 0.f};
  if (tx < c.tiles_x && ty < c.tiles_y) tc = tiles[c.tile_offset + ty * c.tiles_x + tx];
  const bool live = tc.beta >= 0.f;
  members[(int64_t)g * kGroupTiles + threadIdx.x] = make_float4(tc.ax, tc.ay, tc.az, chord_radius(tc.beta));
  float sx = live ? tc.ax : 0.f, sy = live ? tc.ay : 0.f, sz = live ? tc.az : 0.f, cnt = live ? 1.f : 0.f;
  float bmax = live ? tc.beta : -1.f, cm = live ? tc.cmax : 0.f;
  for (int o = 32; o > 0; o >>= 1) {
    sx += __shfl_xor(sx, o);
    sy += __shfl_xor(sy, o);
    sz += __shfl_xor(sz, o);
    cnt += __shfl_xor(cnt, o);
    bmax = fmaxf(bmax, __shfl_xor(bmax, o));
    cm = fmaxf(cm, __shfl_xor(cm, o));
  }
  float4 out = make_float4(0.f, 0.f, 1.f, kChordNever);
  if (cnt > 0.f) {
    const float nrm = sqrtf(sx * sx + sy * sy + sz * sz);
    const float ax = sx / nrm, ay = sy / nrm, az = sz / nrm;
    float ang = -1.f;
    if (live) {
      const float dx = ax - tc.ax, dy = ay - tc.ay, dz = az - tc.az;
      ang = 2.f * asinf(fminf(1.f, 0.5f * sqrtf(dx * dx + dy * dy + dz * dz))) + tc.beta;
    }
    for (int o = 32; o > 0; o >>= 1) ang = fmaxf(ang, __shfl_xor(ang, o));
    float beta = ang * 1.0001f + 2e-6f;
    if (bmax >= kPiF || nrm < 0.5f * cnt) beta = kPiF;
    out = make_float4(ax, ay, az, chord_radius(beta));
  }
  if (threadIdx.x == 0) {
    groups[g] = out;
    // non-negative floats order like their bit patterns
    atomicMax(reinterpret_cast<unsigned int*>(&view_cmax[v]), __float_as_uint(cm));
  }
}

hipError_t launch_group_cones(const DevCamera* cams, int n_views, int total_groups, const TileCone* tiles,
                              float4* groups, float4* members, float* view_cmax,
                              hipStream_t s) {
  if (total_groups == 0) return hipSuccess;
  k_group_cones<<<dim3(total_groups), dim3(kGroupTiles), 0, s>>>(cams, n_views, tiles, groups, members,
                                                                view_cmax);
  return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_fill_u32<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(p, v, n);
  return hipGetLastError();
}

// Counts the words of g[0, n) that differ from v (guard bands after scratch buffers).
__global__ void k_guard_check(const uint32_t* g, int n, uint32_t v, uint32_t* bad) {
  uint32_t k = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) k += g[i] != v;
  if (k) atomicAdd(bad, k);
}

hipError_t launch_guard_check(const uint32_t* g, int n, uint32_t v, uint32_t* bad, hipStream_t s) {
  k_guard_check<<<dim3(1), dim3(64), 0, s>>>(g, n, v, bad);
  return hipGetLastError();
}

}  // namespace cg
