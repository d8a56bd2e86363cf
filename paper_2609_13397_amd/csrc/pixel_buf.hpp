// Per-pixel ray buffer.  The camera stage computes each pixel's PairPixel once (three
// FP64 inverse mappings Pi^{-1}, Sec. 3 and the half-edge rays of Sec. 4.1, one of them
// a Newton solve for the fisheye) and the forward and backward render kernels read it
// back instead of recomputing it.
//
// Slot layout follows the render's thread mapping: the pixel of thread q in tile t's
// workgroup sits at slot t * 256 + q, wave w = q / 64 covering the 8x8 quadrant
// (w % 2, w / 2) of the 16x16 tile and lane l the pixel (l % 8, l / 8) in it.  The 64
// bytes of a PairPixel are split over four planes of 16 bytes (plane k at float4
// offset k * n_slots), so each of a wave's four loads reads 1 KiB of contiguous memory.
// A pixel outside the crop or outside the camera's valid domain is stored as zeros:
// its float32 direction is then the zero vector, which a unit ray never is.
#pragma once

#include "pair_math.hpp"
#include "wave_ops.hpp"

namespace cg {

constexpr int kPixPlanes = 4;
static_assert(sizeof(PairPixel) == kPixPlanes * 16, "PairPixel is four 16-byte planes");

union PixelPlanes {
  PairPixel p;
  float4 q[kPixPlanes];
};

// Pixel (i, j) of the view handled by thread q of the workgroup of local tile lt.
__device__ __forceinline__ void tile_pixel(const DevCamera& c, int lt, int q, int& i, int& j) {
  const int tx = lt % c.tiles_x, ty = lt / c.tiles_x;
  const int w = q >> 6, l = q & 63;
  i = tx * kTile + (w & 1) * 8 + (l & 7);
  j = ty * kTile + (w >> 1) * 8 + (l >> 3);
}

__device__ __forceinline__ void store_pair_pixel(float4* __restrict__ buf, int64_t n_slots, int64_t slot,
                                                 const PairPixel& p) {
  PixelPlanes u;
  u.p = p;
#pragma unroll
  for (int k = 0; k < kPixPlanes; ++k) buf[k * n_slots + slot] = u.q[k];
}

__device__ __forceinline__ PairPixel load_pair_pixel(const float4* __restrict__ buf, int64_t n_slots, int64_t slot) {
  PixelPlanes u;
#pragma unroll
  for (int k = 0; k < kPixPlanes; ++k) u.q[k] = buf[k * n_slots + slot];
  return u.p;
}

__device__ __forceinline__ bool pixel_valid(const PairPixel& p) { return p.a0 != 0.f || p.a1 != 0.f || p.a2 != 0.f; }

// Wave-level view of a tile quadrant: its cone (axis = normalised mean of the
// quadrant's valid centre rays, chord radius = largest chord from the axis to one of
// them) lets a wave drop, 64 records at a time, every record whose influence cone
// cannot reach any of its pixels: |a - u| > lim + radius implies |d - u| > lim for
// every ray d of the quadrant.  Called with the whole wave active.
struct WaveCone {
  float ax, ay, az, rad;
  bool live;
};

__device__ __forceinline__ WaveCone wave_cone(const PairPixel& p, bool valid) {
  float sx = valid ? p.a0 : 0.f, sy = valid ? p.a1 : 0.f, sz = valid ? p.a2 : 0.f;
  float cnt = valid ? 1.f : 0.f;
  sx = wave_total(sx);
  sy = wave_total(sy);
  sz = wave_total(sz);
  cnt = wave_total(cnt);
  WaveCone w;
  w.live = cnt > 0.f;
  const float nrm = sqrtf(sx * sx + sy * sy + sz * sz);
  const float inv = nrm > 0.f ? 1.f / nrm : 0.f;
  w.ax = sx * inv;
  w.ay = sy * inv;
  w.az = sz * inv;
  float ch = 0.f;
  if (valid) {
    const float dx = w.ax - p.a0, dy = w.ay - p.a1, dz = w.az - p.a2;
    ch = sqrtf(dx * dx + dy * dy + dz * dz);
  }
  ch = wave_max(ch);
  w.rad = ch * 1.0001f + 2e-6f;
  if (nrm < 0.5f * cnt) w.rad = 3.f;  // rays spread too widely for a mean axis
  return w;
}

}  // namespace cg
