// Conservative tests of a render record against a cone of ray directions, shared by
// the binning (a tile's cone) and the render (a wave's cone).
#pragma once

#include "cg_common.hpp"

namespace cg {

// Tangent-cone test bounded over the cone |d - a| <= rad (a unit, rad a chord length):
// with n = v x d, |n|_S >= |v x a|_S - sqrt(lambda_max(S)) |v| rad, where S is a
// multiple of R diag(s'^2) R^T, so lambda_max(S) = tr S max(s'^2) / sum(s'^2); and
// |W d| <= |W a| + rad / s'_min.  False means no ray of the cone passes the per-pixel
// test n^T S n <= |W d|^2 (and so none passes the pre-rejection it bounds).
__device__ __forceinline__ bool tangent_cone_reaches(const Record& R, float ax, float ay, float az, float rad) {
  if (rad >= 2.f) return true;
  const float vv = R.vx * R.vx + R.vy * R.vy + R.vz * R.vz;
  const float nx = R.vy * az - R.vz * ay, ny = R.vz * ax - R.vx * az, nz = R.vx * ay - R.vy * ax;
  const float* S = R.S;
  const float nsn = nx * (S[0] * nx + S[1] * ny + S[2] * nz) + ny * (S[3] * ny + S[4] * nz) + S[5] * nz * nz;
  const float* W = R.W;
  const float wx = W[0] * ax + W[1] * ay + W[2] * az;
  const float wy = W[3] * ax + W[4] * ay + W[5] * az;
  const float wz = W[6] * ax + W[7] * ay + W[8] * az;
  const float smax = fmaxf(R.sp2[0], fmaxf(R.sp2[1], R.sp2[2]));
  const float lmax = (S[0] + S[3] + S[5]) * smax * fast_rcp(R.sp2[0] + R.sp2[1] + R.sp2[2]) * 1.0001f;
  const float lo = fast_sqrt(fmaxf(nsn, 0.f)) * 0.9999f - fast_sqrt(lmax) * fast_sqrt(vv) * rad;
  const float hi = fast_sqrt(wx * wx + wy * wy + wz * wz) * 1.0001f + fast_sqrt(R.kg) * rad * 1.0001f;
  return lo <= hi;
}

// Whether R can pass pair_cheap for some ray of a wave's cone |d - a| <= rad: the chord
// test of its influence cone, then the tangent-cone bound.
__device__ __forceinline__ bool record_reaches_cone(const Record& R, float ax, float ay, float az, float rad) {
  if (R.lim < 0.f) return false;
  const float vv = R.vx * R.vx + R.vy * R.vy + R.vz * R.vz;
  const float iv = vv > 0.f ? rsqrtf(vv) : 0.f;  // v = 0 only for records seen in every direction
  const float dx = ax - R.vx * iv, dy = ay - R.vy * iv, dz = az - R.vz * iv;
  const float lim = R.lim + rad;
  if (dx * dx + dy * dy + dz * dz > lim * lim) return false;
  return tangent_cone_reaches(R, ax, ay, az, rad);
}

}  // namespace cg
