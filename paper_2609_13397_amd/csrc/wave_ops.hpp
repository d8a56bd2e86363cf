// Cross-lane sums on a 64-lane CDNA wave without LDS traffic.
//
// __shfl_xor lowers to ds_bpermute (an LDS-unit round trip per step); these use
// the VALU's own lane movers instead: v_permlane32_swap / v_permlane16_swap (gfx950)
// for lane bits 5 and 4, and DPP mirrors / quad permutes within a row for bits 3..0.
// Every function here must be called with the whole wave active.
#pragma once

#include <hip/hip_runtime.h>

namespace cg {

__device__ __forceinline__ float as_f(unsigned int u) { return __uint_as_float(u); }
__device__ __forceinline__ unsigned int as_u(float f) { return __float_as_uint(f); }

// Lane l < 32 returns a[l] + a[l + 32]; lane l >= 32 returns b[l - 32] + b[l].
__device__ __forceinline__ float swap_add32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(as_u(a), as_u(b), false, false);
  return as_f(r[0]) + as_f(r[1]);
}

// Within each 32-lane half: lanes of the lower 16 return a[l] + a[l + 16], lanes of
// the upper 16 return b[l - 16] + b[l].
__device__ __forceinline__ float swap_add16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(as_u(a), as_u(b), false, false);
  return as_f(r[0]) + as_f(r[1]);
}

// DPP controls: mirror within 16 lanes (l ^ 15), within 8 (l ^ 7), within 4 (l ^ 3),
// and swap of neighbours (l ^ 1).
constexpr int kDppMirror16 = 0x140, kDppMirror8 = 0x141, kDppMirror4 = 0x1b, kDppSwap1 = 0xb1;

template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
  return as_f(__builtin_amdgcn_update_dpp(0u, as_u(x), CTRL, 0xf, 0xf, false));
}

// One butterfly step across a DPP partner that has the opposite `hi`: each lane
// keeps one of (a, b) and adds the partner's copy of the same value.
template <int CTRL>
__device__ __forceinline__ float dpp_pair_add(float a, float b, bool hi) {
  const float keep = hi ? b : a, send = hi ? a : b;
  return keep + dpp_move<CTRL>(send);
}

// Plain sum over the wave, returned in every lane.
__device__ __forceinline__ float wave_total(float v) {
  v = swap_add32(v, v);
  v = swap_add16(v, v);
  v += dpp_move<kDppMirror16>(v);
  v += dpp_move<kDppMirror8>(v);
  v += dpp_move<kDppMirror4>(v);
  v += dpp_move<kDppSwap1>(v);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
  auto r = __builtin_amdgcn_permlane32_swap(as_u(v), as_u(v), false, false);
  v = fmaxf(as_f(r[0]), as_f(r[1]));
  r = __builtin_amdgcn_permlane16_swap(as_u(v), as_u(v), false, false);
  v = fmaxf(as_f(r[0]), as_f(r[1]));
  v = fmaxf(v, dpp_move<kDppMirror16>(v));
  v = fmaxf(v, dpp_move<kDppMirror8>(v));
  v = fmaxf(v, dpp_move<kDppMirror4>(v));
  v = fmaxf(v, dpp_move<kDppSwap1>(v));
  return v;
}

// Sums of 20 per-lane values over the wave, transposed: each step across a lane bit
// halves the number of values a lane carries (20 -> 10 -> 5 -> 3 -> 2 -> 1, odd counts
// padded with a zero), so the whole reduction costs 22 lane moves instead of 120.
// Lane l ends with the total of value wave_sum20_index(l), or of a padding slot when
// that index is negative; each of the 20 values ends in exactly one even lane.  Lanes
// with keep false add zeros (their v is not read), and v[19] is taken as zero: the
// selections feed the first swaps directly, so no lane needs to clear its values first.
__device__ __forceinline__ float wave_sum20(const float v[20], bool keep, int lane) {
  float w[10], u[5], n3[3], n2[2];
#pragma unroll
  for (int i = 0; i < 10; ++i) w[i] = swap_add32(keep ? v[i] : 0.f, (keep && i < 9) ? v[i + 10] : 0.f);
#pragma unroll
  for (int i = 0; i < 5; ++i) u[i] = swap_add16(w[i], w[i + 5]);
  const bool h3 = (lane >> 3) & 1, h2 = (lane >> 2) & 1, h1 = (lane >> 1) & 1;
  n3[0] = dpp_pair_add<kDppMirror16>(u[0], u[3], h3);
  n3[1] = dpp_pair_add<kDppMirror16>(u[1], u[4], h3);
  n3[2] = dpp_pair_add<kDppMirror16>(u[2], 0.f, h3);
  n2[0] = dpp_pair_add<kDppMirror8>(n3[0], n3[2], h2);
  n2[1] = dpp_pair_add<kDppMirror8>(n3[1], 0.f, h2);
  float s = dpp_pair_add<kDppMirror4>(n2[0], n2[1], h1);
  return s + dpp_move<kDppSwap1>(s);
}

// Which of the 20 values lane `lane` holds after wave_sum20 (-1: padding or odd lane).
__device__ __forceinline__ int wave_sum20_index(int lane) {
  if (lane & 1) return -1;
  const int i2 = ((lane >> 1) & 1) + 2 * ((lane >> 2) & 1);  // slot among the 3 after the bit-3 step
  if (i2 >= 3) return -1;
  const int i3 = i2 + 3 * ((lane >> 3) & 1);  // slot among the 5 after the bit-4 step
  if (i3 >= 5) return -1;
  return i3 + 5 * ((lane >> 4) & 1) + 10 * ((lane >> 5) & 1);
}

}  // namespace cg
