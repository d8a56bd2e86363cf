// Shared declarations of the ConeGaussian HIP library (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "conegauss.h"

namespace cg {

constexpr int kTile = 16;             // tile edge in pixels (one workgroup of 256 threads)
constexpr int kTilePx = kTile * kTile;
constexpr int kGroup = 8;             // tile group edge in tiles (64 tiles = one wave64)
constexpr int kGroupTiles = kGroup * kGroup;

// Pair indices, per-item offsets and sort element counts are 32-bit; a forward call's
// (tile, Gaussian) pairs must stay below this (an argument error otherwise).
constexpr uint64_t kMaxPairs = 0xF0000000ull;

constexpr float kPiF = 3.14159265358979323846f;
constexpr double kPi = 3.14159265358979323846;

// Device-side copy of a cg_camera, with the derived quantities the kernels need.
// Ray arithmetic is FP64 (see the ray section of camera_dev.hpp), so the intrinsics
// are kept in double.
struct DevCamera {
  int32_t model, full_w, full_h, crop_x0, crop_y0, crop_w, crop_h;
  int32_t tiles_x, tiles_y, groups_x, groups_y;
  int32_t tile_offset;   // first global tile index of this view
  int32_t group_offset;  // first global group index of this view
  uint32_t seg_len;      // split tile render: pairs per segment of this view's lists (0: whole tiles)
  int64_t px_offset;     // first pixel of this view in the per-pixel arrays
  float* out;            // this view's RGBA output, [crop_h][crop_w][4]
  double fx, fy, cx, cy, inv_fx, inv_fy, inv_w, inv_h;
  double k[4];
  double R[9];           // row-major camera-to-world
  double Rinv[9];        // inverse of R (world-to-camera)
  double o[3];
  double theta_max, thd_max;
  double eq_step[4];     // equirect: cos, sin of the half-pixel steps pi / W and -pi / (2 H)
  float of[3];           // origin as given (float32), for the float32 depth key
  float pad1;
};

// Bounding cone of the pixel-centre rays of a tile: unit axis, half angle beta (< 0:
// empty; >= pi: everything), sin/cos of beta/2 and the tile's largest footprint
// coefficient.
struct TileCone {
  float ax, ay, az, beta;
  float sb, cb, cmax, pad;
};

// Chord form of a cone, as the binning tests use it (a float4): unit axis (x, y, z) and
// chord radius w, the cone holding the unit directions d with |d - axis| <= w.  Two
// cones can share a direction only if |a - b| <= w_a + w_b (triangle inequality for
// the chord distance on the unit sphere).  kChordNever marks an empty cone (it
// overlaps nothing, even a kChordAll one); kChordAll one that holds every direction.
constexpr float kChordNever = -8.f, kChordAll = 4.f;

// Per (view, Gaussian) render record (128 bytes).  Cull cone: a ray direction d can
// reach the Gaussian only if |d - u| <= lim, u = v / |v| (the influence cone of the
// binning as a chord length; lim < 0: never, lim >= 2: always).  Tangent-cone test:
// with n = v x d, D^2(d) = n^T Sigma' n / (P^2 |W d|^2) (P = s'_1 s'_2 s'_3), and
// S = Sigma' / (Lambda P^2) turns the pre-rejection bound D^2 <= Lambda into
// n^T S n <= |W d|^2 (S = 0 accepts every ray).
struct alignas(16) Record {
  float vx, vy, vz, lim;   // v = mu - o rounded from FP64; chord limit of the cull cone
  float W[9];              // whitening diag(1/s') R^T, row-major
  float mu[3];             // mean
  float sigma;             // effective opacity sigma_eff (Eq. 10)
  float rgb[3];            // view-dependent colour
  float sp2[3];            // s'^2 (floored squared scales)
  float rho2;              // floor variance (0 when the floor is off)
  float Lg;                // 2 ln(sigma_eff / alpha_min): bound of the pre-rejection
  float kg;                // 1 / min(s'^2)
  float S[6];              // S00, 2 S01, 2 S02, S11, 2 S12, S22
};
static_assert(sizeof(Record) == 128, "Record layout");

// Stages the records of pairs first .. first + count - 1 of a sorted tile list into
// srec[0 .. count) with TPR threads of a 256-thread workgroup per record, 128 / TPR
// bytes each (count <= 256 / TPR): a wave's loads cover 64 / TPR whole records at once.
template <int TPR = 4>
__device__ __forceinline__ void stage_records(Record* srec, const Record* __restrict__ vrec,
                                              const uint32_t* __restrict__ sorted_gid, uint32_t first, int count) {
  static_assert(TPR == 2 || TPR == 4, "8 or 4 float4 per record and thread");
  constexpr int kVec = 8 / TPR;
  const int r = (int)(threadIdx.x / TPR), part = (int)(threadIdx.x % TPR);
  if (r < count) {
    const float4* src = reinterpret_cast<const float4*>(vrec + sorted_gid[first + (uint32_t)r]) + kVec * part;
    float4* dst = reinterpret_cast<float4*>(srec + r) + kVec * part;
#pragma unroll
    for (int k = 0; k < kVec; ++k) dst[k] = src[k];
  }
}

// Training forward: the sorted values are gradient slots.  The render kernel that
// stages a pair finds its Gaussian in the slot table and stores it in gid_out, for the
// backward (entries of pairs the forward never staged keep the value they had).
struct SlotGather {
  const uint32_t* slots = nullptr;
  const uint32_t* slot_gid = nullptr;
  uint32_t* gid_out = nullptr;
};

// stage_records for the training forward (TPR = 4): the Gaussian of each pair through
// the slot table, also stored for the backward.
__device__ __forceinline__ void stage_records_slots(Record* srec, const Record* __restrict__ vrec,
                                                    const SlotGather& sg, uint32_t first, int count) {
  constexpr int kTPR = 4, kVec = 8 / kTPR;
  const int r = (int)(threadIdx.x / kTPR), part = (int)(threadIdx.x % kTPR);
  if (r < count) {
    const uint32_t gid = sg.slot_gid[sg.slots[first + (uint32_t)r]];
    if (part == 0) sg.gid_out[first + (uint32_t)r] = gid;
    const float4* src = reinterpret_cast<const float4*>(vrec + gid) + kVec * part;
    float4* dst = reinterpret_cast<float4*>(srec + r) + kVec * part;
#pragma unroll
    for (int k = 0; k < kVec; ++k) dst[k] = src[k];
  }
}

// Hardware square root, reciprocal square root and reciprocal (about 1 ulp, no
// correctly-rounded expansion): for per-pair arithmetic whose tolerance is far above
// float32 rounding, and for conservative bounds that carry relative margins.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }

struct Opts {
  int filter_mode, use_floor, composition;
  float alpha_min, alpha_max, T_min, t_near;
  float bg[3];
  float fs;  // footprint scale
  int order_mode;
  int count_pairs;
  int backbone;  // 1: ray-integral factor 1 / (g |W d|) (the record's sigma carries 1 / g)
};

struct GaussPtrs {
  int64_t n;
  int color_mode;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* logits;
  const float* color;
  const float* rho2;
};

// Two small device arrays (p[k], n[k] 32-bit words) that a kernel zeroes on the side,
// in place of a fill launch of their own.
struct ClearPair {
  uint32_t* p[2];
  int n[2];
};

// ---------------------------------------------------------------- host-side launch API
// (each wraps kernels defined in one .hip translation unit)

// camera.hip
hipError_t launch_unproject(const DevCamera* cam, int64_t n, const float* pix_xy, float* dirs, uint8_t* valid,
                            hipStream_t s);
// pix: the per-pixel ray buffer, 4 * 16 bytes per slot, total_tiles * 256 slots; clr:
// two small arrays zeroed on the side
hipError_t launch_tile_cones(const DevCamera* cams, int n_views, int total_tiles, float fs, TileCone* tiles,
                             float4* pix, const ClearPair& clr, hipStream_t s);
// Per 8x8 tile group: its chord cone (groups), and a group-major copy of its 64 member
// tiles' chord cones (members, kChordNever for tiles outside the view; member l of
// group (gx, gy) is tile (8 gx + l % 8, 8 gy + l / 8)).  view_cmax: per-view maximum
// footprint coefficient, zeroed beforehand.
hipError_t launch_group_cones(const DevCamera* cams, int n_views, int total_groups, const TileCone* tiles,
                              float4* groups, float4* members, float* view_cmax,
                              hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_guard_check(const uint32_t* g, int n, uint32_t v, uint32_t* bad, hipStream_t s);

// preprocess.hip
// items[k] = k for every (view, Gaussian) item k, beside its depth key
hipError_t launch_preprocess(const GaussPtrs& g, const DevCamera* cams, int n_views, const float* view_cmax,
                             const Opts& o, Record* rec, uint32_t* depth_key, uint32_t* items, float4* cone,
                             hipStream_t s);

// binning.hip
// cone: per (view, Gaussian) chord cone of its influence cone (from the preprocess)
// The count pass keeps each (view, Gaussian) item's overlapping tile groups for the
// emit pass: hit_n[item] (their number, capped at 255) and hit_list[16 item ...] (the
// first 16, ascending).
constexpr int kBinHitList = 16;
hipError_t launch_bin_count(int64_t n, int n_views, const DevCamera* cams, const float4* cone, const float4* groups,
                            const float4* members, uint32_t* counts, uint8_t* hit_n, uint16_t* hit_list,
                            hipStream_t s);
// Emit pass: pair (tile, Gaussian) of item gv at positions offsets[gv] + j (compositing
// order).  Inference: vals = Gaussian index.  Training (slot_offs, slot_gid non-null):
// vals = the pair's gradient slot slot_offs[gv] + j, and slot_gid[slot] = Gaussian.
// The per-tile ranges (total_tiles entries) are zeroed on the side for k_tile_ranges.
// Pairs at positions (and slots) from cap on are dropped: the buffers hold cap entries.
hipError_t launch_bin_emit(int64_t n, int n_views, const DevCamera* cams, const float4* cone, const float4* groups,
                           const float4* members, const uint32_t* offsets, const uint32_t* slot_offs,
                           uint32_t* keys, uint32_t* vals, uint32_t* slot_gid, uint8_t* hit_n,
                           uint16_t* hit_list, uint2* ranges, int64_t total_tiles, int64_t cap, hipStream_t s);
hipError_t launch_gather_u32(const uint32_t* src, const uint32_t* idx, int64_t m, uint32_t* dst, hipStream_t s);
// The gather above that also adds the sum of the gathered values to *total (64 bits,
// zeroed beforehand): the exact pair count, which 32-bit offsets cannot hold.
hipError_t launch_gather_total(const uint32_t* src, const uint32_t* idx, int64_t m, uint32_t* dst,
                               unsigned long long* total, hipStream_t s);
hipError_t launch_scatter_u32(const uint32_t* src, const uint32_t* idx, int64_t m, uint32_t* dst, hipStream_t s);
hipError_t launch_tile_ranges(const uint32_t* keys, int64_t n, uint2* ranges, hipStream_t s);
// order: a permutation of the tiles, heaviest (most pairs) first, for the render launches
hipError_t launch_tile_order(const uint2* ranges, int total_tiles, uint32_t* order, hipStream_t s);
// Per view v with fewer than max_tiles tiles: stats[2v] = its longest tile list,
// stats[2v + 1] = its pairs (0, 0 for larger views).
hipError_t launch_view_stats(const DevCamera* cams, int n_views, const uint2* ranges, int64_t max_tiles,
                             uint32_t* stats, hipStream_t s);

// sort.hip
size_t scan_temp_bytes(int64_t n);
hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, void* temp, hipStream_t s);
// out[perm[k]] = sum of vals[perm[k']] over k' < k (the exclusive scan in the order perm
// gives, written back in vals' order), vals_perm[k] = vals[perm[k]], and the sum of all
// added to *total (64 bits, zeroed beforehand).  vals_perm_scan: scratch of n words for
// the many-tile path; temp: scan_temp_bytes(n).
hipError_t launch_permuted_scan(const uint32_t* vals, const uint32_t* perm, int64_t n, uint32_t* vals_perm,
                                uint32_t* vals_perm_scan, uint32_t* out, unsigned long long* total, void* temp,
                                hipStream_t s);
size_t radix_temp_bytes(int64_t n);
// Sorts (keys, vals) stably on bits [0, end_bit) (bits from end_bit up ride along and
// need not be zero); returns 0 if the result is in (keys, vals) and 1 if it is in
// (keys_alt, vals_alt).
hipError_t launch_radix_sort32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, int64_t n,
                               int end_bit, void* temp, int* result_in_alt, hipStream_t s);

// render_fwd.hip
// Per pair of the sorted tile lists: the smallest lower bound of t* over the pair and
// every later pair of its tile (order_mode RAY).
hipError_t launch_order_bounds(const DevCamera* cams, int n_views, int total_tiles, const Record* rec,
                               int64_t n_gauss, const uint2* ranges, const uint32_t* sorted_gid, float* tlo_suffix,
                               hipStream_t s);
// tile_order: the launch's tile sequence (launch_tile_order).  wmask (training forward,
// else NULL): 4 bitsets of mask_words 64-bit words, zeroed beforehand; bit p of bitset
// w is set when some pixel of wave w had alpha >= alpha_min at sorted pair p.  The
// training forward finds each pair's Gaussian through sg (sorted_gid unused).
hipError_t launch_render_fwd(const DevCamera* cams, int n_views, int total_tiles, const Opts& o, const Record* rec,
                             int64_t n_gauss, const uint2* ranges, const uint32_t* tile_order,
                             const uint32_t* sorted_gid, const float4* pix, const float* tlo_suffix, float* out_rgba,
                             float* final_T, uint32_t* n_last, unsigned long long* wmask, int64_t mask_words,
                             unsigned long long* counters, const SlotGather& sg, hipStream_t s);

// Split tile render (long lists on views with few tiles; render_fwd.hip).  The tiles of
// views with DevCamera::seg_len > 0 are cut into segments of that many pairs; the
// others are left to launch_render_fwd (which skips the split views' tiles).  Buffers:
// nseg, seg_off: total_tiles entries; seg_tile: max_segs; seg_prod: max_segs * 256
// floats; seg_out: max_segs * 256 float4; scan_tmp: scan_temp_bytes(total_tiles).
// max_segs must be at least the sum over split views of tiles + pairs / seg_len.
struct SegPlan {
  int64_t max_segs;
  uint32_t* nseg;
  uint32_t* seg_off;
  uint32_t* seg_tile;
  float* seg_prod;
  float4* seg_out;
  void* scan_tmp;
};
hipError_t launch_render_fwd_split(const DevCamera* cams, int n_views, int total_tiles, const Opts& o,
                                   const Record* rec, int64_t n_gauss, const uint2* ranges, const SegPlan& sp,
                                   const uint32_t* sorted_gid, const float4* pix, hipStream_t s);
// The thresholds of the split render (cg_set_tile_split; runtime.cpp).
struct SplitPolicy {
  int64_t max_tiles, min_longest, seg_len;
};
SplitPolicy split_policy();
// Segment length of the split render: about kSegTarget segments in all, at least
// kMinSegLen pairs each.
constexpr int64_t kMinSegLen = 384, kSegTarget = 16384;
// The one-workgroup-per-tile render takes at least as long as its longest list on one
// workgroup; the split render about two passes over all P pairs spread over the chip's
// ~2048 resident workgroups, plus its set-up.  Split when the longest list exceeds
// both policy.min_longest and P / kSplitShare.
constexpr int64_t kSplitShare = 1024;
inline bool split_wins(const SplitPolicy& p, int64_t longest, int64_t P) {
  return longest > p.min_longest && longest > P / kSplitShare;
}

// bake.hip
hipError_t launch_bake_rho2(const GaussPtrs& g, const DevCamera* cams, int n_views, float t_near, float* rho2,
                            hipStream_t s);

// ---------------------------------------------------------------- profiling (pool.cpp)
enum Stage {
  ST_CAMERA = 0, ST_PREPROCESS, ST_BIN_COUNT, ST_DEPTH_SORT, ST_SCAN, ST_BIN_EMIT, ST_SORT, ST_RANGES, ST_RENDER,
  ST_BWD_RENDER, ST_BWD_REDUCE, ST_BWD_PREPROCESS, ST_BAKE, ST_PROBE, ST_NUM
};
void prof_begin(int stage, hipStream_t s);
void prof_end(int stage, hipStream_t s);

}  // namespace cg
