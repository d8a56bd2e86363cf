// Backward pass.
//
// 1. Tile backward (k_render_bwd): the same tiles, wave quadrants and batches as the
//    forward.  Each pixel replays the forward front to back, so transmittance is
//    recomputed, never divided.  For a composited pair k with colour c_k, alpha_k and
//    transmittance T_k in front of it,
//      dL/dalpha_k = sum_ch G_ch (c_k T_k - (S_k + T_fin bg) / (1 - alpha_k)) + G_a T_fin / (1 - alpha_k),
//      dL/dc_k     = G alpha_k T_k,
//    where S_k = C_fin - C_{<=k} is the colour composited behind k (C_fin from the
//    forward output).  dL/dT_k = dL/dalpha_k below the alpha_max clamp.  The record
//    gradient of each pair (pair_grad) is summed over the quadrant's pixels by a
//    transposed wave reduction on the VALU lane movers (wave_ops.hpp) and over the
//    four quadrants through LDS, and written, without atomics, to the pair's
//    emission slot.
// 2. Per (view, Gaussian) sum of its pairs' partial gradients (contiguous slots).
// 3. Preprocess backward to the raw parameters, summing views in a fixed order.
#include <algorithm>

#include "fwd_state.hpp"
#include "pair_grad.hpp"
#include "pixel_buf.hpp"
#include "sh.hpp"

namespace cg {

constexpr int kGradLen = 20;  // dW[9] dmu[3] dsigma dsp2[3] drgb[3] pad (zero)

// stage_records with each Gaussian index clamped into the records: the training
// forward writes the indices of the pairs it stages, the same batches as an exact
// replay, so only a replay that walks further than the forward (which the mismatch
// diagnostic reports) reads entries it never wrote.
__device__ __forceinline__ void stage_replay_records(Record* srec, const Record* __restrict__ vrec,
                                                     const uint32_t* __restrict__ sorted_gid, int64_t n_gauss,
                                                     uint32_t first, int count) {
  constexpr int kTPR = 4, kVec = 8 / kTPR;
  const int r = (int)(threadIdx.x / kTPR), part = (int)(threadIdx.x % kTPR);
  if (r < count) {
    const uint32_t gid = min(sorted_gid[first + (uint32_t)r], (uint32_t)(n_gauss - 1));
    const float4* src = reinterpret_cast<const float4*>(vrec + gid) + kVec * part;
    float4* dst = reinterpret_cast<float4*>(srec + r) + kVec * part;
#pragma unroll
    for (int k = 0; k < kVec; ++k) dst[k] = src[k];
  }
}

// Four waves per SIMD: the register budget (128 VGPRs) that pair_grad fits in without
// spilling.
template <int FILTER, bool MARGINAL, bool GEER>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_render_bwd(const DevCamera* __restrict__ cams, int n_views, int total_tiles,
                                                    Opts o, const Record* __restrict__ rec,
                                                    int64_t n_gauss, const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ tile_order,
                                                    const uint32_t* __restrict__ sorted_gid,
                                                    const uint32_t* __restrict__ sorted_slots,
                                                    const float4* __restrict__ pix,
                                                    const unsigned long long* __restrict__ wmask,
                                                    int64_t mask_words,
                                                    const float* __restrict__ out_rgba,
                                                    const float* __restrict__ final_T,
                                                    const float* __restrict__ grad_rgba, float* __restrict__ partial,
                                                    unsigned int* __restrict__ mismatch,
                                                    uint32_t* __restrict__ n_long) {
  __shared__ Record srec[64];
  __shared__ float gacc[4][64][kGradLen + 1];
  // per-pixel constants read only where a pair contributes, kept in LDS (each thread its
  // own slot) instead of registers: at the 128-VGPR cap they would otherwise spill
  __shared__ float4 s_up[256], s_fo[256];
  const int t = (int)tile_order[blockIdx.x];
  const int v = view_of_tile(cams, n_views, t);
  const DevCamera& c = cams[v];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_long = 0u;  // the slot sums' long-item counter
  int i, j;
  tile_pixel(c, t - c.tile_offset, threadIdx.x, i, j);
  const bool inside = i < c.crop_w && j < c.crop_h;
  const PairPixel px = load_pair_pixel(pix, (int64_t)total_tiles * kTilePx, (int64_t)t * kTilePx + threadIdx.x);
  const bool valid = pixel_valid(px);
  const Origin org = make_origin(c);
  const unsigned long long* __restrict__ wm = wmask + (int64_t)wave * mask_words;
  const int red_idx = wave_sum20_index(lane);  // which gradient component this lane's wave sum holds

  // upstream gradient and forward result of this pixel
  // Fo: the forward output, C_fin + T_fin bg, which is all dL/dalpha needs of C_fin and
  // the background (S_k + T_fin bg = Fo - C_{<=k})
  // GaT: the upstream alpha gradient times T_fin, the only form dL/dalpha uses
  // s_up: (G_r, G_g, G_b, G_a T_fin), s_fo: (Fo_r, Fo_g, Fo_b, unused)
  int64_t p = 0;
  {
    float4 up = make_float4(0.f, 0.f, 0.f, 0.f), fo = up;
    if (inside) {
      p = c.px_offset + (int64_t)j * c.crop_w + i;
      up = reinterpret_cast<const float4*>(grad_rgba)[p];
      fo = reinterpret_cast<const float4*>(c.out)[(int64_t)j * c.crop_w + i];
      up.w *= final_T[p];
    }
    s_up[threadIdx.x] = up;
    s_fo[threadIdx.x] = fo;
  }

  const uint2 rg = ranges[t];
  float Ttr = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  bool done = !valid;
  const Record* vrec = rec + (int64_t)v * n_gauss;
  uint32_t stop_at = rg.y;
  for (uint32_t base = rg.x; base < rg.y; base += 64) {
    if (__syncthreads_count(!done) == 0) {
      stop_at = base;
      break;
    }
    const int cnt = (int)min(64u, rg.y - base);
    stage_replay_records(srec, vrec, sorted_gid, n_gauss, base, cnt);
    for (int k = lane; k < 64 * (kGradLen + 1); k += 64) (&gacc[wave][0][0])[k] = 0.f;
    __syncthreads();
    if (__ballot(!done) != 0) {
      // the pairs of this batch at which some pixel of the wave had alpha >= alpha_min in
      // the forward: every other pair leaves every pixel's state unchanged
      const uint32_t w0 = base >> 6, sh = base & 63u;
      uint64_t m = wm[w0] >> sh;
      if (sh) m |= wm[w0 + 1] << (64u - sh);
      if (cnt < 64) m &= (1ull << cnt) - 1ull;
      while (m) {
        const int k = (int)__builtin_ctzll(m);
        m &= m - 1;
        float gv[kGradLen];  // written by the contributing lanes only (the reduction adds zeros for the others)
        bool contrib = false;
        if (!done) {
          const Record& R = srec[k];
          // the forward's tests and response (pair_response), keeping the intermediates
          // that the reverse pass needs
          PairGeom gm;
          PairFoot ft;
          PairFloor fl;
          bool filt = true;
          if (pair_cheap<FILTER>(R, px, org, o, gm)) {
            const float T = pair_full_keep<FILTER, MARGINAL, GEER>(R, px, gm, ft, fl, filt);
            const float alpha = fminf(T, o.alpha_max);
            if (alpha >= o.alpha_min) {
              const float test = Ttr * (1.f - alpha);
              if (test < o.T_min) {
                done = true;
              } else {
                contrib = true;
                const float w = Ttr * alpha;
                C0 = fmaf(w, R.rgb[0], C0);
                C1 = fmaf(w, R.rgb[1], C1);
                C2 = fmaf(w, R.rgb[2], C2);
                const float inv1 = fast_rcp(1.f - alpha);
                // colour behind this pair plus the background it lets through
                const float4 up = s_up[threadIdx.x], fo = s_fo[threadIdx.x];
                const float G0 = up.x, G1 = up.y, G2 = up.z;
                const float B0 = fo.x - C0, B1 = fo.y - C1, B2 = fo.z - C2;
                float dalpha = up.w * inv1;
                dalpha += G0 * (R.rgb[0] * Ttr - B0 * inv1);
                dalpha += G1 * (R.rgb[1] * Ttr - B1 * inv1);
                dalpha += G2 * (R.rgb[2] * Ttr - B2 * inv1);
                gv[16] = G0 * w;
                gv[17] = G1 * w;
                gv[18] = G2 * w;
                // alpha clamped at alpha_max: no gradient through T (every adjoint of
                // pair_grad is a multiple of dL/dT, so dL/dT = 0 gives exact zeros)
                pair_grad<FILTER, MARGINAL, GEER>(R, px, gm, ft, fl, filt, T < o.alpha_max ? dalpha : 0.f, T, gv);
                Ttr = test;
              }
            }
          }
        }
        if (__ballot(contrib) != 0) {
          // the lanes that did not contribute add zeros; gv[19] is the padding component
          const float s = wave_sum20(gv, contrib, lane);
          if (red_idx >= 0) gacc[wave][k][red_idx] = s;
        }
      }
    }
    __syncthreads();
    // sum the four quadrants and write each pair's partial gradient to its slot
    for (int e = threadIdx.x; e < cnt * kGradLen; e += 256) {
      const int k = e / kGradLen, q = e % kGradLen;
      const float s = gacc[0][k][q] + gacc[1][k][q] + gacc[2][k][q] + gacc[3][k][q];
      partial[(int64_t)sorted_slots[base + k] * kGradLen + q] = s;
    }
  }
  // pairs after the point where every pixel of the tile had terminated get no gradient
  for (int64_t e = threadIdx.x; e < (int64_t)(rg.y - stop_at) * kGradLen; e += 256)
    partial[(int64_t)sorted_slots[stop_at + e / kGradLen] * kGradLen + e % kGradLen] = 0.f;
  // pixels that ran to the end of their list must have reached the stored transmittance;
  // the tile's count of those that did not (every entry written: no zeroing needed)
  const int bad = __syncthreads_count(valid && !done && Ttr != (inside ? final_T[p] : 1.f));
  if (threadIdx.x == 0) mismatch[blockIdx.x] = (unsigned int)bad;
}

// Per (view, Gaussian) item: sum of its pairs' partials, gradient slots [off, off + cnt),
// added in slot order.  The forward lays the slots out item by item, in item order, so
// the items' slot ranges follow each other and the sums are read and written front to
// back.  5 lanes per item, each
// holding 4 of the 20 components of a row (one 16-byte load per lane; a row is one
// contiguous 80-byte segment).  Each lane group owns a run of kReduceRun consecutive
// items, i.e. one contiguous stretch of rows, which it streams kReduceBatch rows at a
// time whatever the items' sizes, closing an item's sum at its last row.  Plain
// (temporal) loads: a 128-byte line holds parts of two rows that one group reads in
// consecutive batches, and it must still be in the cache for the second.  The sums are
// kept in LDS and written once the whole chunk is summed: vector loads and stores
// share one wait counter, so a store among the loads would make every later wait for
// data also wait for that store's completion.  An item with more than kReduceLong
// slots (a Gaussian over many tiles) would hold its lane group for cnt / kReduceBatch
// batches after the others have finished: its rows are skipped here, and
// k_reduce_long sums it with a whole workgroup.
constexpr int kReduceLanes = kGradLen / 4;
constexpr int kReduceItemsPerWave = 64 / kReduceLanes;         // 12 lane groups
constexpr int kReduceBatch = 16;
constexpr int kReduceLong = 128;
constexpr int kReduceRun = 8;                                   // consecutive items per lane group
constexpr int kReduceChunk = kReduceRun * kReduceItemsPerWave;  // 96 items per wave
constexpr int kReduceBlocks = 16384;
constexpr int kReduceLongBlocks = 2048;
typedef float red4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_reduce_items(const uint32_t* __restrict__ counts,
                                                      const uint32_t* __restrict__ offsets, int64_t nv,
                                                      const float* __restrict__ partial,
                                                      float* __restrict__ item_grad,
                                                      uint32_t* __restrict__ long_items,
                                                      uint32_t* __restrict__ n_long) {
  __shared__ uint32_t s_cnt[4][kReduceChunk];
  __shared__ red4 s_sum[4][kReduceChunk][kReduceLanes];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sub = lane / kReduceLanes, c = lane - sub * kReduceLanes;
  const bool grp = sub < kReduceItemsPerWave;
  const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const red4 zero = {0.f, 0.f, 0.f, 0.f};
  red4* __restrict__ sums = &s_sum[wave][0][0];
  for (int64_t ch = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; ch * kReduceChunk < nv; ch += n_waves) {
    const int64_t base = ch * kReduceChunk;
    const int m = (int)min<int64_t>(kReduceChunk, nv - base);
    for (int k = lane; k < m; k += 64) s_cnt[wave][k] = counts[base + k];
    // empty and long items keep a zero sum here (k_reduce_long writes the long ones later)
    for (int k = lane; k < m * kReduceLanes; k += 64) sums[k] = zero;
    __builtin_amdgcn_wave_barrier();
    // this group's run of items [j, jend): a contiguous stretch of rows, except that the
    // rows of long items are skipped
    int j = grp ? sub * kReduceRun : m;
    const int jend = min(j + kReduceRun, m);
    uint32_t row = 0;
    if (j < m) row = offsets[base + j];
    for (int q = j; q < jend; ++q)
      if (s_cnt[wave][q] > (uint32_t)kReduceLong && c == 0) long_items[atomicAdd(n_long, 1u)] = (uint32_t)(base + q);
    // Positions the group at its next item with rows, jumping over the rows of long
    // items; seg_end: where the next long item (or the run's rows) begins, the end of
    // the stretch that the batches may read.
    uint32_t left = 0, seg_end = row;
    auto settle = [&]() {
      while (j < jend) {
        const uint32_t cq = s_cnt[wave][j];
        if (cq == 0u) {
          ++j;
        } else if (cq > (uint32_t)kReduceLong) {
          row += cq;
          ++j;
        } else {
          break;
        }
      }
      if (j < jend) {
        left = s_cnt[wave][j];
        if (row >= seg_end) {
          seg_end = row;
          for (int q = j; q < jend; ++q) {
            const uint32_t cq = s_cnt[wave][q];
            if (cq > (uint32_t)kReduceLong) break;
            seg_end += cq;
          }
        }
      }
    };
    settle();
    red4 acc = zero;
    while (__ballot(j < jend) != 0) {
      if (j < jend) {
        const uint32_t r0 = row;
        red4 v[kReduceBatch];
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u)
          v[u] = reinterpret_cast<const red4*>(partial)[(int64_t)min(r0 + (uint32_t)u, seg_end - 1u) * kReduceLanes + c];
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) {
          if (r0 + (uint32_t)u < seg_end && j < jend) {
            acc += v[u];
            ++row;
            if (--left == 0u) {
              sums[j * kReduceLanes + c] = acc;
              acc = zero;
              ++j;
              while (j < jend && s_cnt[wave][j] == 0u) ++j;
              if (j < jend) left = s_cnt[wave][j];
            }
          }
        }
        if (row >= seg_end) settle();
      }
    }
    __builtin_amdgcn_wave_barrier();
    // the chunk's sums: one contiguous stretch of item_grad
    red4* __restrict__ out = reinterpret_cast<red4*>(item_grad + base * kGradLen);
    for (int k = lane; k < m * kReduceLanes; k += 64) out[k] = sums[k];
    __builtin_amdgcn_wave_barrier();
  }
}

// The items k_reduce_items listed (more than kReduceLong slots), one workgroup each:
// its 48 lane groups take every 48th slot, kReduceLongBatch slots in flight per group,
// and their 48 partial sums are added in group order through LDS.  The order of the
// list does not matter: each item's sum is formed the same way wherever it is listed.
constexpr int kReduceLongGroups = 256 / 64 * kReduceItemsPerWave;  // 48
constexpr int kReduceLongBatch = 4;

__global__ __launch_bounds__(256) void k_reduce_long(const uint32_t* __restrict__ counts,
                                                     const uint32_t* __restrict__ offsets,
                                                     const float* __restrict__ partial,
                                                     float* __restrict__ item_grad,
                                                     const uint32_t* __restrict__ long_items,
                                                     const uint32_t* __restrict__ n_long) {
  __shared__ red4 part[kReduceLongGroups][kReduceLanes];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sub = lane / kReduceLanes, c = lane - sub * kReduceLanes;
  const bool active = sub < kReduceItemsPerWave;
  const int grp = wave * kReduceItemsPerWave + sub;
  const uint32_t total = *n_long;
  for (uint32_t e = blockIdx.x; e < total; e += gridDim.x) {
    const uint32_t it = long_items[e];
    const uint32_t cnt = counts[it];
    if (active) {
      const red4* src = reinterpret_cast<const red4*>(partial + (int64_t)offsets[it] * kGradLen) + c;
      red4 acc = {0.f, 0.f, 0.f, 0.f};
      for (uint32_t k = grp; k < cnt; k += kReduceLongGroups * kReduceLongBatch) {
        red4 v[kReduceLongBatch];
#pragma unroll
        for (int u = 0; u < kReduceLongBatch; ++u) {
          const uint32_t r = min(k + (uint32_t)(u * kReduceLongGroups), cnt - 1u);
          v[u] = __builtin_nontemporal_load(src + (int64_t)r * kReduceLanes);
        }
#pragma unroll
        for (int u = 0; u < kReduceLongBatch; ++u)
          if (k + (uint32_t)(u * kReduceLongGroups) < cnt) acc += v[u];
      }
      part[grp][c] = acc;
    }
    __syncthreads();
    if (threadIdx.x < kReduceLanes) {
      red4 s = part[0][threadIdx.x];
      for (int q = 1; q < kReduceLongGroups; ++q) s += part[q][threadIdx.x];
      reinterpret_cast<red4*>(item_grad + (int64_t)it * kGradLen)[threadIdx.x] = s;
    }
    __syncthreads();
  }
}

// Preprocess backward: per Gaussian, the per-view record gradients back to the raw
// parameters (activations of Sec. 3, the floor of Eq. 10, the colour).  Views are
// summed in index order; outputs are overwritten.  Each view's gradient row is read
// once, as five 16-byte loads; the colour gradients of the first kBwdKeepViews views
// wait in LDS for the colour passes (a strided 4-byte re-read of the rows there, after
// they have left the caches, fetched whole lines for one word each).
constexpr int kBwdKeepViews = 4;
__global__ __launch_bounds__(256) void k_preprocess_bwd(GaussPtrs g, const DevCamera* __restrict__ cams, int n_views, Opts o,
                                 const float* __restrict__ item_grad, float* __restrict__ d_means,
                                 float* __restrict__ d_log_scales, float* __restrict__ d_quats,
                                 float* __restrict__ d_logits, float* __restrict__ d_color) {
  __shared__ float s_dc[kBwdKeepViews][3][256];  // each thread its own column
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = g.n;
  if (i >= n) return;
  const float mu[3] = {g.means[i], g.means[n + i], g.means[2 * n + i]};
  const float q[4] = {g.quats[i], g.quats[n + i], g.quats[2 * n + i], g.quats[3 * n + i]};
  const float qnorm = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float qn = 1.f / qnorm;
  const float w = q[0] * qn, x = q[1] * qn, y = q[2] * qn, z = q[3] * qn;
  const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                      2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                      2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
  const float sigma = 1.f / (1.f + expf(-g.logits[i]));
  const float rho2 = (o.use_floor && g.rho2) ? g.rho2[i] : 0.f;
  float s[3], sp[3], sp2[3];
  float ratio = 1.f;
  for (int k = 0; k < 3; ++k) {
    s[k] = expf(g.log_scales[k * n + i]);
    if (rho2 > 0.f) {
      sp2[k] = s[k] * s[k] + rho2;
      sp[k] = sqrtf(sp2[k]);
      ratio *= s[k] / sp[k];
    } else {
      sp[k] = s[k];
      sp2[k] = s[k] * s[k];
    }
  }
  float dmu[3] = {0.f, 0.f, 0.f}, dR[9], dsp2[3] = {0.f, 0.f, 0.f}, dsig_eff = 0.f;
  for (int k = 0; k < 9; ++k) dR[k] = 0.f;
#pragma unroll 1
  for (int v = 0; v < n_views; ++v) {
    static_assert(kGradLen == 20, "a gradient row is five float4");
    const float4* r4 = reinterpret_cast<const float4*>(item_grad + ((int64_t)v * n + i) * kGradLen);
    const float4 r0 = r4[0], r1 = r4[1], r2 = r4[2], r3 = r4[3], r4v = r4[4];
    const float gr[19] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w, r2.x, r2.y,
                          r2.z, r2.w, r3.x, r3.y, r3.z, r3.w, r4v.x, r4v.y, r4v.z};
    if (v < kBwdKeepViews) {
      s_dc[v][0][threadIdx.x] = gr[16];
      s_dc[v][1][threadIdx.x] = gr[17];
      s_dc[v][2][threadIdx.x] = gr[18];
    }
    // W[a][b] = R[b][a] / s'_a
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float acc = 0.f;
#pragma unroll
      for (int b2 = 0; b2 < 3; ++b2) {
        dR[3 * b2 + a] += gr[3 * a + b2] / sp[a];
        acc += gr[3 * a + b2] * R[3 * b2 + a];
      }
      // d s'_a = -acc / s'_a^2  ->  d s'^2_a = d s'_a / (2 s'_a)
      dsp2[a] += -acc / (sp[a] * sp[a]) / (2.f * sp[a]);
    }
    dmu[0] += gr[9];
    dmu[1] += gr[10];
    dmu[2] += gr[11];
    dsig_eff += gr[12];
    dsp2[0] += gr[13];
    dsp2[1] += gr[14];
    dsp2[2] += gr[15];
  }
  // colour, one channel at a time so that a thread holds 16 coefficients, 16 basis
  // values and 16 accumulators (views again in index order)
  if (g.color_mode == 0) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float acc = 0.f;
#pragma unroll 1
      for (int v = 0; v < n_views; ++v)
        acc += v < kBwdKeepViews ? s_dc[v][ch][threadIdx.x] : item_grad[((int64_t)v * n + i) * kGradLen + 16 + ch];
      d_color[(int64_t)ch * n + i] = acc;
    }
  } else {
#pragma unroll 1
    for (int ch = 0; ch < 3; ++ch) {
      float cf[16], dcol[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        cf[k] = g.color[(int64_t)(3 * k + ch) * n + i];
        dcol[k] = 0.f;
      }
#pragma unroll 1
      for (int v = 0; v < n_views; ++v) {
        const float drgb =
            v < kBwdKeepViews ? s_dc[v][ch][threadIdx.x] : item_grad[((int64_t)v * n + i) * kGradLen + 16 + ch];
        const DevCamera& c = cams[v];
        const double vd[3] = {(double)mu[0] - c.o[0], (double)mu[1] - c.o[1], (double)mu[2] - c.o[2]};
        const double dist = sqrt(vd[0] * vd[0] + vd[1] * vd[1] + vd[2] * vd[2]);
        const float ux = (float)(vd[0] / dist), uy = (float)(vd[1] / dist), uz = (float)(vd[2] / dist);
        float Y[16];
        sh_basis3(ux, uy, uz, Y);
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < 16; ++k) acc += cf[k] * Y[k];
        const float dc = acc + 0.5f <= 0.f ? 0.f : drgb;  // a clamped channel passes nothing back
#pragma unroll
        for (int k = 0; k < 16; ++k) dcol[k] += dc * Y[k];
        // through the direction u = v / |v|: du = dc sum_k cf_k grad Y_k
        float du[3];
        sh_basis3_vjp(ux, uy, uz, cf, du);
        du[0] *= dc;
        du[1] *= dc;
        du[2] *= dc;
        const float ud = du[0] * ux + du[1] * uy + du[2] * uz;
        const float idist = (float)(1.0 / dist);
        dmu[0] += (du[0] - ud * ux) * idist;
        dmu[1] += (du[1] - ud * uy) * idist;
        dmu[2] += (du[2] - ud * uz) * idist;
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) d_color[(int64_t)(3 * k + ch) * n + i] = dcol[k];
    }
  }
  // sigma_eff = sigma * prod s / s'
  if (o.backbone == CG_BACKBONE_RAY_INTEGRAL) {
    // the record carries sigma_eff / g with g = (prod s'^2)^(1/6) (as in the forward)
    const double gm = pow((double)sp2[0] * (double)sp2[1] * (double)sp2[2], 1.0 / 6.0);
    const float ig = (float)(1.0 / gm);
    const float sig_rec = sigma * ratio * ig;
#pragma unroll
    for (int k = 0; k < 3; ++k) dsp2[k] += dsig_eff * sig_rec * (-1.f / (6.f * sp2[k]));
    dsig_eff *= ig;
  }
  const float dsig = dsig_eff * ratio;
  const float dratio = dsig_eff * sigma;
  for (int k = 0; k < 3; ++k) {
    // s'^2 = s^2 + rho2; ratio depends on s_k through s_k / sqrt(s_k^2 + rho2)
    float ds = dsp2[k] * 2.f * s[k];
    if (rho2 > 0.f) ds += dratio * ratio * (1.f / s[k] - s[k] / sp2[k]);
    d_log_scales[k * n + i] = ds * s[k];
  }
  d_logits[i] = dsig * sigma * (1.f - sigma);
  for (int k = 0; k < 3; ++k) d_means[k * n + i] = dmu[k];
  // R(q_hat) -> q_hat -> q
  const float dw = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  const float dx = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                          2.f * x * dR[8]);
  const float dy = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                          2.f * y * dR[8]);
  const float dz = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] + y * dR[5] +
                          x * dR[6] + y * dR[7]);
  const float dot = dw * w + dx * x + dy * y + dz * z;
  d_quats[i] = (dw - dot * w) * qn;
  d_quats[n + i] = (dx - dot * x) * qn;
  d_quats[2 * n + i] = (dy - dot * y) * qn;
  d_quats[3 * n + i] = (dz - dot * z) * qn;
}

template <int FILTER, bool MARGINAL, bool GEER>
static void launch_bwd_g(const cg_fwd_state* st, const float* grad_rgba, float* partial, unsigned int* mismatch,
                         uint32_t* n_long, hipStream_t s) {
  k_render_bwd<FILTER, MARGINAL, GEER><<<dim3((unsigned)st->total_tiles), dim3(256), 0, s>>>(
      st->dcams, st->n_views, (int)st->total_tiles, st->opts, st->rec, st->g.n, st->ranges, st->tile_order,
      st->sorted_gid,
      st->sorted_slots, st->pix, st->wmask, st->mask_words, st->out_rgba, st->final_T, grad_rgba, partial, mismatch,
      n_long);
}

template <int FILTER, bool MARGINAL>
static void launch_bwd_t(const cg_fwd_state* st, const float* grad_rgba, float* partial, unsigned int* mismatch,
                         uint32_t* n_long, hipStream_t s) {
  if (st->opts.backbone == CG_BACKBONE_RAY_INTEGRAL)
    launch_bwd_g<FILTER, MARGINAL, true>(st, grad_rgba, partial, mismatch, n_long, s);
  else
    launch_bwd_g<FILTER, MARGINAL, false>(st, grad_rgba, partial, mismatch, n_long, s);
}

void run_backward(cg_fwd_state* st, const float* grad_rgba, float* d_means, float* d_log_scales, float* d_quats,
                  float* d_opacity, float* d_color, hipStream_t s) {
  CG_CHECK_ARG(st, "null forward state");
  CG_CHECK_ARG(st->sorted_slots || st->P == 0, "state was not created for a backward pass");
  const int64_t n = st->g.n;
  if (n == 0) return;
  CG_CHECK_ARG(d_means && d_log_scales && d_quats && d_opacity && d_color, "null gradient output");
  CG_CHECK_ARG(grad_rgba || st->total_px == 0, "null grad_rgba");
  const int64_t nv = n * st->n_views;
  Scratch sc(&st->alloc, s);
  float *partial, *item_grad;
  uint32_t *long_items, *n_long;
  unsigned int* mismatch = st->bwd_mismatch;
  {
    Carve c;
    c.add(&partial, (size_t)std::max<int64_t>(st->P, 1) * kGradLen);
    c.add(&item_grad, (size_t)nv * kGradLen);
    // items with more than kReduceLong slots: at most P / kReduceLong of them
    c.add(&long_items, (size_t)(st->P / kReduceLong + 1));
    c.add(&n_long, 1);
    sc.get(c);
  }
  // k_render_bwd zeroes n_long (and writes every tile's mismatch count); without pairs
  // it does not run
  if (st->P == 0) CG_HIP(launch_fill_u32(n_long, 0u, 1, s));
  if (st->P > 0) {
    ProfScope ps(ST_BWD_RENDER, s);
    const Opts& o = st->opts;
    const bool marginal = o.use_floor && o.composition == CG_COMPOSE_MARGINAL;
    switch (o.filter_mode) {
      case CG_FILTER_CENTER_RAY: launch_bwd_t<0, false>(st, grad_rgba, partial, mismatch, n_long, s); break;
      case CG_FILTER_ISOTROPIC:
        if (marginal) launch_bwd_t<2, true>(st, grad_rgba, partial, mismatch, n_long, s);
        else launch_bwd_t<2, false>(st, grad_rgba, partial, mismatch, n_long, s);
        break;
      default:
        if (marginal) launch_bwd_t<1, true>(st, grad_rgba, partial, mismatch, n_long, s);
        else launch_bwd_t<1, false>(st, grad_rgba, partial, mismatch, n_long, s);
    }
    CG_HIP(hipGetLastError());
  }
  {
    ProfScope ps(ST_BWD_REDUCE, s);
    const int64_t waves = (nv + kReduceChunk - 1) / kReduceChunk;
    const int64_t blocks = std::min<int64_t>((waves + 3) / 4, kReduceBlocks);
    k_reduce_items<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(st->counts, st->offsets, nv,
                                                                partial, item_grad, long_items, n_long);
    CG_HIP(hipGetLastError());
    k_reduce_long<<<dim3(kReduceLongBlocks), dim3(256), 0, s>>>(st->counts, st->offsets, partial,
                                                               item_grad, long_items, n_long);
    CG_HIP(hipGetLastError());
  }
  {
    ProfScope ps(ST_BWD_PREPROCESS, s);
    k_preprocess_bwd<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(
        st->g, st->dcams, st->n_views, st->opts, item_grad, d_means, d_log_scales, d_quats, d_opacity, d_color);
    CG_HIP(hipGetLastError());
  }
  // no host synchronisation: the replay diagnostic stays on the device until asked for
  st->bwd_stream = s;
  st->bwd_ran = true;
  sc.check_guards();
}

}  // namespace cg

extern "C" cg_status cg_render_backward(cg_fwd_state* st, const float* grad_rgba, float* d_means,
                                        float* d_log_scales, float* d_quats, float* d_opacity_logits, float* d_color,
                                        hipStream_t stream) {
  try {
    cg::run_backward(st, grad_rgba, d_means, d_log_scales, d_quats, d_opacity_logits, d_color, stream);
    return CG_OK;
  } catch (const cg::Error& e) {
    cg::set_last_error(e.what());
    return e.status;
  } catch (const std::exception& e) {
    cg::set_last_error(e.what());
    return CG_ERR_STATE;
  }
}

extern "C" int64_t cg_bwd_replay_mismatches(const cg_fwd_state* st) {
  if (!st || !st->bwd_ran) return -1;
  if (st->P == 0) return 0;  // nothing was replayed
  std::vector<uint32_t> host((size_t)st->total_tiles);
  if (hipMemcpyAsync(host.data(), st->bwd_mismatch, host.size() * sizeof(uint32_t), hipMemcpyDeviceToHost,
                     st->bwd_stream) != hipSuccess ||
      hipStreamSynchronize(st->bwd_stream) != hipSuccess)
    return -1;
  int64_t total = 0;
  for (uint32_t x : host) total += x;
  return total;
}
