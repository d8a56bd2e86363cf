// Tile render: one 256-thread workgroup per 16x16 tile, one pixel per thread, one 8x8
// quadrant per wavefront.  The tile's depth-sorted list of Gaussians is walked in
// batches of kFwdBatch records staged in LDS; each wavefront keeps the records whose
// influence cone can reach its quadrant, and every pixel evaluates the filtered
// closed-form response of Eq. 9 (with the marginal floor composition of Eq. 12) and
// composites front to back (Eq. 4).  The workgroup stops fetching batches once every
// pixel has terminated.
#include "pixel_buf.hpp"

namespace cg {

// Records staged per batch (128 B each, loaded by the first kFwdBatch threads).  With
// 8 KiB of LDS per workgroup and at most 64 VGPRs (amdgpu_waves_per_eu(8) on the
// kernel), eight waves per SIMD stay resident: the loop is VALU-bound with long LDS
// and FP64 latencies, which more resident waves hide.  One wave's worth of records per
// batch: the workgroup checks for termination and waits for its staging once per
// batch, so short batches stop sooner after the last pixel terminates.
constexpr int kFwdBatch = 64;
static_assert(kFwdBatch == 64, "one wave of records per batch, staged by stage_records (at most 64)");

// COUNT: also count, per pixel, the pairs that reached the per-pixel tests, those that
// needed the full footprint arithmetic and those composited, into counters[0..2].
// MASK (training forward): also set, per wave, the bit of every pair of the sorted list
// for which some pixel of the wave had alpha >= alpha_min (it composited or terminated
// there), in wmask[wave][pair / 64]; the backward replays only those pairs.
template <int FILTER, bool MARGINAL, bool COUNT, bool GEER, bool MASK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_render(const DevCamera* __restrict__ cams, int n_views, int total_tiles,
                                                Opts o, const Record* __restrict__ rec, int64_t n_gauss,
                                                const uint2* __restrict__ ranges,
                                                const uint32_t* __restrict__ tile_order,
                                                const uint32_t* __restrict__ sorted_gid,
                                                const float4* __restrict__ pix, float* __restrict__ out_rgba,
                                                float* __restrict__ final_T, uint32_t* __restrict__ n_last,
                                                unsigned long long* __restrict__ wmask, int64_t mask_words,
                                                unsigned long long* __restrict__ counters, SlotGather sg) {
  __shared__ Record srec[kFwdBatch];
  __shared__ unsigned int scount[3];
  uint32_t c_eval = 0, c_full = 0, c_contrib = 0;
  const int t = (int)tile_order[blockIdx.x];
  const int v = view_of_tile(cams, n_views, t);
  const DevCamera& c = cams[v];
  if (c.seg_len != 0u) return;  // a view of the split tile render (launch_render_fwd_split)
  const int lane = threadIdx.x & 63;
  int i, j;
  tile_pixel(c, t - c.tile_offset, threadIdx.x, i, j);
  const bool inside = i < c.crop_w && j < c.crop_h;
  const PairPixel px = load_pair_pixel(pix, (int64_t)total_tiles * kTilePx, (int64_t)t * kTilePx + threadIdx.x);
  const bool valid = pixel_valid(px);
  const Origin org = make_origin(c);
  const WaveCone wc = wave_cone(px, valid);
  unsigned long long* const wm = MASK ? wmask + (int64_t)(threadIdx.x >> 6) * mask_words : nullptr;

  const uint2 rg = ranges[t];
  float Ttr = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  bool done = !valid;
  uint32_t last = rg.x;
  const Record* vrec = rec + (int64_t)v * n_gauss;
  for (uint32_t base = rg.x; base < rg.y; base += kFwdBatch) {
    if (__syncthreads_count(!done) == 0) break;
    const int cnt = (int)min((uint32_t)kFwdBatch, rg.y - base);
    if (MASK)
      stage_records_slots(srec, vrec, sg, base, cnt);
    else
      stage_records(srec, vrec, sorted_gid, base, cnt);
    __syncthreads();
    if (wc.live && __ballot(!done) != 0) {
      for (int sub = 0; sub < cnt; sub += 64) {
        bool rel = false;
        if (sub + lane < cnt) {
          rel = record_reaches_cone(srec[sub + lane], wc.ax, wc.ay, wc.az, wc.rad);
        }
        uint64_t m = __ballot(rel);
        uint64_t hits = 0;  // MASK: bit k - sub for the pairs with some pixel at alpha >= alpha_min
        while (m) {
          const int k = sub + (int)__builtin_ctzll(m);
          m &= m - 1;
          bool hit = false;
          if (!done) {
            float T;
            if (COUNT) ++c_eval;
            if (pair_response<FILTER, MARGINAL, GEER>(srec[k], px, org, o, T)) {
              if (COUNT) ++c_full;
              const float alpha = fminf(T, o.alpha_max);
              if (alpha >= o.alpha_min) {
                hit = true;
                const float test = Ttr * (1.f - alpha);
                if (test < o.T_min) {
                  done = true;
                  last = base + (uint32_t)k;
                } else {
                  if (COUNT) ++c_contrib;
                  const float w = Ttr * alpha;
                  C0 = fmaf(w, srec[k].rgb[0], C0);
                  C1 = fmaf(w, srec[k].rgb[1], C1);
                  C2 = fmaf(w, srec[k].rgb[2], C2);
                  Ttr = test;
                }
              }
            }
          }
          if (MASK && __ballot(hit) != 0) hits |= 1ull << (k - sub);
          if (__ballot(!done) == 0) break;
        }
        if (MASK && hits != 0 && lane == 0) {  // pair base + sub is bit 0 of hits
          const uint32_t r0 = base + (uint32_t)sub, sh = r0 & 63u;
          atomicOr(&wm[r0 >> 6], (unsigned long long)(hits << sh));
          if (sh != 0 && (hits >> (64u - sh)) != 0) atomicOr(&wm[(r0 >> 6) + 1], (unsigned long long)(hits >> (64u - sh)));
        }
        if (__ballot(!done) == 0) break;
      }
    }
    if (!done) last = base + (uint32_t)cnt;
    __syncthreads();
  }
  if (inside) {
    const int64_t p = c.px_offset + (int64_t)j * c.crop_w + i;
    float4 out;
    out.x = C0 + Ttr * o.bg[0];
    out.y = C1 + Ttr * o.bg[1];
    out.z = C2 + Ttr * o.bg[2];
    out.w = 1.f - Ttr;
    reinterpret_cast<float4*>(c.out)[(int64_t)j * c.crop_w + i] = out;
    if (final_T) final_T[p] = Ttr;
    if (n_last) n_last[p] = valid ? last : rg.x;
  }
  if (COUNT) {
    if (threadIdx.x < 3) scount[threadIdx.x] = 0;
    __syncthreads();
    atomicAdd(&scount[0], c_eval);
    atomicAdd(&scount[1], c_full);
    atomicAdd(&scount[2], c_contrib);
    __syncthreads();
    if (threadIdx.x < 3) atomicAdd(&counters[threadIdx.x], (unsigned long long)scount[threadIdx.x]);
  }
}

// ---------------------------------------------------------------------------- per-ray order
// order_mode RAY: each pixel composites its pairs in the order of their own t* along
// its ray (Sec. 3), ties broken by list position: the key of a pair is (t*, position).
// The tile list is in per-Gaussian key order, and every record bounds from below the t*
// of any pair it can form (record_tstar_lower); with the suffix minimum of those bounds
// over the rest of the list, a pending pair whose t* is at most that minimum can no
// longer be preceded and is composited.  Pending pairs (t*, alpha, list position) wait
// in a per-pixel buffer in registers.  When it is full, the pair with the largest key
// (the new one or a pending one) is deferred, and the pixel's horizon h becomes the
// smallest deferred key: from then on this walk composites only keys below h, and
// every such key is either composited or pending when the walk ends.  A pixel with a
// horizon walks the list again for the keys from h on, and so on: each walk composites
// the keys of [lo, h) in order, so the order is exact however many pairs a pixel has.
constexpr int kRayBuf = 16;
// Records staged per batch of the per-ray-order kernel (one thread per record).
constexpr int kRayBatch = 128;

// Lower bound of t* over the pairs record R can form: pair_cheap admits only D <=
// D_max (the tangent-cone test; D_max^2 = sum s'^2 / (tr S prod s'^2) from S =
// Sigma' / (D_max^2 P^2)), and the max-response point lies within s'_max D of the
// mean, so t* >= |v| - s'_max D_max.  Culled records give +inf, unbounded ones -inf.
__device__ __forceinline__ float record_tstar_lower(const Record& R) {
  if (R.lim < 0.f) return INFINITY;
  const float trS = R.S[0] + R.S[3] + R.S[5];
  if (!(trS > 0.f)) return -INFINITY;
  const float vlen = sqrtf(R.vx * R.vx + R.vy * R.vy + R.vz * R.vz);
  const float P2 = R.sp2[0] * R.sp2[1] * R.sp2[2];
  const float dmax2 = (R.sp2[0] + R.sp2[1] + R.sp2[2]) / (trS * P2);
  const float smax = sqrtf(fmaxf(R.sp2[0], fmaxf(R.sp2[1], R.sp2[2])));
  return vlen * (1.f - 1e-5f) - smax * sqrtf(dmax2) * 1.0001f - 1e-6f;
}

// One workgroup per tile: tlo_suffix[j] = min of record_tstar_lower over list entries
// j.. end of the tile, walking the list from its end in chunks of 256.
__global__ __launch_bounds__(256) void k_order_bounds(const DevCamera* __restrict__ cams, int n_views,
                                                      const Record* __restrict__ rec, int64_t n_gauss,
                                                      const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ sorted_gid,
                                                      float* __restrict__ tlo_suffix) {
  __shared__ float sm[256];
  const int t = blockIdx.x;
  const int v = view_of_tile(cams, n_views, t);
  const Record* vrec = rec + (int64_t)v * n_gauss;
  const uint2 rg = ranges[t];
  float carry = INFINITY;
  for (int64_t end = rg.y; end > (int64_t)rg.x; end -= 256) {
    const int64_t idx = end - 1 - threadIdx.x;  // thread 0 holds the chunk's last entry
    float x = idx >= (int64_t)rg.x ? record_tstar_lower(vrec[sorted_gid[idx]]) : INFINITY;
    // inclusive min-scan over thread order = suffix minimum in list order
    sm[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const float y = threadIdx.x >= (unsigned)off ? sm[threadIdx.x - off] : INFINITY;
      __syncthreads();
      x = fminf(x, y);
      sm[threadIdx.x] = x;
      __syncthreads();
    }
    if (idx >= (int64_t)rg.x) tlo_suffix[idx] = fminf(x, carry);
    carry = fminf(carry, sm[255]);
    __syncthreads();
  }
}

template <int FILTER, bool MARGINAL, bool COUNT, bool GEER>
__global__ __launch_bounds__(256) void k_render_ray(const DevCamera* __restrict__ cams, int n_views, int total_tiles,
                                                    Opts o, const Record* __restrict__ rec,
                                                    int64_t n_gauss, const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ tile_order,
                                                    const uint32_t* __restrict__ sorted_gid,
                                                    const float4* __restrict__ pix,
                                                    const float* __restrict__ tlo_suffix,
                                                    unsigned long long* __restrict__ counters) {
  __shared__ Record srec[kRayBatch];
  __shared__ float slo[kRayBatch + 1];
  __shared__ unsigned int scount[4];
  uint32_t c_eval = 0, c_full = 0, c_contrib = 0, c_defer = 0;
  const int t = (int)tile_order[blockIdx.x];
  const int v = view_of_tile(cams, n_views, t);
  const DevCamera& c = cams[v];
  const int lane = threadIdx.x & 63;
  int i, j;
  tile_pixel(c, t - c.tile_offset, threadIdx.x, i, j);
  const bool inside = i < c.crop_w && j < c.crop_h;
  const PairPixel px = load_pair_pixel(pix, (int64_t)total_tiles * kTilePx, (int64_t)t * kTilePx + threadIdx.x);
  const bool valid = pixel_valid(px);
  const Origin org = make_origin(c);
  const WaveCone wc = wave_cone(px, valid);

  float Ttr = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  bool done = !valid;  // terminated (or no valid ray): nothing more to composite
  bool idle = done;    // no key left for this pixel in the current walk range
  const Record* vrec = rec + (int64_t)v * n_gauss;
  // pending pairs: t* (INFINITY = empty slot), alpha, list position; bmin = smallest t*
  float bt[kRayBuf], ba[kRayBuf];
  uint32_t bpos[kRayBuf];
#pragma unroll
  for (int q = 0; q < kRayBuf; ++q) {
    bt[q] = INFINITY;
    ba[q] = 0.f;
    bpos[q] = 0u;
  }
  float bmin = INFINITY;
  // keys (t*, position) of this walk: lo <= key < h; h = (INFINITY, ~0) while nothing
  // has been deferred
  float lo_t = -INFINITY, h_t = INFINITY;
  uint32_t lo_p = 0u, h_p = ~0u;
  // composites the pending pair with the smallest key; called only with bmin < INFINITY,
  // so every call removes one entry and each flush loop ends
  auto pop_min = [&]() {
    int sel = 0;
    float st = INFINITY;
    uint32_t sp = ~0u;
#pragma unroll
    for (int q = 0; q < kRayBuf; ++q)
      if (bt[q] < st || (bt[q] == st && bt[q] < INFINITY && bpos[q] < sp)) {
        st = bt[q];
        sp = bpos[q];
        sel = q;
      }
    float a = 0.f;
#pragma unroll
    for (int q = 0; q < kRayBuf; ++q)
      if (q == sel) {
        a = ba[q];
        bt[q] = INFINITY;
      }
    bmin = bt[0];
#pragma unroll
    for (int q = 1; q < kRayBuf; ++q) bmin = fminf(bmin, bt[q]);
    const float test = Ttr * (1.f - a);
    if (test < o.T_min) {
      done = idle = true;
      return;
    }
    if (COUNT) ++c_contrib;
    const float* rgb = vrec[sorted_gid[sp]].rgb;
    const float w = Ttr * a;
    C0 = fmaf(w, rgb[0], C0);
    C1 = fmaf(w, rgb[1], C1);
    C2 = fmaf(w, rgb[2], C2);
    Ttr = test;
  };

  const uint2 rg = ranges[t];
  // Every walk in which a pixel defers composites at least the kRayBuf pairs pending at
  // its end (or ends the pixel), and each pair of the list is composited once, so a list
  // of L pairs needs at most L / kRayBuf + 1 walks: the loop bound is never reached.
  const int max_walks = (int)((rg.y - rg.x) / kRayBuf) + 2;
  for (int walk = 0; walk < max_walks; ++walk) {
    for (uint32_t base = rg.x; base < rg.y; base += kRayBatch) {
      if (__syncthreads_count(!idle) == 0) break;
      const uint32_t idx = base + threadIdx.x;
      const int cnt = (int)min((uint32_t)kRayBatch, rg.y - base);
      // one thread per record: this kernel's pending buffers leave no registers for the
      // wider copies of stage_records
      if ((int)threadIdx.x < cnt) srec[threadIdx.x] = vrec[sorted_gid[idx]];
      if ((int)threadIdx.x <= cnt) slo[threadIdx.x] = idx < rg.y ? tlo_suffix[idx] : INFINITY;
      __syncthreads();
      if (wc.live && __ballot(!idle) != 0) {
        for (int sub = 0; sub < cnt; sub += 64) {
          bool rel = false;
          if (sub + lane < cnt) rel = record_reaches_cone(srec[sub + lane], wc.ax, wc.ay, wc.az, wc.rad);
          uint64_t m = __ballot(rel);
          while (m) {
            const int k = sub + (int)__builtin_ctzll(m);
            m &= m - 1;
            if (!idle) {
              if (COUNT && walk == 0) ++c_eval;
              const Record& R = srec[k];
              const uint32_t pos = base + (uint32_t)k;
              PairGeom g;
              if (pair_cheap<FILTER>(R, px, org, o, g)) {
                const float ts = g.tstar;
                // inside this walk's key range [lo, h)?
                const bool above_lo = ts > lo_t || (ts == lo_t && pos >= lo_p);
                const bool below_h = ts < h_t || (ts == h_t && pos < h_p);
                if (above_lo && below_h) {
                  if (COUNT) ++c_full;
                  const float alpha = fminf(pair_full<FILTER, MARGINAL, GEER>(R, px, g), o.alpha_max);
                  if (alpha >= o.alpha_min) {
                    bool full = true;
#pragma unroll
                    for (int q = 0; q < kRayBuf; ++q) full = full && bt[q] < INFINITY;
                    float nt = ts, na = alpha;
                    uint32_t np = pos;
                    if (full) {
                      // defer the largest key of the pending pairs and the new one
                      int sel = -1;
                      float mt = ts;
                      uint32_t mp = pos;
#pragma unroll
                      for (int q = 0; q < kRayBuf; ++q)
                        if (bt[q] > mt || (bt[q] == mt && bpos[q] > mp)) {
                          mt = bt[q];
                          mp = bpos[q];
                          sel = q;
                        }
                      ++c_defer;
                      h_t = mt;
                      h_p = mp;
#pragma unroll
                      for (int q = 0; q < kRayBuf; ++q)
                        if (q == sel) {
                          bt[q] = nt;
                          ba[q] = na;
                          bpos[q] = np;
                        }
                      if (sel >= 0) {
                        bmin = bt[0];
#pragma unroll
                        for (int q = 1; q < kRayBuf; ++q) bmin = fminf(bmin, bt[q]);
                      }
                    } else {
                      bool placed = false;
#pragma unroll
                      for (int q = 0; q < kRayBuf; ++q)
                        if (!placed && !(bt[q] < INFINITY)) {
                          bt[q] = nt;
                          ba[q] = na;
                          bpos[q] = np;
                          placed = true;
                        }
                      bmin = fminf(bmin, nt);
                    }
                  }
                }
              }
              // no record after k can precede a pending t* at or below this bound
              const float bound = slo[k + 1];
              while (!done && bmin < INFINITY && bmin <= bound) pop_min();
            }
            if (__ballot(!idle) == 0) break;
          }
          if (__ballot(!idle) == 0) break;
        }
      }
      while (!done && bmin < INFINITY && bmin <= slo[cnt]) pop_min();
      __syncthreads();
    }
    // the list is walked: every pending key is below h and nothing later precedes it
    while (!done && bmin < INFINITY) pop_min();
    const bool again = !done && h_t < INFINITY;
    lo_t = h_t;
    lo_p = h_p;
    h_t = INFINITY;
    h_p = ~0u;
    idle = !again;
    if (__syncthreads_count(again) == 0) break;
  }
  if (inside) {
    float4 out;
    out.x = C0 + Ttr * o.bg[0];
    out.y = C1 + Ttr * o.bg[1];
    out.z = C2 + Ttr * o.bg[2];
    out.w = 1.f - Ttr;
    reinterpret_cast<float4*>(c.out)[(int64_t)j * c.crop_w + i] = out;
  }
  if (threadIdx.x < 4) scount[threadIdx.x] = 0;
  __syncthreads();
  if (COUNT) {
    atomicAdd(&scount[0], c_eval);
    atomicAdd(&scount[1], c_full);
    atomicAdd(&scount[2], c_contrib);
  }
  if (c_defer) atomicAdd(&scount[3], c_defer);
  __syncthreads();
  if (threadIdx.x < 4 && scount[threadIdx.x]) atomicAdd(&counters[threadIdx.x], (unsigned long long)scount[threadIdx.x]);
}

// ---------------------------------------------------------------------------- split tiles
// A view with few tiles and a few very long lists (a small view of a large scene, or a
// low resolution) leaves most of the GPU idle while one workgroup walks the longest
// list.  That view's lists are then cut into segments of L = DevCamera::seg_len pairs,
// each rendered by its own workgroup (k_seg_count / scan / k_seg_fill list them:
// nseg[t] segments per tile from seg_off[t], seg_tile[b] the tile of segment b; tiles
// of views rendered whole get none).
// Pass 1 composites every segment on its own, per pixel, from T = 1: its colour with
// the segment-local weights, and its transmittance product (the factors (1 - alpha) of
// its pairs with alpha >= alpha_min, ending with the first factor that takes the
// product below T_min).  A tile of one segment is then done.  k_seg_prefix turns the
// products into each segment's T_in = the product of the earlier segments' factors
// (left to right).  The walk of k_render ends inside segment q exactly when T_in >=
// T_min > T_in * (product of q): only there does pass 2 composite the segment again,
// from T_in and with the termination test.  k_seg_combine adds the segments' colours,
// each local one scaled by its T_in, up to the one where the pixel terminated.  Up to
// the order of the products and sums, this is the walk of k_render.
__global__ void k_seg_count(const DevCamera* __restrict__ cams, int n_views, const uint2* __restrict__ ranges,
                            int total_tiles, uint32_t* __restrict__ nseg) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total_tiles) return;
  const uint32_t L = cams[view_of_tile(cams, n_views, t)].seg_len;  // 0: a view rendered in whole tiles
  const uint32_t len = ranges[t].y - ranges[t].x;
  nseg[t] = L == 0u ? 0u : (len > L ? (len + L - 1) / L : 1u);
}

__global__ void k_seg_fill(const uint32_t* __restrict__ nseg, const uint32_t* __restrict__ seg_off, int total_tiles,
                           uint32_t* __restrict__ seg_tile) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total_tiles) return;
  for (uint32_t q = 0; q < nseg[t]; ++q) seg_tile[seg_off[t] + q] = (uint32_t)t;
}

template <int FILTER, bool MARGINAL, bool GEER, int PASS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_render_seg(
    const DevCamera* __restrict__ cams, int n_views, int total_tiles, Opts o, const Record* __restrict__ rec,
    int64_t n_gauss, const uint2* __restrict__ ranges, const uint32_t* __restrict__ nseg,
    const uint32_t* __restrict__ seg_off, const uint32_t* __restrict__ seg_tile,
    const uint32_t* __restrict__ sorted_gid, const float4* __restrict__ pix, float* __restrict__ seg_prod,
    float4* __restrict__ seg_out) {
  __shared__ Record srec[kFwdBatch];
  const uint32_t n_segs = seg_off[total_tiles - 1] + nseg[total_tiles - 1];
  const uint32_t b = blockIdx.x;
  if (b >= n_segs) return;
  const int t = (int)seg_tile[b];
  const uint32_t ns = nseg[t], q = b - seg_off[t];
  if (PASS == 2 && ns == 1) return;  // a one-segment tile was finished by pass 1
  const int v = view_of_tile(cams, n_views, t);
  const DevCamera& c = cams[v];
  const int lane = threadIdx.x & 63;
  int i, j;
  tile_pixel(c, t - c.tile_offset, threadIdx.x, i, j);
  const bool inside = i < c.crop_w && j < c.crop_h;
  const PairPixel px = load_pair_pixel(pix, (int64_t)total_tiles * kTilePx, (int64_t)t * kTilePx + threadIdx.x);
  const bool valid = pixel_valid(px);
  const Origin org = make_origin(c);
  const WaveCone wc = wave_cone(px, valid);
  const uint2 rg = ranges[t];
  const uint32_t L = c.seg_len;
  const uint32_t s0 = rg.x + q * L, s1 = min(s0 + L, rg.y);
  float Ttr = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  bool done = !valid;
  bool redo = false;  // pass 2: this pixel's walk ends inside this segment
  if (PASS == 2) {
    // T_in (k_seg_prefix) and the segment's own product (pass 1): composite again only
    // where the walk terminates inside this segment
    const int64_t slot = (int64_t)b * kTilePx + threadIdx.x;
    const float T_in = q > 0 ? seg_prod[slot] : 1.f;
    const float f = seg_out[slot].w;
    redo = valid && T_in >= o.T_min && T_in * f < o.T_min;
    done = !redo;
    Ttr = T_in;
  }
  const Record* vrec = rec + (int64_t)v * n_gauss;
  for (uint32_t base = s0; base < s1; base += kFwdBatch) {
    if (__syncthreads_count(!done) == 0) break;
    const int cnt = (int)min((uint32_t)kFwdBatch, s1 - base);
    stage_records(srec, vrec, sorted_gid, base, cnt);
    __syncthreads();
    if (wc.live && __ballot(!done) != 0) {
      for (int sub = 0; sub < cnt; sub += 64) {
        bool rel = false;
        if (sub + lane < cnt) rel = record_reaches_cone(srec[sub + lane], wc.ax, wc.ay, wc.az, wc.rad);
        uint64_t m = __ballot(rel);
        while (m) {
          const int k = sub + (int)__builtin_ctzll(m);
          m &= m - 1;
          if (!done) {
            float T;
            if (pair_response<FILTER, MARGINAL, GEER>(srec[k], px, org, o, T)) {
              const float alpha = fminf(T, o.alpha_max);
              if (alpha >= o.alpha_min) {
                const float test = Ttr * (1.f - alpha);
                if (test < o.T_min) {
                  done = true;
                  // pass 1 of a multi-segment tile keeps the product, which includes the
                  // factor that ends it; otherwise T stays where the walk ended (Eq. 4)
                  if (PASS == 1 && ns > 1) Ttr = test;
                } else {
                  const float w = Ttr * alpha;
                  C0 = fmaf(w, srec[k].rgb[0], C0);
                  C1 = fmaf(w, srec[k].rgb[1], C1);
                  C2 = fmaf(w, srec[k].rgb[2], C2);
                  Ttr = test;
                }
              }
            }
          }
          if (__ballot(!done) == 0) break;
        }
        if (__ballot(!done) == 0) break;
      }
    }
    __syncthreads();
  }
  const int64_t slot = (int64_t)b * kTilePx + threadIdx.x;
  if (PASS == 1 && ns == 1) {
    if (inside) {  // T_in = 1: the segment's walk is the pixel's
      float4 out;
      out.x = C0 + Ttr * o.bg[0];
      out.y = C1 + Ttr * o.bg[1];
      out.z = C2 + Ttr * o.bg[2];
      out.w = 1.f - Ttr;
      reinterpret_cast<float4*>(c.out)[(int64_t)j * c.crop_w + i] = out;
    }
  } else if (PASS == 1) {
    // the local colour and the segment's product (its factors, up to the one that ends it)
    seg_prod[slot] = Ttr;
    seg_out[slot] = make_float4(C0, C1, C2, Ttr);
  } else if (redo) {
    // composited again from T_in: the absolute colour and the transmittance where the
    // pixel terminated, stored as -(1 + T) (or, if rounding let it run to the end of the
    // segment, the transmittance there as -(3 + T))
    seg_out[slot] = make_float4(C0, C1, C2, done ? -(1.f + Ttr) : -(3.f + Ttr));
  }
}

// Per multi-segment tile and pixel: seg_prod[segment q] <- product of the factors of
// segments 0 .. q - 1 (segment 0 keeps its own product, which no pass reads).
__global__ __launch_bounds__(256) void k_seg_prefix(const uint32_t* __restrict__ nseg,
                                                    const uint32_t* __restrict__ seg_off, float* __restrict__ seg_prod) {
  const int t = blockIdx.x;
  const uint32_t ns = nseg[t];
  if (ns <= 1) return;
  float* p = seg_prod + (int64_t)seg_off[t] * kTilePx + threadIdx.x;
  float T = p[0];
  for (uint32_t q = 1; q < ns; ++q) {
    const float f = p[(int64_t)q * kTilePx];
    p[(int64_t)q * kTilePx] = T;
    T *= f;
  }
}

__global__ __launch_bounds__(256) void k_seg_combine(const DevCamera* __restrict__ cams, int n_views, Opts o,
                                                     const uint32_t* __restrict__ nseg,
                                                     const uint32_t* __restrict__ seg_off,
                                                     const float* __restrict__ seg_prod,
                                                     const float4* __restrict__ seg_out) {
  const int t = blockIdx.x;
  const uint32_t ns = nseg[t];
  if (ns <= 1) return;
  const int v = view_of_tile(cams, n_views, t);
  const DevCamera& c = cams[v];
  int i, j;
  tile_pixel(c, t - c.tile_offset, threadIdx.x, i, j);
  if (i >= c.crop_w || j >= c.crop_h) return;
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;
  for (uint32_t q = 0; q < ns; ++q) {
    const int64_t slot = (int64_t)(seg_off[t] + q) * kTilePx + threadIdx.x;
    const float4 r = seg_out[slot];
    if (r.w < 0.f) {  // composited again from T_in by pass 2: absolute colour
      C0 += r.x;
      C1 += r.y;
      C2 += r.z;
      if (r.w >= -2.f) {  // terminated in this segment
        T = -r.w - 1.f;
        break;
      }
      T = -r.w - 3.f;
      continue;
    }
    const float T_in = q > 0 ? seg_prod[slot] : 1.f;
    C0 = fmaf(T_in, r.x, C0);
    C1 = fmaf(T_in, r.y, C1);
    C2 = fmaf(T_in, r.z, C2);
    T = T_in * r.w;
  }
  float4 out;
  out.x = C0 + T * o.bg[0];
  out.y = C1 + T * o.bg[1];
  out.z = C2 + T * o.bg[2];
  out.w = 1.f - T;
  reinterpret_cast<float4*>(c.out)[(int64_t)j * c.crop_w + i] = out;
}

template <int FILTER, bool MARGINAL, bool GEER>
static void launch_seg_passes(const DevCamera* cams, int n_views, int total_tiles, const Opts& o, const Record* rec,
                              int64_t n_gauss, const uint2* ranges, const SegPlan& sp, const uint32_t* sorted_gid,
                              const float4* pix, hipStream_t s) {
  const dim3 grid((unsigned)sp.max_segs), block(256);
  k_render_seg<FILTER, MARGINAL, GEER, 1><<<grid, block, 0, s>>>(cams, n_views, total_tiles, o, rec, n_gauss, ranges,
                                                                 sp.nseg, sp.seg_off, sp.seg_tile,
                                                                 sorted_gid, pix, sp.seg_prod, sp.seg_out);
  k_seg_prefix<<<dim3((unsigned)total_tiles), block, 0, s>>>(sp.nseg, sp.seg_off, sp.seg_prod);
  k_render_seg<FILTER, MARGINAL, GEER, 2><<<grid, block, 0, s>>>(cams, n_views, total_tiles, o, rec, n_gauss, ranges,
                                                                 sp.nseg, sp.seg_off, sp.seg_tile,
                                                                 sorted_gid, pix, sp.seg_prod, sp.seg_out);
}

hipError_t launch_render_fwd_split(const DevCamera* cams, int n_views, int total_tiles, const Opts& o,
                                   const Record* rec, int64_t n_gauss, const uint2* ranges, const SegPlan& sp,
                                   const uint32_t* sorted_gid, const float4* pix, hipStream_t s) {
  if (total_tiles == 0) return hipSuccess;
  const unsigned tb = (unsigned)((total_tiles + 255) / 256);
  k_seg_count<<<dim3(tb), dim3(256), 0, s>>>(cams, n_views, ranges, total_tiles, sp.nseg);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_exclusive_scan(sp.nseg, sp.seg_off, total_tiles, sp.scan_tmp, s);
  if (e != hipSuccess) return e;
  k_seg_fill<<<dim3(tb), dim3(256), 0, s>>>(sp.nseg, sp.seg_off, total_tiles, sp.seg_tile);
  const bool marginal = o.use_floor && o.composition == CG_COMPOSE_MARGINAL;
  const bool geer = o.backbone == CG_BACKBONE_RAY_INTEGRAL;
#define CG_SEG(F, M)                                                                                               \
  (geer ? launch_seg_passes<F, M, true>(cams, n_views, total_tiles, o, rec, n_gauss, ranges, sp, sorted_gid, pix, s) \
        : launch_seg_passes<F, M, false>(cams, n_views, total_tiles, o, rec, n_gauss, ranges, sp, sorted_gid, pix, s))
  switch (o.filter_mode) {
    case CG_FILTER_CENTER_RAY:
      CG_SEG(0, false);
      break;
    case CG_FILTER_ISOTROPIC:
      if (marginal) CG_SEG(2, true); else CG_SEG(2, false);
      break;
    default:
      if (marginal) CG_SEG(1, true); else CG_SEG(1, false);
      break;
  }
#undef CG_SEG
  k_seg_combine<<<dim3((unsigned)total_tiles), dim3(256), 0, s>>>(cams, n_views, o, sp.nseg, sp.seg_off, sp.seg_prod,
                                                                  sp.seg_out);
  return hipGetLastError();
}

template <int FILTER, bool MARGINAL, bool GEER, bool COUNT>
static void launch_key(const DevCamera* cams, int n_views, int total_tiles, const Opts& o, const Record* rec,
                       int64_t n_gauss, const uint2* ranges, const uint32_t* tile_order, const uint32_t* sorted_gid,
                       const float4* pix, float* out_rgba, float* final_T, uint32_t* n_last, unsigned long long* wmask,
                       int64_t mask_words, unsigned long long* counters, const SlotGather& sg, hipStream_t s) {
  const dim3 grid(total_tiles), block(256);
  if (wmask)
    k_render<FILTER, MARGINAL, COUNT, GEER, true><<<grid, block, 0, s>>>(
        cams, n_views, total_tiles, o, rec, n_gauss, ranges, tile_order, nullptr, pix, out_rgba, final_T, n_last,
        wmask, mask_words, counters, sg);
  else
    k_render<FILTER, MARGINAL, COUNT, GEER, false><<<grid, block, 0, s>>>(
        cams, n_views, total_tiles, o, rec, n_gauss, ranges, tile_order, sorted_gid, pix, out_rgba, final_T, n_last,
        nullptr, 0, counters, SlotGather{});
}

template <int FILTER, bool MARGINAL, bool GEER>
static hipError_t launch_t(const DevCamera* cams, int n_views, int total_tiles, const Opts& o, const Record* rec,
                           int64_t n_gauss, const uint2* ranges, const uint32_t* tile_order, const uint32_t* sorted_gid,
                           const float4* pix, const float* tlo_suffix, float* out_rgba, float* final_T,
                           uint32_t* n_last, unsigned long long* wmask, int64_t mask_words,
                           unsigned long long* counters, const SlotGather& sg, hipStream_t s) {
  const dim3 grid(total_tiles), block(256);
  if (o.order_mode == CG_ORDER_RAY) {
    if (o.count_pairs)
      k_render_ray<FILTER, MARGINAL, true, GEER><<<grid, block, 0, s>>>(
          cams, n_views, total_tiles, o, rec, n_gauss, ranges, tile_order, sorted_gid, pix, tlo_suffix, counters);
    else
      k_render_ray<FILTER, MARGINAL, false, GEER><<<grid, block, 0, s>>>(
          cams, n_views, total_tiles, o, rec, n_gauss, ranges, tile_order, sorted_gid, pix, tlo_suffix, counters);
  } else if (o.count_pairs) {
    launch_key<FILTER, MARGINAL, GEER, true>(cams, n_views, total_tiles, o, rec, n_gauss, ranges, tile_order,
                                            sorted_gid, pix, out_rgba, final_T, n_last, wmask, mask_words, counters,
                                            sg, s);
  } else {
    launch_key<FILTER, MARGINAL, GEER, false>(cams, n_views, total_tiles, o, rec, n_gauss, ranges, tile_order,
                                             sorted_gid, pix, out_rgba, final_T, n_last, wmask, mask_words, nullptr,
                                             sg, s);
  }
  return hipGetLastError();
}

template <int FILTER, bool MARGINAL>
static hipError_t launch_fm(const DevCamera* cams, int n_views, int total_tiles, const Opts& o, const Record* rec,
                            int64_t n_gauss, const uint2* ranges, const uint32_t* tile_order,
                            const uint32_t* sorted_gid, const float4* pix, const float* tlo_suffix, float* out_rgba,
                            float* final_T, uint32_t* n_last, unsigned long long* wmask, int64_t mask_words,
                            unsigned long long* counters, const SlotGather& sg, hipStream_t s) {
  if (o.backbone == CG_BACKBONE_RAY_INTEGRAL)
    return launch_t<FILTER, MARGINAL, true>(cams, n_views, total_tiles, o, rec, n_gauss, ranges, tile_order,
                                            sorted_gid, pix, tlo_suffix, out_rgba, final_T, n_last, wmask, mask_words,
                                            counters, sg, s);
  return launch_t<FILTER, MARGINAL, false>(cams, n_views, total_tiles, o, rec, n_gauss, ranges, tile_order, sorted_gid,
                                           pix, tlo_suffix, out_rgba, final_T, n_last, wmask, mask_words, counters, sg,
                                           s);
}

hipError_t launch_order_bounds(const DevCamera* cams, int n_views, int total_tiles, const Record* rec,
                               int64_t n_gauss, const uint2* ranges, const uint32_t* sorted_gid, float* tlo_suffix,
                               hipStream_t s) {
  if (total_tiles == 0) return hipSuccess;
  k_order_bounds<<<dim3(total_tiles), dim3(256), 0, s>>>(cams, n_views, rec, n_gauss, ranges, sorted_gid, tlo_suffix);
  return hipGetLastError();
}

hipError_t launch_render_fwd(const DevCamera* cams, int n_views, int total_tiles, const Opts& o, const Record* rec,
                             int64_t n_gauss, const uint2* ranges, const uint32_t* tile_order,
                             const uint32_t* sorted_gid, const float4* pix, const float* tlo_suffix, float* out_rgba,
                             float* final_T, uint32_t* n_last, unsigned long long* wmask, int64_t mask_words,
                             unsigned long long* counters, const SlotGather& sg, hipStream_t s) {
  if (total_tiles == 0) return hipSuccess;
  const bool marginal = o.use_floor && o.composition == CG_COMPOSE_MARGINAL;
#define CG_FM(F, M)                                                                                                  \
  launch_fm<F, M>(cams, n_views, total_tiles, o, rec, n_gauss, ranges, tile_order, sorted_gid, pix, tlo_suffix,     \
                  out_rgba, final_T, n_last, wmask, mask_words, counters, sg, s)
  switch (o.filter_mode) {
    case CG_FILTER_CENTER_RAY:
      return CG_FM(0, false);
    case CG_FILTER_ISOTROPIC:
      return marginal ? CG_FM(2, true) : CG_FM(2, false);
    default:
      return marginal ? CG_FM(1, true) : CG_FM(1, false);
  }
#undef CG_FM
}

}  // namespace cg
