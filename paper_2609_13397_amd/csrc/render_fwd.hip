// Tile render: one 256-thread workgroup per 16x16 tile, one pixel per thread.  The
// tile's depth-sorted list of Gaussians is walked in batches of 256 records staged
// in LDS; every pixel evaluates the filtered closed-form response of Eq. 9 (with the
// marginal floor composition of Eq. 12) and composites front to back (Eq. 4).  The
// workgroup stops fetching batches once every pixel has terminated.
#include "pair_math.hpp"

namespace cg {

// COUNT: also count, per pixel, the pairs walked through, those that needed the full
// footprint arithmetic and those composited, and add them to counters[0..2].
template <int FILTER, bool MARGINAL, bool COUNT>
__global__ __launch_bounds__(256) void k_render(const DevCamera* __restrict__ cams, int n_views, int total_tiles,
                                                int per_xcd, Opts o, const Record* __restrict__ rec, int64_t n_gauss,
                                                const uint2* __restrict__ ranges,
                                                const uint32_t* __restrict__ sorted_gid, float* __restrict__ out_rgba,
                                                float* __restrict__ final_T, uint32_t* __restrict__ n_last,
                                                unsigned long long* __restrict__ counters) {
  __shared__ Record srec[256];
  __shared__ unsigned int scount[3];
  uint32_t c_eval = 0, c_full = 0, c_contrib = 0;
  // Workgroup b is dispatched to XCD b % 8: hand each XCD a contiguous band of tiles,
  // so neighbouring tiles (which share most of their Gaussians) share one L2.
  const int b = blockIdx.x;
  const int t = (b & 7) * per_xcd + (b >> 3);
  if (t >= total_tiles) return;
  const int v = view_of_tile(cams, n_views, t);
  const DevCamera& c = cams[v];
  const int lt = t - c.tile_offset;
  const int tx = lt % c.tiles_x, ty = lt / c.tiles_x;
  const int i = tx * kTile + (threadIdx.x & (kTile - 1));
  const int j = ty * kTile + (threadIdx.x / kTile);
  const bool inside = i < c.crop_w && j < c.crop_h;
  PixelRay r;
  r.valid = false;
  if (inside) r = pixel_ray(c, i, j, o.fs);
  const PairPixel px = make_pair_pixel(r, c);

  const uint2 rg = ranges[t];
  float Ttr = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  bool done = !r.valid;
  uint32_t last = rg.x;
  const Record* vrec = rec + (int64_t)v * n_gauss;
  for (uint32_t base = rg.x; base < rg.y; base += 256) {
    if (__syncthreads_count(!done) == 0) break;
    const uint32_t idx = base + threadIdx.x;
    if (idx < rg.y) srec[threadIdx.x] = vrec[sorted_gid[idx]];
    __syncthreads();
    const int cnt = (int)min(256u, rg.y - base);
    if (!done) {
      int k = 0;
      for (; k < cnt; ++k) {
        float T;
        if (COUNT) ++c_eval;
        if (!pair_response<FILTER, MARGINAL>(srec[k], px, o, T)) continue;
        if (COUNT) ++c_full;
        const float alpha = fminf(T, o.alpha_max);
        if (alpha < o.alpha_min) continue;
        const float test = Ttr * (1.f - alpha);
        if (test < o.T_min) {
          done = true;
          break;
        }
        if (COUNT) ++c_contrib;
        const float w = Ttr * alpha;
        C0 = fmaf(w, srec[k].rgb[0], C0);
        C1 = fmaf(w, srec[k].rgb[1], C1);
        C2 = fmaf(w, srec[k].rgb[2], C2);
        Ttr = test;
      }
      last = base + (uint32_t)k;
    }
    __syncthreads();
  }
  if (inside) {
    const int64_t p = c.px_offset + (int64_t)j * c.crop_w + i;
    float4 out;
    out.x = C0 + Ttr * o.bg[0];
    out.y = C1 + Ttr * o.bg[1];
    out.z = C2 + Ttr * o.bg[2];
    out.w = 1.f - Ttr;
    reinterpret_cast<float4*>(out_rgba)[p] = out;
    if (final_T) final_T[p] = Ttr;
    if (n_last) n_last[p] = last;
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

template <int FILTER, bool MARGINAL>
static hipError_t launch_t(const DevCamera* cams, int n_views, int total_tiles, const Opts& o, const Record* rec,
                           int64_t n_gauss, const uint2* ranges, const uint32_t* sorted_gid, float* out_rgba,
                           float* final_T, uint32_t* n_last, unsigned long long* counters, hipStream_t s) {
  const int per_xcd = (total_tiles + 7) / 8;
  if (counters)
    k_render<FILTER, MARGINAL, true><<<dim3(per_xcd * 8), dim3(256), 0, s>>>(
        cams, n_views, total_tiles, per_xcd, o, rec, n_gauss, ranges, sorted_gid, out_rgba, final_T, n_last,
        counters);
  else
    k_render<FILTER, MARGINAL, false><<<dim3(per_xcd * 8), dim3(256), 0, s>>>(
        cams, n_views, total_tiles, per_xcd, o, rec, n_gauss, ranges, sorted_gid, out_rgba, final_T, n_last,
        nullptr);
  return hipGetLastError();
}

hipError_t launch_render_fwd(const DevCamera* cams, int n_views, int total_tiles, const Opts& o, const Record* rec,
                             int64_t n_gauss, const uint2* ranges, const uint32_t* sorted_gid, float* out_rgba,
                             float* final_T, uint32_t* n_last, unsigned long long* counters, hipStream_t s) {
  if (total_tiles == 0) return hipSuccess;
  const bool marginal = o.use_floor && o.composition == CG_COMPOSE_MARGINAL;
  switch (o.filter_mode) {
    case CG_FILTER_CENTER_RAY:
      return launch_t<0, false>(cams, n_views, total_tiles, o, rec, n_gauss, ranges, sorted_gid, out_rgba, final_T,
                                n_last, counters, s);
    case CG_FILTER_ISOTROPIC:
      return marginal ? launch_t<2, true>(cams, n_views, total_tiles, o, rec, n_gauss, ranges, sorted_gid, out_rgba,
                                          final_T, n_last, counters, s)
                      : launch_t<2, false>(cams, n_views, total_tiles, o, rec, n_gauss, ranges, sorted_gid, out_rgba,
                                           final_T, n_last, counters, s);
    default:
      return marginal ? launch_t<1, true>(cams, n_views, total_tiles, o, rec, n_gauss, ranges, sorted_gid, out_rgba,
                                          final_T, n_last, counters, s)
                      : launch_t<1, false>(cams, n_views, total_tiles, o, rec, n_gauss, ranges, sorted_gid, out_rgba,
                                           final_T, n_last, counters, s);
  }
}

}  // namespace cg
