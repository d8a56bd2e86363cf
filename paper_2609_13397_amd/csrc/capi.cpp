// The C ABI: argument validation, camera set-up and the orchestration of the
// forward pipeline
//   tile cones -> group cones -> preprocess -> bin count -> scan -> (read back P)
//   -> bin emit -> radix sort on (tile, depth) -> tile ranges -> tile render.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fwd_state.hpp"

using namespace cg;

namespace {

double kb_poly(const cg_camera& c, double th) {
  const double t2 = th * th;
  return th * (1.0 + t2 * (c.k[0] + t2 * (c.k[1] + t2 * (c.k[2] + t2 * c.k[3]))));
}

}  // namespace

namespace cg {

void check_camera(const cg_camera& c, int idx) {
  const std::string w = "camera " + std::to_string(idx) + ": ";
  CG_CHECK_ARG(c.model == CG_PINHOLE || c.model == CG_FISHEYE_KB || c.model == CG_EQUIRECT, w + "unknown model");
  CG_CHECK_ARG(c.full_w > 0 && c.full_h > 0, w + "full image size must be positive");
  CG_CHECK_ARG(c.crop_w >= 0 && c.crop_h >= 0 && c.crop_x0 >= 0 && c.crop_y0 >= 0 &&
                   (int64_t)c.crop_x0 + c.crop_w <= c.full_w && (int64_t)c.crop_y0 + c.crop_h <= c.full_h,
               w + "crop window outside the image");
  for (int k = 0; k < 9; ++k) CG_CHECK_ARG(std::isfinite(c.R_c2w[k]), w + "non-finite rotation");
  for (int k = 0; k < 3; ++k) CG_CHECK_ARG(std::isfinite(c.origin[k]), w + "non-finite origin");
  if (c.model != CG_EQUIRECT) {
    CG_CHECK_ARG(std::isfinite(c.fx) && std::isfinite(c.fy) && c.fx > 0 && c.fy > 0, w + "focal lengths must be > 0");
    CG_CHECK_ARG(std::isfinite(c.cx) && std::isfinite(c.cy), w + "non-finite principal point");
  }
  if (c.model == CG_FISHEYE_KB) {
    CG_CHECK_ARG(c.theta_max > 0 && c.theta_max <= 3.14159265f, w + "theta_max must be in (0, pi]");
    for (int k = 0; k < 4; ++k) CG_CHECK_ARG(std::isfinite(c.k[k]), w + "non-finite distortion");
    // theta_d must increase on [0, theta_max] for the inverse to exist
    const int steps = 4096;
    double prev = 0.0;
    for (int s = 1; s <= steps; ++s) {
      const double th = c.theta_max * s / steps;
      const double v = kb_poly(c, th);
      CG_CHECK_ARG(v > prev, w + "Kannala-Brandt polynomial is not increasing on [0, theta_max]");
      prev = v;
    }
  }
  // rotation must be invertible
  const float* R = c.R_c2w;
  const double det = (double)R[0] * ((double)R[4] * R[8] - (double)R[5] * R[7]) -
                     (double)R[1] * ((double)R[3] * R[8] - (double)R[5] * R[6]) +
                     (double)R[2] * ((double)R[3] * R[7] - (double)R[4] * R[6]);
  CG_CHECK_ARG(std::fabs(det) > 1e-3, w + "rotation is singular");
}

}  // namespace cg

namespace {

void inv3(const double* A, double* I) {
  const double d = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                   A[2] * (A[3] * A[7] - A[4] * A[6]);
  I[0] = (A[4] * A[8] - A[5] * A[7]) / d;
  I[1] = (A[2] * A[7] - A[1] * A[8]) / d;
  I[2] = (A[1] * A[5] - A[2] * A[4]) / d;
  I[3] = (A[5] * A[6] - A[3] * A[8]) / d;
  I[4] = (A[0] * A[8] - A[2] * A[6]) / d;
  I[5] = (A[2] * A[3] - A[0] * A[5]) / d;
  I[6] = (A[3] * A[7] - A[4] * A[6]) / d;
  I[7] = (A[1] * A[6] - A[0] * A[7]) / d;
  I[8] = (A[0] * A[4] - A[1] * A[3]) / d;
}

}  // namespace

namespace cg {

DevCamera make_dev_camera(const cg_camera& c) {
  DevCamera d;
  std::memset(&d, 0, sizeof(d));
  d.model = c.model;
  d.full_w = c.full_w;
  d.full_h = c.full_h;
  d.crop_x0 = c.crop_x0;
  d.crop_y0 = c.crop_y0;
  d.crop_w = c.crop_w;
  d.crop_h = c.crop_h;
  d.tiles_x = (c.crop_w + kTile - 1) / kTile;
  d.tiles_y = (c.crop_h + kTile - 1) / kTile;
  d.groups_x = (d.tiles_x + kGroup - 1) / kGroup;
  d.groups_y = (d.tiles_y + kGroup - 1) / kGroup;
  d.fx = c.fx;
  d.fy = c.fy;
  d.cx = c.cx;
  d.cy = c.cy;
  d.inv_fx = c.model == CG_EQUIRECT ? 0.0 : 1.0 / (double)c.fx;
  d.inv_fy = c.model == CG_EQUIRECT ? 0.0 : 1.0 / (double)c.fy;
  d.inv_w = 1.0 / (double)c.full_w;
  d.inv_h = 1.0 / (double)c.full_h;
  for (int k = 0; k < 4; ++k) d.k[k] = c.k[k];
  for (int k = 0; k < 9; ++k) d.R[k] = c.R_c2w[k];
  inv3(d.R, d.Rinv);
  for (int k = 0; k < 3; ++k) {
    d.o[k] = c.origin[k];
    d.of[k] = c.origin[k];
  }
  d.theta_max = c.theta_max;
  d.thd_max = c.model == CG_FISHEYE_KB ? kb_poly(c, (double)c.theta_max) : 0.0;
  const double dphi = kPi * d.inv_w, dlam = -0.5 * kPi * d.inv_h;
  d.eq_step[0] = std::cos(dphi);
  d.eq_step[1] = std::sin(dphi);
  d.eq_step[2] = std::cos(dlam);
  d.eq_step[3] = std::sin(dlam);
  return d;
}

Opts make_opts(const cg_render_opts& o) {
  CG_CHECK_ARG(o.filter_mode >= 0 && o.filter_mode <= 2, "filter_mode must be 0, 1 or 2");
  CG_CHECK_ARG(o.composition == CG_COMPOSE_MARGINAL || o.composition == CG_COMPOSE_ADDITIVE,
               "composition must be 0 or 1");
  CG_CHECK_ARG(std::isfinite(o.alpha_min) && std::isfinite(o.alpha_max) && o.alpha_min > 0.f &&
                   o.alpha_min < o.alpha_max && o.alpha_max <= 1.f,
               "need 0 < alpha_min < alpha_max <= 1");
  CG_CHECK_ARG(std::isfinite(o.T_min) && o.T_min >= 0.f && o.T_min < 1.f, "T_min must be in [0, 1)");
  CG_CHECK_ARG(std::isfinite(o.t_near) && o.t_near >= 0.f, "t_near must be >= 0");
  CG_CHECK_ARG(std::isfinite(o.footprint_scale) && o.footprint_scale >= 0.f, "footprint_scale must be >= 0");
  CG_CHECK_ARG(o.order_mode == CG_ORDER_KEY || o.order_mode == CG_ORDER_RAY, "order_mode must be 0 or 1");
  CG_CHECK_ARG(o.backbone == CG_BACKBONE_MAX_RESPONSE || o.backbone == CG_BACKBONE_RAY_INTEGRAL,
               "backbone must be 0 or 1");
  Opts r;
  r.filter_mode = o.filter_mode;
  r.use_floor = o.use_floor ? 1 : 0;
  r.composition = o.composition;
  r.alpha_min = o.alpha_min;
  r.alpha_max = o.alpha_max;
  r.T_min = o.T_min;
  r.t_near = o.t_near;
  for (int k = 0; k < 3; ++k) r.bg[k] = o.bg[k];
  r.fs = o.footprint_scale;
  r.order_mode = o.order_mode;
  r.count_pairs = o.count_pairs ? 1 : 0;
  r.backbone = o.backbone;
  return r;
}

GaussPtrs make_gauss(const cg_gaussians& g) {
  CG_CHECK_ARG(g.n >= 0, "negative Gaussian count");
  CG_CHECK_ARG(g.color_mode == 0 || g.color_mode == 3, "color_mode must be 0 (rgb) or 3 (SH degree 3)");
  if (g.n > 0)
    CG_CHECK_ARG(g.means && g.log_scales && g.quats && g.opacity_logits && g.color,
                 "null Gaussian parameter pointer");
  GaussPtrs p;
  p.n = g.n;
  p.color_mode = g.color_mode;
  p.means = g.means;
  p.log_scales = g.log_scales;
  p.quats = g.quats;
  p.logits = g.opacity_logits;
  p.color = g.color;
  p.rho2 = g.rho2;
  return p;
}

}  // namespace cg

namespace {

int bits_for(int64_t v) {
  int b = 0;
  while (b < 63 && (int64_t(1) << b) <= v) ++b;
  return b;
}

// A pinned host word per thread for the pair count's read-back (a copy into pageable
// memory would not return before it completed); freed when the thread ends.
struct PinnedWord {
  unsigned long long* p = nullptr;
  ~PinnedWord() {
    if (p) (void)hipHostFree(p);
  }
};

unsigned long long* host_word() {
  thread_local PinnedWord w;
  if (!w.p) {
    void* p = nullptr;
    CG_HIP(hipHostMalloc(&p, 64, hipHostMallocPortable));
    w.p = static_cast<unsigned long long*>(p);
  }
  return w.p;
}

// An event the host waits on: the pair count's copy, not the work queued after it.  A
// call that leaves early (an error) still waits for the copy before it returns, so that
// it cannot land in the thread's pinned word during a later call on another stream.
struct ReadEvent {
  hipEvent_t e = nullptr;
  ReadEvent() { CG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming)); }
  ~ReadEvent() {
    if (e) {
      (void)hipEventSynchronize(e);
      (void)hipEventDestroy(e);
    }
  }
  ReadEvent(const ReadEvent&) = delete;
  ReadEvent& operator=(const ReadEvent&) = delete;
};

// The shape of a forward call and its pair count (-1: none), per thread.
struct CallShape {
  int64_t n = -1;
  int n_views = 0;
  int64_t total_tiles = 0, total_px = 0;
  bool train = false;
  int64_t pairs = -1;
  bool same(const CallShape& o) const {
    return n == o.n && n_views == o.n_views && total_tiles == o.total_tiles && total_px == o.total_px &&
           train == o.train;
  }
};

CallShape& last_call_shape() {
  thread_local CallShape s;
  return s;
}

}  // namespace

// ---------------------------------------------------------------------------- forward

namespace cg {

// Pair indices, offsets and the radix sort's element counts are 32-bit.
void check_pair_total(uint64_t total) {
  CG_CHECK_ARG(total < kMaxPairs, "too many (tile, Gaussian) pairs for 32-bit indices: " + std::to_string(total));
}

void run_forward(const cg_gaussians* g_in, const cg_camera* cams, int n_views, const cg_render_opts* opts_in,
                 const cg_allocator* alloc, float* out_rgba, float* const* view_out, cg_fwd_state** state_out,
                 cg_fwd_stats* stats, hipStream_t s, const FixedRegion* fixed) {
  CG_CHECK_ARG(g_in && cams && opts_in, "null argument");
  CG_CHECK_ARG(!(fixed && state_out), "a fixed scratch region serves inference calls only");
  CG_CHECK_ARG(n_views >= 1 && n_views <= 4096, "n_views must be in [1, 4096]");
  const GaussPtrs g = make_gauss(*g_in);
  const Opts o = make_opts(*opts_in);
  if (o.order_mode == CG_ORDER_RAY && state_out)
    throw Error(CG_ERR_UNSUPPORTED, "order_mode RAY is forward-only: pass state_out = NULL");
  std::vector<DevCamera> hc(n_views);
  int64_t total_tiles = 0, total_groups = 0, total_px = 0;
  for (int v = 0; v < n_views; ++v) {
    check_camera(cams[v], v);
    hc[v] = make_dev_camera(cams[v]);
    hc[v].tile_offset = (int32_t)total_tiles;
    hc[v].group_offset = (int32_t)total_groups;
    hc[v].px_offset = total_px;
    hc[v].out = view_out ? view_out[v] : (out_rgba ? out_rgba + 4 * total_px : nullptr);
    CG_CHECK_ARG(hc[v].out || (int64_t)cams[v].crop_w * cams[v].crop_h == 0, "null output for a non-empty view");
    CG_CHECK_ARG((int64_t)hc[v].groups_x * hc[v].groups_y <= 65535, "view too large (more than 65535 tile groups)");
    total_tiles += (int64_t)hc[v].tiles_x * hc[v].tiles_y;
    total_groups += (int64_t)hc[v].groups_x * hc[v].groups_y;
    total_px += (int64_t)cams[v].crop_w * cams[v].crop_h;
  }
  CG_CHECK_ARG(total_tiles < (int64_t(1) << 31) / 8 - 8, "too many tiles");

  const int64_t n = g.n;
  const int64_t nv = n * n_views;
  CG_CHECK_ARG(nv < (int64_t(1) << 31), "n * n_views must be below 2^31");

  Scratch sc(alloc, s, fixed);
  cg_fwd_state* st = nullptr;
  if (state_out) {
    st = new cg_fwd_state();
    st->alloc = sc.allocator();
    st->stream = s;
  }
  try {
    // phase 1 (sizes known up front): per view, tile, pixel and (view, Gaussian) item
    const int64_t nv1 = std::max<int64_t>(nv, 1);
    DevCamera* dcams;
    TileCone* tiles;
    float4 *groups, *members, *pix, *cone;
    uint32_t *depth_key, *counts, *offsets, *items, *items_alt, *counts_sorted, *offs_sorted;
    float* view_cmax;
    unsigned long long* pair_total;
    Record* rec;
    uint32_t* dkeys_alt;
    void *scan_tmp, *dsort_tmp;
    uint8_t* hit_n;
    uint16_t* hit_list;
    uint32_t* slot_offs = nullptr;  // training: first gradient slot per item, in item order
    {
      Carve c;
      c.add(&dcams, n_views);
      c.add(&tiles, total_tiles);
      c.add(&groups, total_groups);
      c.add(&members, total_groups * kGroupTiles);
      c.add(&view_cmax, n_views);
      c.add(&pair_total, 1);
      c.add(&pix, std::max<int64_t>(total_tiles, 1) * kTilePx * 4);
      c.add(&rec, nv1);
      c.add(&depth_key, nv1);
      c.add(&cone, nv1);
      c.add(&counts, nv1);
      c.add(&hit_n, nv1);
      if (state_out) {
        c.add(&slot_offs, nv1);
        c.add(&st->bwd_mismatch, std::max<int64_t>(total_tiles, 1));
      }
      c.add(&hit_list, nv1 * kBinHitList);
      c.add(&offsets, nv1);
      c.add_bytes(&scan_tmp, scan_temp_bytes(nv));
      c.add(&dkeys_alt, nv1);
      c.add(&items, nv1);
      c.add(&items_alt, nv1);
      c.add(&counts_sorted, nv1);
      c.add(&offs_sorted, nv1);
      c.add_bytes(&dsort_tmp, radix_temp_bytes(nv));
      sc.get(c);
    }
    CG_HIP(hipMemcpyAsync(dcams, hc.data(), sizeof(DevCamera) * n_views, hipMemcpyHostToDevice, s));

    {
      ProfScope ps(ST_CAMERA, s);
      const ClearPair clr{{reinterpret_cast<uint32_t*>(view_cmax), reinterpret_cast<uint32_t*>(pair_total)},
                          {n_views, 2}};
      CG_HIP(launch_tile_cones(dcams, n_views, (int)total_tiles, o.fs, tiles, pix, clr, s));
      CG_HIP(launch_group_cones(dcams, n_views, (int)total_groups, tiles, groups, members,
                                view_cmax, s));
    }
    {
      ProfScope ps(ST_PREPROCESS, s);
      CG_HIP(launch_preprocess(g, dcams, n_views, view_cmax, o, rec, depth_key, items, cone, s));
    }
    {
      ProfScope ps(ST_BIN_COUNT, s);
      CG_HIP(launch_bin_count(n, n_views, dcams, cone, groups, members, counts, hit_n, hit_list, s));
    }
    // compositing order of the (view, Gaussian) items, then pair offsets in that order.
    // The items of all views are sorted together, stably, on the float32 depth key
    // alone (it is consumed here): a tile holds pairs of one view only, so each tile's
    // list comes out in its view's depth order, equal keys in Gaussian index order,
    // whatever the order between views.
    const uint32_t* sorted_items = items;
    if (nv > 0) {
      int d_alt = 0;
      {
        ProfScope ps(ST_DEPTH_SORT, s);
        CG_HIP(launch_radix_sort32(depth_key, items, dkeys_alt, items_alt, nv, 32, dsort_tmp, &d_alt, s));
      }
      sorted_items = d_alt ? items_alt : items;
      {
        ProfScope ps(ST_SCAN, s);
        CG_HIP(launch_permuted_scan(counts, sorted_items, nv, counts_sorted, offs_sorted, offsets, pair_total, scan_tmp,
                                    s));
        // training: the pairs' gradient slots are laid out item by item (each item's
        // slots contiguous, items in index order), so that the backward's per-item sums
        // read and write in one front-to-back sweep
        if (slot_offs) CG_HIP(launch_exclusive_scan(counts, slot_offs, nv, scan_tmp, s));
      }
      CG_HIP(hipMemcpyAsync(host_word(), pair_total, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    }
    ReadEvent ev;
    CG_HIP(hipEventRecord(ev.e, s));

    // phase 2 (sizes from the pair count): pairs emitted in compositing order, then
    // sorted stably by tile, per-tile ranges and the render's state
    const bool ray_order = o.order_mode == CG_ORDER_RAY;
    // long lists on views with few tiles: each such view's longest list and pair count,
    // read back after the tile sort, decide whether its lists are cut into segments on
    // separate workgroups (per view, so that a view renders the same alone or fused)
    const SplitPolicy pol = split_policy();
    bool small_views = false;
    for (int v = 0; v < n_views; ++v) {
      const int64_t tv = (int64_t)hc[v].tiles_x * hc[v].tiles_y;
      small_views = small_views || (tv > 0 && tv < pol.max_tiles);
    }
    const bool split_candidate = !st && !opts_in->count_pairs && !ray_order && small_views;
    uint32_t *keys, *vals, *keys_alt, *vals_alt, *tile_order;
    uint32_t *slot_gid = nullptr, *sorted_gid_buf = nullptr, *n_last = nullptr;
    uint2* ranges;
    void* sort_tmp;
    unsigned long long *wmask = nullptr, *counters = nullptr;
    float *final_T = nullptr, *tlo_suffix = nullptr;
    uint32_t* view_stats = nullptr;
    // training: per wave, the pairs at which some pixel had alpha >= alpha_min (4 waves
    // per tile; two words of slack so the backward can read the word after a batch)
    int64_t mask_words = 0, cap = -1;
    // the phase-2 block for up to `pairs` pairs
    auto carve_phase2 = [&](int64_t pairs) {
      const int64_t P1 = std::max<int64_t>(pairs, 1);
      cap = pairs;
      mask_words = pairs / 64 + 2;
      Carve c;
      c.add(&keys, P1);
      c.add(&vals, P1);
      c.add(&keys_alt, P1);
      c.add(&vals_alt, P1);
      c.add(&ranges, std::max<int64_t>(total_tiles, 1));
      c.add(&tile_order, std::max<int64_t>(total_tiles, 1));
      c.add_bytes(&sort_tmp, radix_temp_bytes(pairs));
      if (st) {
        c.add(&slot_gid, P1);
        c.add(&sorted_gid_buf, P1);
        c.add(&wmask, 4 * mask_words);
        c.add(&final_T, std::max<int64_t>(total_px, 1));
        c.add(&n_last, std::max<int64_t>(total_px, 1));
      }
      // counters [0..2]: pair counts (count_pairs); [3]: early composites (order_mode RAY)
      if (opts_in->count_pairs || ray_order) c.add(&counters, 4);
      if (ray_order) c.add(&tlo_suffix, P1);
      if (split_candidate) c.add(&view_stats, 2 * (int64_t)n_views);
      sc.get(c);
    };
    auto emit = [&]() {
      ProfScope ps(ST_BIN_EMIT, s);
      CG_HIP(launch_bin_emit(n, n_views, dcams, cone, groups, members, offsets, slot_offs, keys, vals, slot_gid,
                             hit_n, hit_list, ranges, total_tiles, cap, s));
    };
    // A call shaped like this thread's previous one (same Gaussian count, views, tiles
    // and pixels, and both training or both not: a render or training loop) sizes
    // phase 2 from that call's pair count, with a margin, and queues the emit pass
    // before it waits for its own count: the GPU emits while the host reads the count
    // back.  If the count exceeds the guess, the emit dropped the pairs past it; the
    // block is carved again and the pass queued again.  Calls on a fixed scratch region
    // do not guess.
    const CallShape shape{n, n_views, total_tiles, total_px, st != nullptr, -1};
    CallShape& last = last_call_shape();
    const bool guess = !fixed && nv > 0 && last.pairs >= 0 && last.same(shape);
    if (guess) {
      carve_phase2(last.pairs + last.pairs / 16 + 4096);
      emit();
    }
    CG_HIP(hipEventSynchronize(ev.e));
    const unsigned long long host_total = nv > 0 ? *host_word() : 0ull;
    last.pairs = -1;  // (a failing call leaves no guess behind)
    // the exact 64-bit total: below the limit, the 32-bit offsets of the scan did not wrap
    check_pair_total(host_total);
    const int64_t P = (int64_t)host_total;
    if (!guess || P > cap) {
      if (guess) sc.release_last();
      carve_phase2(P);
      if (P > 0) emit();
    }
    last = shape;
    last.pairs = P;
    const bool may_split = split_candidate && P > 0;

    const int tile_bits = bits_for(std::max<int64_t>(total_tiles - 1, 1));
    int in_alt = 0;
    if (P > 0) {
      {
        ProfScope ps(ST_SORT, s);
        CG_HIP(launch_radix_sort32(keys, vals, keys_alt, vals_alt, P, tile_bits, sort_tmp, &in_alt, s));
      }
    }
    uint32_t* skeys = in_alt ? keys_alt : keys;
    uint32_t* svals = in_alt ? vals_alt : vals;
    // inference: the sorted values are the Gaussian indices; training: emission slots
    uint32_t* sorted_gid = st ? sorted_gid_buf : svals;
    uint32_t* sslots = st ? svals : nullptr;
    const int end_bit = tile_bits;
    {
      ProfScope ps(ST_RANGES, s);
      // (the emit pass zeroed the ranges; with no pairs it did not run)
      if (P == 0) CG_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, 2 * total_tiles, s));
      // training: each sorted pair's Gaussian is found through the slot table by the
      // forward render when it stages the pair (it walks only the pairs before its
      // tiles' termination, and its other loads hide the gather)
      CG_HIP(launch_tile_ranges(skeys, P, ranges, s));
      CG_HIP(launch_tile_order(ranges, (int)total_tiles, tile_order, s));
    }
    int64_t max_tile_pairs = -1;
    int n_split = 0;
    SegPlan sp{};
    if (may_split) {
      std::vector<uint32_t> vs(2 * (size_t)n_views);
      CG_HIP(launch_view_stats(dcams, n_views, ranges, pol.max_tiles, view_stats, s));
      CG_HIP(hipMemcpyAsync(vs.data(), view_stats, sizeof(uint32_t) * vs.size(), hipMemcpyDeviceToHost, s));
      CG_HIP(hipStreamSynchronize(s));
      for (int v = 0; v < n_views; ++v) {
        const int64_t tv = (int64_t)hc[v].tiles_x * hc[v].tiles_y, longest = vs[2 * v], pv = vs[2 * v + 1];
        if (tv == 0 || tv >= pol.max_tiles) continue;
        max_tile_pairs = std::max(max_tile_pairs, longest);
        if (!split_wins(pol, longest, pv)) continue;
        int64_t L = pol.seg_len > 0 ? pol.seg_len : std::max<int64_t>(kMinSegLen, (pv + kSegTarget - 1) / kSegTarget);
        L = std::min<int64_t>(L, int64_t(1) << 30);
        hc[v].seg_len = (uint32_t)L;
        sp.max_segs += tv + (pv + L - 1) / L;
        ++n_split;
      }
    }
    const bool split = n_split > 0;
    if (split) {
      CG_CHECK_ARG(sp.max_segs < (int64_t(1) << 31), "too many tile segments");
      // the split views' segment lengths, for the render kernels
      CG_HIP(hipMemcpyAsync(dcams, hc.data(), sizeof(DevCamera) * n_views, hipMemcpyHostToDevice, s));
      // phase 3: the split render's per-segment state
      Carve c;
      c.add(&sp.nseg, total_tiles);
      c.add(&sp.seg_off, total_tiles);
      c.add(&sp.seg_tile, sp.max_segs);
      c.add(&sp.seg_prod, sp.max_segs * kTilePx);
      c.add(&sp.seg_out, sp.max_segs * kTilePx);
      c.add_bytes(&sp.scan_tmp, scan_temp_bytes(total_tiles));
      sc.get(c);
    }
    if (counters) CG_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(counters), 0u, 8, s));
    if (ray_order && P > 0) {
      ProfScope ps(ST_RANGES, s);
      CG_HIP(launch_order_bounds(dcams, n_views, (int)total_tiles, rec, n, ranges, sorted_gid, tlo_suffix, s));
    }
    {
      ProfScope ps(ST_RENDER, s);
      if (wmask) CG_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(wmask), 0u, 8 * mask_words, s));
      if (split)
        CG_HIP(launch_render_fwd_split(dcams, n_views, (int)total_tiles, o, rec, n, ranges, sp, sorted_gid, pix, s));
      // the views rendered in whole tiles (the kernel skips the split views' tiles)
      if (n_split < n_views)
        CG_HIP(launch_render_fwd(dcams, n_views, (int)total_tiles, o, rec, n, ranges, tile_order, sorted_gid, pix,
                                 tlo_suffix, out_rgba, final_T, n_last, wmask, mask_words, counters,
                                 st ? SlotGather{svals, slot_gid, sorted_gid_buf} : SlotGather{}, s));
    }
    unsigned long long host_counters[4] = {~0ull, ~0ull, ~0ull, ~0ull};
    if (counters && (opts_in->count_pairs || stats)) {
      CG_HIP(hipMemcpyAsync(host_counters, counters, sizeof(host_counters), hipMemcpyDeviceToHost, s));
      CG_HIP(hipStreamSynchronize(s));
    }
    if (!opts_in->count_pairs) host_counters[0] = host_counters[1] = host_counters[2] = ~0ull;
    if (stats) {
      stats->n_evaluated = (int64_t)host_counters[0];
      stats->n_full = (int64_t)host_counters[1];
      stats->n_contrib = (int64_t)host_counters[2];
      stats->n_order_overflow = ray_order ? (int64_t)host_counters[3] : -1;
      stats->n_pairs = P;
      stats->n_tiles = total_tiles;
      stats->n_pixels = total_px;
      stats->n_gaussian_views = nv;
      stats->sort_bits = end_bit;
      stats->n_segments = split ? (int32_t)sp.max_segs : 0;
      stats->max_tile_pairs = max_tile_pairs;
    }
    sc.check_guards();
    if (st) {
      st->g = g;
      st->opts = o;
      st->n_views = n_views;
      st->hcams = hc;
      st->dcams = dcams;
      st->total_tiles = total_tiles;
      st->total_px = total_px;
      st->P = P;
      st->rec = rec;
      st->counts = counts;
      st->offsets = slot_offs;
      st->sorted_slots = sslots;
      st->sorted_gid = sorted_gid;
      st->ranges = ranges;
      st->tile_order = tile_order;
      st->pix = pix;
      st->wmask = wmask;
      st->mask_words = mask_words;
      st->final_T = final_T;
      st->n_last = n_last;
      st->out_rgba = out_rgba;
      sc.transfer(st->blocks);
      *state_out = st;
    }
  } catch (...) {
    if (st) {
      sc.transfer(st->blocks);
      cg_fwd_state_release(st);
    }
    throw;
  }
}

}  // namespace cg

// ---------------------------------------------------------------------------- C entry points

extern "C" {

int cg_version(void) { return CG_VERSION; }

void cg_default_opts(cg_render_opts* o) {
  if (!o) return;
  o->filter_mode = CG_FILTER_ANISOTROPIC;
  o->use_floor = 0;
  o->composition = CG_COMPOSE_MARGINAL;
  o->alpha_min = 1.0f / 255.0f;
  o->alpha_max = 0.99f;
  o->T_min = 1e-4f;
  o->t_near = 0.2f;
  o->bg[0] = o->bg[1] = o->bg[2] = 0.f;
  o->footprint_scale = 1.f;
  o->count_pairs = 0;
  o->order_mode = CG_ORDER_KEY;
  o->backbone = CG_BACKBONE_MAX_RESPONSE;
}

cg_status cg_render_forward(const cg_gaussians* g, const cg_camera* cams, int32_t n_views,
                            const cg_render_opts* opts, const cg_allocator* alloc, float* out_rgba,
                            cg_fwd_state** state_out, cg_fwd_stats* stats_out, hipStream_t stream) {
  if (state_out) *state_out = nullptr;
  return guarded([&] { run_forward(g, cams, n_views, opts, alloc, out_rgba, nullptr, state_out, stats_out, stream); });
}

void cg_fwd_state_release(cg_fwd_state* st) {
  if (!st) return;
  // the blocks go back in the order of the forward's stream; a backward enqueued on
  // another stream may still read them
  if (st->bwd_ran && st->bwd_stream != st->stream) (void)hipStreamSynchronize(st->bwd_stream);
  for (void* p : st->blocks) free_block(st->alloc, p, st->stream);
  delete st;
}

cg_status cg_camera_unproject(const cg_camera* cam, int64_t n, const float* pix_xy, float* dirs, uint8_t* valid,
                              hipStream_t stream) {
  return guarded([&] {
    CG_CHECK_ARG(cam, "null camera");
    CG_CHECK_ARG(n >= 0, "negative count");
    check_camera(*cam, 0);
    if (n == 0) return;
    CG_CHECK_ARG(pix_xy && dirs && valid, "null array");
    const DevCamera hc = make_dev_camera(*cam);
    Scratch sc(nullptr, stream);
    DevCamera* dc = sc.get_n<DevCamera>(1);
    CG_HIP(hipMemcpyAsync(dc, &hc, sizeof(hc), hipMemcpyHostToDevice, stream));
    {
      ProfScope ps(ST_CAMERA, stream);
      CG_HIP(launch_unproject(dc, n, pix_xy, dirs, valid, stream));
    }
    // keep the host copy alive until the upload has happened
    CG_HIP(hipStreamSynchronize(stream));
  });
}

cg_status cg_bake_rho2(const cg_gaussians* g, const cg_camera* cams, int32_t n_views, float t_near, float* rho2_out,
                       hipStream_t stream) {
  return guarded([&] {
    CG_CHECK_ARG(g && cams, "null argument");
    CG_CHECK_ARG(n_views >= 1, "need at least one view");
    CG_CHECK_ARG(std::isfinite(t_near) && t_near >= 0.f, "t_near must be >= 0");
    const GaussPtrs gp = make_gauss(*g);
    if (gp.n == 0) return;
    CG_CHECK_ARG(rho2_out, "null output");
    std::vector<DevCamera> hc(n_views);
    for (int v = 0; v < n_views; ++v) {
      check_camera(cams[v], v);
      hc[v] = make_dev_camera(cams[v]);
    }
    Scratch sc(nullptr, stream);
    DevCamera* dc = sc.get_n<DevCamera>(n_views);
    CG_HIP(hipMemcpyAsync(dc, hc.data(), sizeof(DevCamera) * n_views, hipMemcpyHostToDevice, stream));
    {
      ProfScope ps(ST_BAKE, stream);
      CG_HIP(launch_bake_rho2(gp, dc, n_views, t_near, rho2_out, stream));
    }
    CG_HIP(hipStreamSynchronize(stream));
  });
}

}  // extern "C"
