// The forward state handed to the caller for the backward pass.
#pragma once

#include <vector>

#include "runtime.hpp"

struct cg_fwd_state {
  cg::GaussPtrs g{};
  cg::Opts opts{};
  int n_views = 0;
  std::vector<cg::DevCamera> hcams;
  cg::DevCamera* dcams = nullptr;
  int64_t total_tiles = 0, total_px = 0, P = 0;
  cg::Record* rec = nullptr;          // [views][n]
  uint32_t* counts = nullptr;         // pairs per (view, Gaussian) item
  uint32_t* offsets = nullptr;        // first gradient slot per item (slots in item order)
  uint32_t* sorted_slots = nullptr;   // gradient slot of each sorted pair
  uint32_t* sorted_gid = nullptr;     // Gaussian of each sorted pair
  uint2* ranges = nullptr;            // per tile [start, end)
  uint32_t* tile_order = nullptr;     // render launch order of the tiles (heaviest first)
  float4* pix = nullptr;              // per-pixel ray buffer (pixel_buf.hpp)
  unsigned long long* wmask = nullptr;  // per wave: pairs with some pixel at alpha >= alpha_min
  int64_t mask_words = 0;             // 64-bit words per wave bitset
  float* final_T = nullptr;           // per pixel final transmittance
  uint32_t* n_last = nullptr;         // per pixel end of its walk through the tile list
  const float* out_rgba = nullptr;    // the forward output (caller-owned)
  cg_allocator alloc{nullptr, nullptr, nullptr};
  hipStream_t stream = nullptr;
  std::vector<void*> blocks;          // scratch owned by the state
  uint32_t* bwd_mismatch = nullptr;   // per tile: the backward replay's mismatched pixels
  hipStream_t bwd_stream = nullptr;   // stream of the last backward call
  bool bwd_ran = false;               // a backward call was enqueued on this state
};

namespace cg {
// view_out: per-view output pointers (NULL: views laid out contiguously in out_rgba).
// fixed: scratch from that region instead of alloc (inference only: state_out NULL).
void run_forward(const cg_gaussians* g, const cg_camera* cams, int n_views, const cg_render_opts* opts,
                 const cg_allocator* alloc, float* out_rgba, float* const* view_out, cg_fwd_state** state_out,
                 cg_fwd_stats* stats, hipStream_t s, const FixedRegion* fixed = nullptr);
// Host-side validation and set-up shared by the entry points (capi.cpp).
void check_camera(const cg_camera& c, int idx);
DevCamera make_dev_camera(const cg_camera& c);
GaussPtrs make_gauss(const cg_gaussians& g);
Opts make_opts(const cg_render_opts& o);
template <class F>
cg_status guarded(F&& f) {
  try {
    f();
    return CG_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host out of memory");
    return CG_ERR_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return CG_ERR_STATE;
  }
}
}
