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
  uint32_t* counts = nullptr;         // pairs per (view, Gaussian)
  uint32_t* offsets = nullptr;        // first emission slot per (view, Gaussian)
  uint32_t* sorted_slots = nullptr;   // emission slot of each sorted pair
  uint32_t* sorted_gid = nullptr;     // Gaussian of each sorted pair
  uint2* ranges = nullptr;            // per tile [start, end)
  float* final_T = nullptr;           // per pixel final transmittance
  uint32_t* n_last = nullptr;         // per pixel end of its walk through the tile list
  const float* out_rgba = nullptr;    // the forward output (caller-owned)
  cg_allocator alloc{nullptr, nullptr, nullptr};
  hipStream_t stream = nullptr;
  std::vector<void*> blocks;          // scratch owned by the state
  int64_t replay_mismatches = -1;     // set by the backward pass
};

namespace cg {
void run_forward(const cg_gaussians* g, const cg_camera* cams, int n_views, const cg_render_opts* opts,
                 const cg_allocator* alloc, float* out_rgba, cg_fwd_state** state_out, cg_fwd_stats* stats,
                 hipStream_t s);
}
