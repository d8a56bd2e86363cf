// cg_render_forward_noalloc: the inference forward render with every scratch buffer
// (per-view cameras, tile cones, the pixel ray buffer, per-Gaussian records, keys,
// pair lists, sort buffers) carved from one file-scope device array instead of an
// allocator, for callers that cannot allocate device memory.
#include <mutex>

#include "fwd_state.hpp"

namespace {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;  // 64 MiB per GPU

}  // namespace

// Each GPU the library runs on holds its own copy until the process ends.  In host
// code `scratch` names a host-side stand-in: kernels get its device address, looked up
// once per device with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device (null until looked up)

// The current device's copy of `scratch`, looked up with that device current.
void* device_scratch() {
  int dev = 0;
  CG_HIP(hipGetDevice(&dev));
  CG_CHECK_ARG(dev >= 0 && dev < kMaxDevices, "device index beyond the no-alloc entry point's table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    CG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    CG_CHECK_ARG(p != nullptr, "no device address for the no-alloc scratch array");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" cg_status cg_render_forward_noalloc(const cg_gaussians* g, const cg_camera* cams, int32_t n_views,
                                               const cg_render_opts* opts, float* out_rgba,
                                               cg_fwd_stats* stats_out, hipStream_t stream) {
  return cg::guarded([&] {
    const cg::FixedRegion region{device_scratch(), kNoAllocScratchBytes};
    cg::run_forward(g, cams, n_views, opts, nullptr, out_rgba, nullptr, nullptr, stats_out, stream, &region);
  });
}
