// Backward pass (placeholder until the kernels land).
#include "fwd_state.hpp"

extern "C" cg_status cg_render_backward(cg_fwd_state* st, const float* grad_rgba, float* d_means,
                                        float* d_log_scales, float* d_quats, float* d_opacity_logits, float* d_color,
                                        hipStream_t stream) {
  (void)st; (void)grad_rgba; (void)d_means; (void)d_log_scales; (void)d_quats; (void)d_opacity_logits;
  (void)d_color; (void)stream;
  cg::set_last_error("backward not built yet");
  return CG_ERR_UNSUPPORTED;
}
