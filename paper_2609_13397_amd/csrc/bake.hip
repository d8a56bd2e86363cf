// Floor variance of Eq. 11: rho^2 = min over the views in which a Gaussian is visible
// of half the trace of the world-space footprint covariance at the pixel its mean
// projects to.  One thread per Gaussian, looping over the views (FP64 throughout; the
// neighbour rays of a continuous pixel position differ from the centre ray by
// ~1e-3 rad, so the differences are formed in double).
#include "camera_dev.hpp"

namespace cg {

__global__ void k_bake_rho2(GaussPtrs g, const DevCamera* __restrict__ cams, int n_views, float t_near,
                            float* __restrict__ rho2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int64_t n = g.n;
  double best = -1.0;
  for (int v = 0; v < n_views; ++v) {
    const DevCamera& c = cams[v];
    const double vv[3] = {(double)g.means[i] - (double)c.of[0], (double)g.means[n + i] - (double)c.of[1],
                          (double)g.means[2 * n + i] - (double)c.of[2]};
    const double t = sqrt(vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]);
    if (!(t > (double)t_near)) continue;
    const double d[3] = {vv[0] / t, vv[1] / t, vv[2] / t};
    double x, y;
    if (!cam_project(c, d, &x, &y)) continue;
    if (!(x >= 0.0 && x < c.full_w && y >= 0.0 && y < c.full_h)) continue;
    double ht = 0.0;
    bool ok = true;
    for (int a = 0; a < 2; ++a) {
      const double ox = a == 0 ? 0.5 : 0.0, oy = a == 0 ? 0.0 : 0.5;
      double di[3];
      if (!cam_unproject(c, x + ox, y + oy, di) && !cam_unproject(c, x - ox, y - oy, di)) {
        ok = false;
        break;
      }
      const double dd[3] = {di[0] - d[0], di[1] - d[1], di[2] - d[2]};
      const double along = d[0] * dd[0] + d[1] * dd[1] + d[2] * dd[2];
      for (int k = 0; k < 3; ++k) {
        const double e = t * (dd[k] - along * d[k]);
        ht += e * e;
      }
    }
    if (!ok) continue;
    ht *= (1.0 / 6.0);
    if (best < 0.0 || ht < best) best = ht;
  }
  rho2[i] = best < 0.0 ? 0.f : (float)best;
}

hipError_t launch_bake_rho2(const GaussPtrs& g, const DevCamera* cams, int n_views, float t_near, float* rho2,
                            hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  k_bake_rho2<<<dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, s>>>(g, cams, n_views, t_near, rho2);
  return hipGetLastError();
}

}  // namespace cg
