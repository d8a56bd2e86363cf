// Per (view, Gaussian) preprocessing: activations (Sec. 3), the floor of Eq. 10,
// whitening W = diag(1/s') R^T (Eq. 1 with Sigma_eff), view-dependent colour, the
// float32 compositing key and the angular influence cone used by the binning.
#include "camera_dev.hpp"
#include "sh.hpp"

namespace cg {

// |mu - o|^2 in float32 with the operation order ((vx*vx + vy*vy) + vz*vz) and no
// fused multiply-add: the compositing key, identical on every platform that rounds
// float32 to nearest.
__device__ __noinline__ float depth_key_f32(float mx, float my, float mz, float ox, float oy, float oz) {
#pragma clang fp contract(off)
  const float vx = mx - ox;
  const float vy = my - oy;
  const float vz = mz - oz;
  const float sx = vx * vx;
  const float sy = vy * vy;
  const float sz = vz * vz;
  float s = sx + sy;
  s = s + sz;
  return s;
}

constexpr int kRecF4 = (int)(sizeof(Record) / sizeof(float4));  // 8
static_assert(sizeof(Record) % sizeof(float4) == 0, "Record is a whole number of 16-byte pieces");

// Block order: workgroup b runs on XCD b % 8.  The views of one 256-Gaussian chunk are
// given to workgroups b, b + 8, b + 16, ... (same XCD, consecutive in dispatch order),
// so the views after the first read the chunk's parameters (48 SH coefficients each)
// from that XCD's L2 instead of HBM.
__global__ __launch_bounds__(256) void k_preprocess(GaussPtrs g, const DevCamera* __restrict__ cams, int n_views,
                                                    const float* __restrict__ view_cmax, Opts o,
                                                    Record* __restrict__ rec, uint32_t* __restrict__ depth_key,
                                                    uint32_t* __restrict__ items, float4* __restrict__ cone) {
  __shared__ float4 s_rec[4][64 * (kRecF4 + 1)];  // per wave: 64 records, padded against bank conflicts
  const int q8 = (int)(blockIdx.x >> 3);
  const int v = q8 % n_views;
  const int64_t chunk = (int64_t)(q8 / n_views) * 8 + (blockIdx.x & 7);
  const int64_t n = g.n;
  const int64_t i0 = chunk * blockDim.x + threadIdx.x;
  const bool live = i0 < n;
  if (__ballot(live) == 0) return;  // the whole wave is past the end
  // lanes past the end (in the last wave) recompute the last item, and write nothing
  const int64_t i = live ? i0 : n - 1;
  const DevCamera& c = cams[v];
  const int64_t out = (int64_t)v * n + i;

  const float mu[3] = {g.means[i], g.means[n + i], g.means[2 * n + i]};
  float q[4] = {g.quats[i], g.quats[n + i], g.quats[2 * n + i], g.quats[3 * n + i]};
  const float qn = 1.f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float w = q[0] * qn, x = q[1] * qn, y = q[2] * qn, z = q[3] * qn;
  // R: columns are the principal axes
  const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                      2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                      2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
  const float sigma = 1.f / (1.f + expf(-g.logits[i]));
  const float rho2 = (o.use_floor && g.rho2) ? g.rho2[i] : 0.f;
  float sp[3], sp2[3];
  float ratio = 1.f;
  for (int k = 0; k < 3; ++k) {
    const float s = expf(g.log_scales[k * n + i]);
    if (rho2 > 0.f) {
      sp2[k] = s * s + rho2;
      sp[k] = sqrtf(sp2[k]);
      ratio *= s / sp[k];
    } else {
      sp[k] = s;
      sp2[k] = s * s;
    }
  }
  const float sig_eff = sigma * ratio;

  Record r;
  for (int a = 0; a < 3; ++a) {
    const float inv = 1.f / sp[a];
    for (int b = 0; b < 3; ++b) r.W[3 * a + b] = R[3 * b + a] * inv;
  }
  r.mu[0] = mu[0]; r.mu[1] = mu[1]; r.mu[2] = mu[2];
  // ray-integral backbone: C = 1 / (g |W d|) with g the geometric mean of s'; the record
  // carries sigma_eff / g and the render multiplies by 1 / |W d|.  C <= s'_max / g, which
  // bounds the response for the culling below.
  float sig_bound = sig_eff;
  r.sigma = sig_eff;
  if (o.backbone == CG_BACKBONE_RAY_INTEGRAL) {
    const double g = pow((double)sp2[0] * (double)sp2[1] * (double)sp2[2], 1.0 / 6.0);
    r.sigma = (float)((double)sig_eff / g);
    sig_bound = (float)((double)sig_eff * sqrt((double)fmaxf(sp2[0], fmaxf(sp2[1], sp2[2]))) / g * 1.0001);
  }
  r.sp2[0] = sp2[0]; r.sp2[1] = sp2[1]; r.sp2[2] = sp2[2];
  r.rho2 = rho2;
  const float sp2min = fminf(sp2[0], fminf(sp2[1], sp2[2]));
  r.kg = 1.f / sp2min;

  // direction and distance from the camera centre in FP64
  const double vd[3] = {(double)mu[0] - c.o[0], (double)mu[1] - c.o[1], (double)mu[2] - c.o[2]};
  const double dist = sqrt(vd[0] * vd[0] + vd[1] * vd[1] + vd[2] * vd[2]);
  const float ux = (float)(vd[0] / dist), uy = (float)(vd[1] / dist), uz = (float)(vd[2] / dist);

  if (g.color_mode == 0) {
    for (int ch = 0; ch < 3; ++ch) r.rgb[ch] = g.color[ch * n + i];
  } else {
    float Y[16];
    sh_basis3(ux, uy, uz, Y);
    for (int ch = 0; ch < 3; ++ch) {
      float acc = 0.f;
      for (int k = 0; k < 16; ++k) acc += g.color[(3 * k + ch) * n + i] * Y[k];
      r.rgb[ch] = fmaxf(acc + 0.5f, 0.f);
    }
  }

  if (live) {
    depth_key[out] = __float_as_uint(depth_key_f32(mu[0], mu[1], mu[2], c.of[0], c.of[1], c.of[2]));
    items[out] = (uint32_t)out;  // the item indices that the depth sort permutes
  }

  // Influence cone.  If T >= alpha_min then q^T A^{-1} q <= L = 2 ln(sigma_b /
  // alpha_min) (sigma_b = sigma_eff times the backbone's largest factor), and
  //  (i) the max-response point x* = o + t* d lies within rho of the mean: |x* - mu| =
  //      |W^{-1} q| <= s'_max |q| <= s'_max sqrt(L lambda_max(A)), with lambda_max(A) <=
  //      1 + t*^2 c / s'_min^2 (c: the pixel footprint coefficient) and t* <= |v| + rho,
  //      which closes to a quadratic in rho; rays from o that meet the ball B(mu, rho)
  //      at positive t form the cone asin(rho / |v|) when |v| > rho;
  // (ii) the perpendicular distance p of the mean from the ray obeys p^2 <= L (s'_max^2 +
  //      t*^2 c): the filtered exponent is the ray's Mahalanobis distance to
  //      N(mu, Sigma_eff + footprint), whose marginal across the ray has variance at
  //      most s'_max^2 + t*^2 c.
  // The half-angle is asin(min(p, rho) / |v|).  FP64 with relative margins.
  float gamma = -1.f;
  if (dist > 0.0 && sig_bound > o.alpha_min) {
    const double L = 2.0 * log((double)sig_bound / (double)o.alpha_min);
    r.Lg = (float)L;
    const double smax = sqrt((double)fmaxf(sp2[0], fmaxf(sp2[1], sp2[2])));
    const double smin = sqrt((double)sp2min);
    const double rr = smax / smin;
    const double cw = o.filter_mode == CG_FILTER_CENTER_RAY ? 0.0 : (double)view_cmax[v] * 1.01;
    // isotropic mode spreads the in-plane trace over both whitened directions
    const double cw_perp = o.filter_mode == CG_FILTER_ISOTROPIC ? cw * rr * rr * 0.5 : cw;
    const double a = L * smax * smax, k = cw / (smin * smin), ak = a * k;
    if (ak >= 0.999) {
      gamma = kPiF;
    } else {
      const double rho =
          (ak * dist + sqrt(ak * dist * ak * dist + (1.0 - ak) * a * (1.0 + k * dist * dist))) / (1.0 - ak) * 1.001;
      if (dist + rho <= (double)o.t_near * 0.999) {
        gamma = -1.f;  // every t* is at most t_near
      } else if (dist <= rho) {
        gamma = kPiF;
      } else {
        const double tmax = dist + rho;
        const double p = sqrt(L * (smax * smax + tmax * tmax * cw_perp)) * 1.001;
        const double gm = asin(fmin(p, rho) / dist) * 1.0001 + 1e-6;
        gamma = gm < kPi ? (float)gm : kPiF;
      }
    }
  } else {
    r.Lg = 0.f;
  }
  // Tangent-cone test.  The render's pre-rejection accepts a pair only if D^2 <=
  // Lambda(t*) = L (1 + t*^2 c k)(1 + 1e-4) + 1e-6 (c <= the view's largest pixel
  // footprint coefficient, k = 1 / s'_min^2), and t* <= |v| + s'_max D (the
  // max-response point lies within s'_max D of the mean), which closes into a
  // quadratic bound D <= D_max.  D_max is widened by the rounding of the float32
  // test: n = v x d from float32 v and d is off by a few ulp of |v|, which moves the
  // tested D by at most that times s'_max / (s'_min s'_mid).  S = 0 (accept all) when
  // the bound does not close or S would not fit float32.
  double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (gamma >= 0.f && dist > 0.0) {
    const double L = (double)r.Lg, kk = (double)r.kg;
    const double cw = o.filter_mode == CG_FILTER_CENTER_RAY ? 0.0 : (double)view_cmax[v] * 1.01;
    const double A0 = 1.0001 * L + 1e-6, B0 = 1.0001 * L * cw * kk;
    double s2[3] = {(double)sp2[0], (double)sp2[1], (double)sp2[2]};
    double lo = fmin(s2[0], fmin(s2[1], s2[2])), hi = fmax(s2[0], fmax(s2[1], s2[2]));
    const double mid = s2[0] + s2[1] + s2[2] - lo - hi;
    const double smax = sqrt(hi), bs2 = B0 * hi;
    if (bs2 < 0.99) {
      const double bvs = B0 * dist * smax;
      double Dm = (bvs + sqrt(bvs * bvs + (1.0 - bs2) * (A0 + B0 * dist * dist))) / (1.0 - bs2);
      Dm = Dm * 1.0002 + 1e-6 * dist * smax / sqrt(lo * mid) + 1e-5;
      const double scale = 1.0 / (Dm * Dm * s2[0] * s2[1] * s2[2]);
      // Sigma' = R diag(s'^2) R^T
      double Sg[6];
      const int ij[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
      bool ok = true;
      for (int e = 0; e < 6; ++e) {
        const int a = ij[e][0], b = ij[e][1];
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += (double)R[3 * a + k] * s2[k] * (double)R[3 * b + k];
        Sg[e] = acc * scale * (a == b ? 1.0 : 2.0);
        ok = ok && fabs(Sg[e]) < 1e30;
      }
      if (ok)
        for (int e = 0; e < 6; ++e) S[e] = Sg[e];
    }
  }
  for (int e = 0; e < 6; ++e) r.S[e] = (float)S[e];
  r.vx = (float)vd[0];
  r.vy = (float)vd[1];
  r.vz = (float)vd[2];
  if (gamma < 0.f) r.lim = -1.f;
  else if (gamma >= kPiF) r.lim = 3.f;
  else r.lim = 2.f * sinf(0.5f * gamma) + 1e-5f;
  if (live) cone[out] = make_float4(ux, uy, uz, chord_radius(gamma));
  // The wave's 64 records are consecutive in rec: staged in LDS and written back as 1 KiB
  // contiguous stores (a direct 128-byte store per lane writes 16 bytes into each of 64
  // different lines per instruction; a staged one, 1 KiB into 8 whole lines).
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float4* __restrict__ stage = s_rec[wave];
  const float4* rv = reinterpret_cast<const float4*>(&r);
#pragma unroll
  for (int k = 0; k < kRecF4; ++k) stage[lane * (kRecF4 + 1) + k] = rv[k];
  __builtin_amdgcn_wave_barrier();
  const int64_t wave_i0 = i0 - lane;  // the wave's first item (the same in every lane)
  const int64_t first = (int64_t)v * n + wave_i0;
  const int64_t n_live = min<int64_t>(64, n - wave_i0);
  float4* __restrict__ dst = reinterpret_cast<float4*>(rec + first);
#pragma unroll
  for (int k = 0; k < kRecF4; ++k) {
    const int e = k * 64 + lane, rr = e / kRecF4, part = e - rr * kRecF4;
    if (rr < n_live) dst[e] = stage[rr * (kRecF4 + 1) + part];
  }
}

hipError_t launch_preprocess(const GaussPtrs& g, const DevCamera* cams, int n_views, const float* view_cmax,
                             const Opts& o, Record* rec, uint32_t* depth_key, uint32_t* items, float4* cone,
                             hipStream_t s) {
  if (g.n == 0 || n_views == 0) return hipSuccess;
  const int64_t chunks8 = (g.n + 8 * 256 - 1) / (8 * 256);  // groups of 8 chunks of 256 Gaussians
  const dim3 grid((unsigned)(chunks8 * 8 * n_views));
  k_preprocess<<<grid, dim3(256), 0, s>>>(g, cams, n_views, view_cmax, o, rec, depth_key, items, cone);
  return hipGetLastError();
}

}  // namespace cg
