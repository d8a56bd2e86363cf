// Device camera models: the inverse mapping Pi^{-1} (Sec. 3) for pinhole,
// equidistant Kannala-Brandt fisheye and equirectangular cameras, and the forward
// mapping Pi used by the floor bake (Eq. 11).
//
// Rays are computed in FP64.  The whitened ray-to-centre offset of Eq. 2 is a small
// difference of large vectors: a 1-ulp float32 error in the ray direction moves a
// Gaussian at distance t by t * 6e-8 across the ray, which for the small, distant
// Gaussians of the workloads is ~1e-3 of their scale.  FP64 directions (once per
// pixel) remove that error; the per-pair arithmetic then needs FP64 only for the
// projection of the mean onto the ray.
#pragma once

#include "cg_common.hpp"

namespace cg {

__device__ __forceinline__ double kb_theta_d(const DevCamera& c, double th) {
  const double t2 = th * th;
  return th * (1.0 + t2 * (c.k[0] + t2 * (c.k[1] + t2 * (c.k[2] + t2 * c.k[3]))));
}

__device__ __forceinline__ double kb_slope(const DevCamera& c, double th) {
  const double t2 = th * th;
  return 1.0 + t2 * (3.0 * c.k[0] + t2 * (5.0 * c.k[1] + t2 * (7.0 * c.k[2] + t2 * 9.0 * c.k[3])));
}

// theta_d(theta) = thd on [0, theta_max] (theta_d is increasing there, checked on the
// host).  A float32 bracketed Newton solve gives a start within about 1e-6; FP64
// bracketed Newton then converges from it in two or three steps.  Each FP64 step
// divides by the slope through a float32 reciprocal: its relative error (~1e-7) only
// scales a step that is already small, and the loop runs until the step is below
// 1e-15, so the root is the FP64 one.  A residual of exactly zero ends the solve (the
// iterate is the root; a Newton step from it would sit on the bracket's end); a step
// that leaves the bracket (or is not a number) is replaced by bisection.
__device__ inline double kb_solve(const DevCamera& c, double thd) {
  const float k0 = (float)c.k[0], k1 = (float)c.k[1], k2 = (float)c.k[2], k3 = (float)c.k[3];
  const float tdf = (float)thd;
  float lof = 0.f, hif = (float)c.theta_max;
  float tf = fminf(tdf, hif);
  for (int it = 0; it < 32; ++it) {
    const float t2 = tf * tf;
    const float f = tf * (1.f + t2 * (k0 + t2 * (k1 + t2 * (k2 + t2 * k3)))) - tdf;
    if (f == 0.f) break;
    const float sl = 1.f + t2 * (3.f * k0 + t2 * (5.f * k1 + t2 * (7.f * k2 + t2 * 9.f * k3)));
    if (f > 0.f) hif = tf; else lof = tf;
    float nt = tf - f * __builtin_amdgcn_rcpf(sl);
    if (!(nt >= lof && nt <= hif)) nt = 0.5f * (lof + hif);
    const bool conv = fabsf(nt - tf) < 1e-6f || hif - lof < 1e-6f;
    tf = nt;
    if (conv) break;
  }
  double lo = 0.0, hi = c.theta_max;
  double th = fmin(fmax((double)tf, 0.0), hi);
  for (int it = 0; it < 64; ++it) {
    const double f = kb_theta_d(c, th) - thd;
    if (f == 0.0) break;
    if (f > 0.0) hi = th; else lo = th;
    double nt = th - f * (double)__builtin_amdgcn_rcpf((float)kb_slope(c, th));
    if (!(nt >= lo && nt <= hi)) nt = 0.5 * (lo + hi);
    const bool conv = fabs(nt - th) < 1e-15 || hi - lo < 1e-15;
    th = nt;
    if (conv) break;
  }
  return th;
}

__device__ __forceinline__ void rot(const double* R, const double v[3], double out[3]) {
  out[0] = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
  out[1] = R[3] * v[0] + R[4] * v[1] + R[5] * v[2];
  out[2] = R[6] * v[0] + R[7] * v[1] + R[8] * v[2];
}

// Pi^{-1}: continuous full-image coordinate -> unit world direction; false when the
// coordinate is outside the camera's valid domain.
__device__ inline bool cam_unproject(const DevCamera& c, double x, double y, double d[3]) {
  double dc[3];
  if (c.model == CG_PINHOLE) {
    const double mx = (x - c.cx) * c.inv_fx, my = (y - c.cy) * c.inv_fy;
    const double ir = 1.0 / sqrt(mx * mx + my * my + 1.0);
    dc[0] = mx * ir; dc[1] = my * ir; dc[2] = ir;
  } else if (c.model == CG_FISHEYE_KB) {
    const double mx = (x - c.cx) * c.inv_fx, my = (y - c.cy) * c.inv_fy;
    const double thd = sqrt(mx * mx + my * my);
    if (thd > c.thd_max) return false;
    if (thd == 0.0) {
      dc[0] = 0.0; dc[1] = 0.0; dc[2] = 1.0;
    } else {
      const double th = kb_solve(c, thd);
      double sn, cs;
      sincos(th, &sn, &cs);
      const double s = sn / thd;
      dc[0] = s * mx; dc[1] = s * my; dc[2] = cs;
    }
  } else {
    const double phi = 2.0 * kPi * (x * c.inv_w - 0.5);
    const double lam = kPi * (0.5 - y * c.inv_h);
    double sp, cp, sl, cl;
    sincos(phi, &sp, &cp);
    sincos(lam, &sl, &cl);
    dc[0] = cl * sp; dc[1] = -sl; dc[2] = cl * cp;
  }
  rot(c.R, dc, d);
  return true;
}

// Pi: unit world direction -> continuous full-image coordinate.
__device__ inline bool cam_project(const DevCamera& c, const double dw[3], double* x, double* y) {
  double dc[3];
  rot(c.Rinv, dw, dc);
  if (c.model == CG_PINHOLE) {
    if (dc[2] <= 0.0) return false;
    *x = c.fx * dc[0] / dc[2] + c.cx;
    *y = c.fy * dc[1] / dc[2] + c.cy;
    return true;
  } else if (c.model == CG_FISHEYE_KB) {
    const double rxy = sqrt(dc[0] * dc[0] + dc[1] * dc[1]);
    const double th = atan2(rxy, dc[2]);
    if (th > c.theta_max) return false;
    if (rxy == 0.0) { *x = c.cx; *y = c.cy; return true; }
    const double thd = kb_theta_d(c, th);
    *x = c.fx * thd * dc[0] / rxy + c.cx;
    *y = c.fy * thd * dc[1] / rxy + c.cy;
    return true;
  } else {
    const double n = sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]);
    const double phi = atan2(dc[0], dc[2]);
    const double lam = asin(fmax(-1.0, fmin(1.0, -dc[1] / n)));
    *x = c.full_w * (phi / (2.0 * kPi) + 0.5);
    *y = c.full_h * (0.5 - lam / kPi);
    return true;
  }
}

// Centre ray and half-pixel edge-ray differentials of one pixel (Sec. 4.1): the
// forward offsets (1/2, 0), (0, 1/2), or the backward ones where the forward offset
// leaves the valid domain.  d in FP64; the differentials d_i - d are formed in FP64
// and then rounded, so they keep full relative precision.
struct PixelRay {
  double d[3];
  float df[3];
  float dx[3], dy[3];
  float cpix;  // (|d_x - d|^2 + |d_y - d|^2) / 3 (times footprint_scale^2)
  bool valid;
};

__device__ inline PixelRay pixel_ray(const DevCamera& c, int i, int j, float fs) {
  PixelRay r;
  const double px = c.crop_x0 + i + 0.5, py = c.crop_y0 + j + 0.5;
  double ex[3], ey[3];
  if (c.model == CG_EQUIRECT) {
    // Pi^{-1} separates in (phi(x), lambda(y)), and the forward half-pixel offsets
    // are always in the domain: the edge rays reuse the centre's sines and cosines
    // through the angle-addition formulas with the camera's fixed half-pixel steps.
    const double phi = 2.0 * kPi * (px * c.inv_w - 0.5);
    const double lam = kPi * (0.5 - py * c.inv_h);
    double sp, cp, sl, cl;
    sincos(phi, &sp, &cp);
    sincos(lam, &sl, &cl);
    const double sp1 = sp * c.eq_step[0] + cp * c.eq_step[1], cp1 = cp * c.eq_step[0] - sp * c.eq_step[1];
    const double sl1 = sl * c.eq_step[2] + cl * c.eq_step[3], cl1 = cl * c.eq_step[2] - sl * c.eq_step[3];
    const double dc[3] = {cl * sp, -sl, cl * cp}, xc[3] = {cl * sp1, -sl, cl * cp1}, yc[3] = {cl1 * sp, -sl1, cl1 * cp};
    rot(c.R, dc, r.d);
    rot(c.R, xc, ex);
    rot(c.R, yc, ey);
    r.valid = true;
  } else {
    r.valid = cam_unproject(c, px, py, r.d);
    if (!r.valid) {
      for (int k = 0; k < 3; ++k) { r.d[k] = 0.0; r.df[k] = 0.f; r.dx[k] = 0.f; r.dy[k] = 0.f; }
      r.cpix = 0.f;
      return r;
    }
    if (!cam_unproject(c, px + 0.5, py, ex) && !cam_unproject(c, px - 0.5, py, ex))
      for (int k = 0; k < 3; ++k) ex[k] = r.d[k];
    if (!cam_unproject(c, px, py + 0.5, ey) && !cam_unproject(c, px, py - 0.5, ey))
      for (int k = 0; k < 3; ++k) ey[k] = r.d[k];
  }
  for (int k = 0; k < 3; ++k) r.dx[k] = (float)((ex[k] - r.d[k]) * (double)fs);
  for (int k = 0; k < 3; ++k) r.dy[k] = (float)((ey[k] - r.d[k]) * (double)fs);
  for (int k = 0; k < 3; ++k) r.df[k] = (float)r.d[k];
  r.cpix = (r.dx[0] * r.dx[0] + r.dx[1] * r.dx[1] + r.dx[2] * r.dx[2] + r.dy[0] * r.dy[0] + r.dy[1] * r.dy[1] +
            r.dy[2] * r.dy[2]) * (1.0f / 3.0f);
  return r;
}

// View of a global tile index (views are few; linear scan).
__device__ __forceinline__ int view_of_tile(const DevCamera* cams, int n_views, int tile) {
  int v = 0;
  while (v + 1 < n_views && cams[v + 1].tile_offset <= tile) ++v;
  return v;
}

__device__ __forceinline__ int view_of_group(const DevCamera* cams, int n_views, int group) {
  int v = 0;
  while (v + 1 < n_views && cams[v + 1].group_offset <= group) ++v;
  return v;
}

// Chord-cone overlap test (the chord form of cg_common.hpp): |a - b| <= w_a + w_b,
// written as |a - b|^2 <= lim |lim| so that a negative sum (an empty cone) fails.
__device__ __forceinline__ bool chords_overlap(const float4& a, float bx, float by, float bz, float bw) {
  const float dx = a.x - bx, dy = a.y - by, dz = a.z - bz;
  const float lim = a.w + bw;
  return dx * dx + dy * dy + dz * dz <= lim * fabsf(lim);
}

// Chord radius of a cone of half angle beta, with a 5e-6 absolute margin for the
// float32 rounding of the test (each side of a test carries one).
__device__ __forceinline__ float chord_radius(float beta) {
  if (beta < 0.f) return kChordNever;
  if (beta >= kPiF) return kChordAll;
  return 2.f * sinf(0.5f * beta) + 5e-6f;
}

}  // namespace cg
