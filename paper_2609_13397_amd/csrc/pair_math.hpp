// Per (pixel, Gaussian) filtered ray response, evaluated in a 2x2 form.
//
// Notation (Sec. 3-4): whitened ray direction a = W d, t* = -<o_u, a>/|a|^2,
// q = M_perp o_u, D^2 = |q|^2 (Eq. 2); half-edges e_i = t* M_perp W (d_i - d) (Eq. 6);
// Sigma_fp^u = E E^T / 3 with E = [e_x e_y] (Eq. 8).  Because Sigma_fp^u is rank 2 and
// orthogonal to a, Eq. 9 reduces to 2x2 algebra on K = E^T E / 3 and h = E^T q / sqrt 3:
//   det A = det(I + K G),   q^T A^{-1} q = D^2 - h^T G (I + K G)^{-1} h,
// with G = I without the floor.  With the floor, the clamp of Eq. 12 acts on the world
// footprint F F^T / 3 (F = W^{-1} E); its nonzero eigenvalues are those of
// Phi = E^T S'^2 E / 3, and [F F^T / 3 - rho^2 I]_+ = F g(Phi) F^T / 3 with
// g(lambda) = max(1 - rho^2 / lambda, 0), so the render footprint is E g(Phi) E^T / 3:
// G = g(Phi), a 2x2 matrix function computed in closed form.
//
// Precision: the mean is projected onto the ray in FP64 (w = v - (v.d) d, v = mu - o),
// and only the small perpendicular offset w is rounded to float32; everything after
// that is float32.
#pragma once

#include "camera_dev.hpp"

namespace cg {

struct PairPixel {
  double d0, d1, d2;     // centre ray (FP64)
  double o0, o1, o2;     // camera centre (FP64)
  float a0, a1, a2;      // centre ray (float32)
  float x0, x1, x2;      // d_x - d
  float y0, y1, y2;      // d_y - d
  float cpix;            // (|d_x - d|^2 + |d_y - d|^2) / 3
};

__device__ __forceinline__ PairPixel make_pair_pixel(const PixelRay& r, const DevCamera& c) {
  PairPixel p;
  p.d0 = r.d[0]; p.d1 = r.d[1]; p.d2 = r.d[2];
  p.o0 = c.o[0]; p.o1 = c.o[1]; p.o2 = c.o[2];
  p.a0 = r.df[0]; p.a1 = r.df[1]; p.a2 = r.df[2];
  p.x0 = r.dx[0]; p.x1 = r.dx[1]; p.x2 = r.dx[2];
  p.y0 = r.dy[0]; p.y1 = r.dy[1]; p.y2 = r.dy[2];
  p.cpix = r.cpix;
  return p;
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Intermediate quantities shared by the forward response and its derivative.
struct PairGeom {
  float ax, ay, az;   // a = W d
  float rn;           // 1 / |a|^2
  float qx, qy, qz;   // q
  float D2, tstar;
};

// Geometry part: a, t*, q, D^2.  Returns false when t* <= t_near (T = 0).
__device__ __forceinline__ bool pair_geom(const Record& R, const PairPixel& p, float t_near, PairGeom& g) {
  const double vx = (double)R.mu[0] - p.o0, vy = (double)R.mu[1] - p.o1, vz = (double)R.mu[2] - p.o2;
  const double te = vx * p.d0 + vy * p.d1 + vz * p.d2;
  const float wx = (float)(vx - te * p.d0), wy = (float)(vy - te * p.d1), wz = (float)(vz - te * p.d2);
  const float* W = R.W;
  g.ax = W[0] * p.a0 + W[1] * p.a1 + W[2] * p.a2;
  g.ay = W[3] * p.a0 + W[4] * p.a1 + W[5] * p.a2;
  g.az = W[6] * p.a0 + W[7] * p.a1 + W[8] * p.a2;
  g.rn = fast_rcp(g.ax * g.ax + g.ay * g.ay + g.az * g.az);
  // y = o_u + t_e a = -W w
  const float yx = -(W[0] * wx + W[1] * wy + W[2] * wz);
  const float yy = -(W[3] * wx + W[4] * wy + W[5] * wz);
  const float yz = -(W[6] * wx + W[7] * wy + W[8] * wz);
  const float f = (yx * g.ax + yy * g.ay + yz * g.az) * g.rn;
  g.tstar = (float)te - f;
  g.qx = yx - f * g.ax;
  g.qy = yy - f * g.ay;
  g.qz = yz - f * g.az;
  g.D2 = g.qx * g.qx + g.qy * g.qy + g.qz * g.qz;
  return g.tstar > t_near;
}

// Footprint part in the 2x2 form.
struct PairFoot {
  float ex0, ex1, ex2, ey0, ey1, ey2;  // e_x, e_y
  float K11, K12, K22;                 // E^T E / 3
  float h1, h2;                        // E^T q / sqrt 3
};

__device__ __forceinline__ void pair_foot(const Record& R, const PairPixel& p, const PairGeom& g, PairFoot& f) {
  const float* W = R.W;
  const float bx0 = W[0] * p.x0 + W[1] * p.x1 + W[2] * p.x2;
  const float bx1 = W[3] * p.x0 + W[4] * p.x1 + W[5] * p.x2;
  const float bx2 = W[6] * p.x0 + W[7] * p.x1 + W[8] * p.x2;
  const float by0 = W[0] * p.y0 + W[1] * p.y1 + W[2] * p.y2;
  const float by1 = W[3] * p.y0 + W[4] * p.y1 + W[5] * p.y2;
  const float by2 = W[6] * p.y0 + W[7] * p.y1 + W[8] * p.y2;
  const float px = (bx0 * g.ax + bx1 * g.ay + bx2 * g.az) * g.rn;
  const float py = (by0 * g.ax + by1 * g.ay + by2 * g.az) * g.rn;
  const float t = g.tstar;
  f.ex0 = t * (bx0 - px * g.ax); f.ex1 = t * (bx1 - px * g.ay); f.ex2 = t * (bx2 - px * g.az);
  f.ey0 = t * (by0 - py * g.ax); f.ey1 = t * (by1 - py * g.ay); f.ey2 = t * (by2 - py * g.az);
  constexpr float third = 1.f / 3.f;
  constexpr float isq3 = 0.57735026918962576f;
  f.K11 = (f.ex0 * f.ex0 + f.ex1 * f.ex1 + f.ex2 * f.ex2) * third;
  f.K12 = (f.ex0 * f.ey0 + f.ex1 * f.ey1 + f.ex2 * f.ey2) * third;
  f.K22 = (f.ey0 * f.ey0 + f.ey1 * f.ey1 + f.ey2 * f.ey2) * third;
  f.h1 = (f.ex0 * g.qx + f.ex1 * g.qy + f.ex2 * g.qz) * isq3;
  f.h2 = (f.ey0 * g.qx + f.ey1 * g.qy + f.ey2 * g.qz) * isq3;
}

// G = g(Phi) for the marginal composition; returns false when G = 0 (the floor
// covers the footprint in every direction).
__device__ __forceinline__ bool floor_G(const Record& R, const PairFoot& f, float& G11, float& G12, float& G22) {
  constexpr float third = 1.f / 3.f;
  const float P11 = (R.sp2[0] * f.ex0 * f.ex0 + R.sp2[1] * f.ex1 * f.ex1 + R.sp2[2] * f.ex2 * f.ex2) * third;
  const float P12 = (R.sp2[0] * f.ex0 * f.ey0 + R.sp2[1] * f.ex1 * f.ey1 + R.sp2[2] * f.ex2 * f.ey2) * third;
  const float P22 = (R.sp2[0] * f.ey0 * f.ey0 + R.sp2[1] * f.ey1 * f.ey1 + R.sp2[2] * f.ey2 * f.ey2) * third;
  const float m = 0.5f * (P11 + P22), dd = 0.5f * (P11 - P22);
  const float rr = sqrtf(dd * dd + P12 * P12);
  const float lp = m + rr, lm = m - rr;
  const float rho2 = R.rho2;
  if (lp <= rho2) return false;
  const float gp = 1.f - rho2 / lp;
  float gm, beta;
  if (lm > rho2) {
    gm = 1.f - rho2 / lm;
    beta = rho2 / (lp * lm);
  } else {
    gm = 0.f;
    beta = gp / (2.f * rr);
  }
  const float gbar = 0.5f * (gp + gm);
  G11 = gbar + beta * dd;
  G22 = gbar - beta * dd;
  G12 = beta * P12;
  return true;
}

// Filtered response T of one pair.  FILTER 0: centre ray; 1: anisotropic (Eq. 9);
// 2: isotropic in-plane covariance of the same trace.  MARGINAL: floor composition by
// Eq. 12 (records with rho2 = 0 take the plain path).  Returns false when the pair
// cannot reach alpha_min (T is then not set): the ray is outside the Gaussian's
// influence cone, t* <= t_near, or the pre-rejection
// D^2 > L (1 + tr Sigma_fp^u) with tr Sigma_fp^u <= t*^2 c_pix / s'_min^2, which
// bounds q^T A^{-1} q from below (Sigma_render^u is dominated by Sigma_fp^u).
template <int FILTER, bool MARGINAL>
__device__ __forceinline__ bool pair_response(const Record& R, const PairPixel& p, const Opts& o, float& T) {
  {  // influence cone of the Gaussian, tested at this pixel's centre ray
    const float cx = p.a0 - R.ux, cy = p.a1 - R.uy, cz = p.a2 - R.uz;
    if (cx * cx + cy * cy + cz * cz > R.lim * R.lim || R.lim < 0.f) return false;
  }
  PairGeom g;
  if (!pair_geom(R, p, o.t_near, g)) return false;
  if (FILTER == 0) {
    if (g.D2 > R.Lg) return false;
    T = R.sigma * __expf(-0.5f * g.D2);
    return true;
  }
  if (g.D2 > R.Lg * fmaf(g.tstar * g.tstar * p.cpix, R.kg, 1.f) * 1.0001f + 1e-6f) return false;
  PairFoot f;
  pair_foot(R, p, g, f);
  float G11 = 1.f, G12 = 0.f, G22 = 1.f;
  bool filt = true;
  if (MARGINAL && R.rho2 > 0.f) filt = floor_G(R, f, G11, G12, G22);
  if (!filt) {
    T = R.sigma * __expf(-0.5f * g.D2);
    return true;
  }
  if (FILTER == 2) {
    const float tau = (MARGINAL && R.rho2 > 0.f) ? (G11 * f.K11 + 2.f * G12 * f.K12 + G22 * f.K22) : (f.K11 + f.K22);
    const float s = 1.f + 0.5f * tau;
    const float is = fast_rcp(s);
    T = R.sigma * is * __expf(-0.5f * g.D2 * is);
    return true;
  }
  float det, quad;
  if (MARGINAL && R.rho2 > 0.f) {
    const float M11 = 1.f + f.K11 * G11 + f.K12 * G12, M12 = f.K11 * G12 + f.K12 * G22;
    const float M21 = f.K12 * G11 + f.K22 * G12, M22 = 1.f + f.K12 * G12 + f.K22 * G22;
    det = M11 * M22 - M12 * M21;
    // G adj(M)
    const float N11 = G11 * M22 - G12 * M21, N12 = G12 * M11 - G11 * M12;
    const float N21 = G12 * M22 - G22 * M21, N22 = G22 * M11 - G12 * M12;
    quad = (f.h1 * (N11 * f.h1 + N12 * f.h2) + f.h2 * (N21 * f.h1 + N22 * f.h2)) * fast_rcp(det);
  } else {
    const float P11 = 1.f + f.K11, P22 = 1.f + f.K22, P12 = f.K12;
    det = P11 * P22 - P12 * P12;
    quad = (P22 * f.h1 * f.h1 - 2.f * P12 * f.h1 * f.h2 + P11 * f.h2 * f.h2) * fast_rcp(det);
  }
  T = R.sigma * rsqrtf(det) * __expf(-0.5f * (g.D2 - quad));
  return true;
}

}  // namespace cg
