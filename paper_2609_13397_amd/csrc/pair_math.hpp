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
#include "record_bounds.hpp"

namespace cg {

// Per-pixel ray data used by every pair (64 bytes, so a wave's pixels fit in LDS).
struct PairPixel {
  double d0, d1, d2;     // centre ray (FP64)
  float a0, a1, a2;      // centre ray (float32)
  float x0, x1, x2;      // d_x - d
  float y0, y1, y2;      // d_y - d
  float cpix;            // (|d_x - d|^2 + |d_y - d|^2) / 3
};

// Camera centre in FP64 (uniform over a tile).
struct Origin {
  double x, y, z;
};

__device__ __forceinline__ PairPixel make_pair_pixel(const PixelRay& r) {
  PairPixel p;
  p.d0 = r.d[0]; p.d1 = r.d[1]; p.d2 = r.d[2];
  p.a0 = r.df[0]; p.a1 = r.df[1]; p.a2 = r.df[2];
  p.x0 = r.dx[0]; p.x1 = r.dx[1]; p.x2 = r.dx[2];
  p.y0 = r.dy[0]; p.y1 = r.dy[1]; p.y2 = r.dy[2];
  p.cpix = r.cpix;
  return p;
}

__device__ __forceinline__ Origin make_origin(const DevCamera& c) { return Origin{c.o[0], c.o[1], c.o[2]}; }


// Intermediate quantities shared by the forward response and its derivative.
struct PairGeom {
  float ax, ay, az;   // a = W d
  float rn;           // 1 / |a|^2
  float qx, qy, qz;   // q
  float D2, tstar;
  float wx, wy, wz;   // w = (I - d d^T)(mu - o), rounded from FP64
  float yx, yy, yz;   // y = -W w = o_u + t_e a
  float ya;           // y . a
};

// a = W d and 1 / |a|^2.
__device__ __forceinline__ float pair_dir(const Record& R, const PairPixel& p, PairGeom& g) {
  const float* W = R.W;
  g.ax = W[0] * p.a0 + W[1] * p.a1 + W[2] * p.a2;
  g.ay = W[3] * p.a0 + W[4] * p.a1 + W[5] * p.a2;
  g.az = W[6] * p.a0 + W[7] * p.a1 + W[8] * p.a2;
  return g.ax * g.ax + g.ay * g.ay + g.az * g.az;
}

// Geometry after pair_dir: t*, q, D^2.  Returns false when t* <= t_near (T = 0).
__device__ __forceinline__ bool pair_geom_rest(const Record& R, const PairPixel& p, const Origin& O, float t_near,
                                               PairGeom& g) {
  const double vx = (double)R.mu[0] - O.x, vy = (double)R.mu[1] - O.y, vz = (double)R.mu[2] - O.z;
  const double te = vx * p.d0 + vy * p.d1 + vz * p.d2;
  const float wx = (float)(vx - te * p.d0), wy = (float)(vy - te * p.d1), wz = (float)(vz - te * p.d2);
  const float* W = R.W;
  // y = o_u + t_e a = -W w
  const float yx = -(W[0] * wx + W[1] * wy + W[2] * wz);
  const float yy = -(W[3] * wx + W[4] * wy + W[5] * wz);
  const float yz = -(W[6] * wx + W[7] * wy + W[8] * wz);
  g.wx = wx; g.wy = wy; g.wz = wz;
  g.yx = yx; g.yy = yy; g.yz = yz;
  g.ya = yx * g.ax + yy * g.ay + yz * g.az;
  const float f = g.ya * g.rn;
  g.tstar = (float)te - f;
  g.qx = yx - f * g.ax;
  g.qy = yy - f * g.ay;
  g.qz = yz - f * g.az;
  g.D2 = g.qx * g.qx + g.qy * g.qy + g.qz * g.qz;
  return g.tstar > t_near;
}

// Geometry part: a, t*, q, D^2.  Returns false when t* <= t_near (T = 0).
__device__ __forceinline__ bool pair_geom(const Record& R, const PairPixel& p, const Origin& O, float t_near,
                                          PairGeom& g) {
  g.rn = fast_rcp(pair_dir(R, p, g));
  return pair_geom_rest(R, p, O, t_near, g);
}

// Footprint part in the 2x2 form.
struct PairFoot {
  float ex0, ex1, ex2, ey0, ey1, ey2;  // e_x, e_y
  float K11, K12, K22;                 // E^T E / 3
  float h1, h2;                        // E^T q / sqrt 3
  float bxa, bya;                      // (W (d_x - d)) . a, (W (d_y - d)) . a
};

// e_x and e_y of Eq. 6 in whitened space.
__device__ __forceinline__ void pair_edges(const Record& R, const PairPixel& p, const PairGeom& g, PairFoot& f) {
  const float* W = R.W;
  const float bx0 = W[0] * p.x0 + W[1] * p.x1 + W[2] * p.x2;
  const float bx1 = W[3] * p.x0 + W[4] * p.x1 + W[5] * p.x2;
  const float bx2 = W[6] * p.x0 + W[7] * p.x1 + W[8] * p.x2;
  const float by0 = W[0] * p.y0 + W[1] * p.y1 + W[2] * p.y2;
  const float by1 = W[3] * p.y0 + W[4] * p.y1 + W[5] * p.y2;
  const float by2 = W[6] * p.y0 + W[7] * p.y1 + W[8] * p.y2;
  f.bxa = bx0 * g.ax + bx1 * g.ay + bx2 * g.az;
  f.bya = by0 * g.ax + by1 * g.ay + by2 * g.az;
  const float px = f.bxa * g.rn;
  const float py = f.bya * g.rn;
  const float t = g.tstar;
  f.ex0 = t * (bx0 - px * g.ax); f.ex1 = t * (bx1 - px * g.ay); f.ex2 = t * (bx2 - px * g.az);
  f.ey0 = t * (by0 - py * g.ax); f.ey1 = t * (by1 - py * g.ay); f.ey2 = t * (by2 - py * g.az);
}

__device__ __forceinline__ void pair_foot(const Record& R, const PairPixel& p, const PairGeom& g, PairFoot& f) {
  pair_edges(R, p, g, f);
  constexpr float third = 1.f / 3.f;
  constexpr float isq3 = 0.57735026918962576f;
  f.K11 = (f.ex0 * f.ex0 + f.ex1 * f.ex1 + f.ex2 * f.ex2) * third;
  f.K12 = (f.ex0 * f.ey0 + f.ex1 * f.ey1 + f.ex2 * f.ey2) * third;
  f.K22 = (f.ey0 * f.ey0 + f.ey1 * f.ey1 + f.ey2 * f.ey2) * third;
  f.h1 = (f.ex0 * g.qx + f.ex1 * g.qy + f.ex2 * g.qz) * isq3;
  f.h2 = (f.ey0 * g.qx + f.ey1 * g.qy + f.ey2 * g.qz) * isq3;
}

// Floor state of one pair: Phi = E^T S'^2 E / 3, its eigen-decomposition quantities and
// G = g(Phi) (kept for the backward).
struct PairFloor {
  float G11, G12, G22;
  float P11, P12, P22;
  float dd, rr, lp, lm, gp;
};

// G = g(Phi) for the marginal composition; returns false when G = 0 (the floor
// covers the footprint in every direction).
__device__ __forceinline__ bool floor_G(const Record& R, const PairFoot& f, PairFloor& fl) {
  constexpr float third = 1.f / 3.f;
  fl.P11 = (R.sp2[0] * f.ex0 * f.ex0 + R.sp2[1] * f.ex1 * f.ex1 + R.sp2[2] * f.ex2 * f.ex2) * third;
  fl.P12 = (R.sp2[0] * f.ex0 * f.ey0 + R.sp2[1] * f.ex1 * f.ey1 + R.sp2[2] * f.ex2 * f.ey2) * third;
  fl.P22 = (R.sp2[0] * f.ey0 * f.ey0 + R.sp2[1] * f.ey1 * f.ey1 + R.sp2[2] * f.ey2 * f.ey2) * third;
  const float m = 0.5f * (fl.P11 + fl.P22);
  fl.dd = 0.5f * (fl.P11 - fl.P22);
  fl.rr = fast_sqrt(fl.dd * fl.dd + fl.P12 * fl.P12);
  fl.lp = m + fl.rr;
  fl.lm = m - fl.rr;
  const float rho2 = R.rho2;
  if (fl.lp <= rho2) return false;
  // hardware reciprocals (about 1 ulp) instead of IEEE divisions: this runs for every
  // floored pair, and the forward and its backward replay share it
  const float ilp = fast_rcp(fl.lp);
  fl.gp = 1.f - rho2 * ilp;
  float gm, beta;
  if (fl.lm > rho2) {
    const float ilm = fast_rcp(fl.lm);
    gm = 1.f - rho2 * ilm;
    beta = rho2 * ilp * ilm;
  } else {
    gm = 0.f;  // lm <= rho2 < lp, so rr > 0
    beta = fl.gp * fast_rcp(2.f * fl.rr);
  }
  const float gbar = 0.5f * (fl.gp + gm);
  fl.G11 = gbar + beta * fl.dd;
  fl.G22 = gbar - beta * fl.dd;
  fl.G12 = beta * fl.P12;
  return true;
}

// Above this tr K the 2x2 form below loses accuracy: D^2 - h^T G (I + K G)^{-1} h and
// det(I + K G) cancel (a thin Gaussian seen at a grazing angle can have K ~ 1e4, with
// D^2 and the subtracted term both ~ 1e8), and foot_stable takes over.  At or below it
// the absolute error of the exponent stays below about 1e-4 (float32 rounding of terms
// bounded by the pre-rejection's D^2 <= L (1 + 3 tr K)).
constexpr float kStableTrace = 16.f;

// det A and q^T A^{-1} q of Eq. 9 without cancellation.  q, e_x and e_y lie in the plane
// orthogonal to a.  With the orthogonal basis e_x, v = e_y - mu e_x of that plane
// (mu = K12 / K11, n1 = |e_x|^2 = 3 K11, n2 = |v|^2), write q = c_x e_x + c_y e_y; in the
// orthonormal basis of (e_x, v) the footprint E G E^T / 3 is M = R G R^T / 3 with
// E = Q R, so det A = det(I + M) = 1 + tr(G K) + N det(G) / 9 and
// q^T A^{-1} q = (|q|^2 + N c^T adj(G) c / 3) / det A, sums of non-negative terms, with
// N = n1 n2 = |e_x x e_y|^2.  N would cancel as 9 (K11 K22 - K12^2); instead, since both
// edges are orthogonal to a, e_x x e_y = t*^2 det(W) (d . (dx x dy)) a / |a|^2 (from
// (W x) x (W y) = det(W) W^{-T} (x x y)), so N = (t*^2 tau)^2 / (|a|^2 P^2) with the
// pixel's triple product tau = d . (dx x dy) and P^2 = s'1^2 s'2^2 s'3^2: products only.
// c_x = sqrt3 h1 / n1 and c_y = s / n2 with s = q . v = sqrt3 (h2 - mu h1), which loses
// only about ulp / sin(angle of e_x, e_y).  Returns false for a footprint of rank one
// (e_y parallel to e_x), which the caller leaves to the 2x2 form.
template <bool FLOOR>
__device__ __forceinline__ bool foot_stable(const Record& R, const PairPixel& p, const PairGeom& g,
                                            const PairFoot& f, const PairFloor& fl, float& det, float& expo) {
  const float c0 = p.x1 * p.y2 - p.x2 * p.y1, c1 = p.x2 * p.y0 - p.x0 * p.y2, c2 = p.x0 * p.y1 - p.x1 * p.y0;
  const float tt = g.tstar * g.tstar * (p.a0 * c0 + p.a1 * c1 + p.a2 * c2);
  const float N = tt * tt * g.rn * fast_rcp(R.sp2[0] * R.sp2[1] * R.sp2[2]);
  const float n1 = 3.f * f.K11;
  if (!(N > 1e-14f * n1 * n1)) return false;
  const float G11 = FLOOR ? fl.G11 : 1.f, G12 = FLOOR ? fl.G12 : 0.f, G22 = FLOOR ? fl.G22 : 1.f;
  constexpr float sq3 = 1.7320508075688772f;
  const float i1 = fast_rcp(n1);
  const float mu = f.K12 * 3.f * i1;
  const float cx = sq3 * f.h1 * i1;
  const float s = sq3 * (f.h2 - mu * f.h1);
  const float z1 = N * i1 * cx - mu * s;  // n2 c_x, with c_y = s / n2
  const float adjG = G22 * z1 * z1 - 2.f * G12 * z1 * s + G11 * s * s;
  const float detG = FLOOR ? (fl.lm > R.rho2 ? fl.gp * (1.f - R.rho2 * fast_rcp(fl.lm)) : 0.f) : 1.f;
  det = 1.f + (G11 * f.K11 + 2.f * G12 * f.K12 + G22 * f.K22) + N * detG * (1.f / 9.f);
  expo = (g.D2 + n1 * n1 * fast_rcp(N) * adjG * (1.f / 3.f)) * fast_rcp(det);
  return true;
}

// The cheap tests of one pair, in order: the tangent-cone test n^T S n <= |W d|^2
// (n = v x d; it passes every ray that can meet the pre-rejection bound below),
// t* > t_near, and the pre-rejection D^2 <= L (1 + tr Sigma_fp^u) with tr Sigma_fp^u
// <= t*^2 c_pix / s'_min^2, which bounds q^T A^{-1} q from below (Sigma_render^u is
// dominated by Sigma_fp^u).  False means the pair cannot reach alpha_min.  On true, g
// holds the geometry of Eq. 2.
// Tangent-cone test of pair_cheap; on true, g holds a = W d and aa = |a|^2.
__device__ __forceinline__ bool pair_tangent(const Record& R, const PairPixel& p, PairGeom& g, float& aa) {
  const float nx = R.vy * p.a2 - R.vz * p.a1;
  const float ny = R.vz * p.a0 - R.vx * p.a2;
  const float nz = R.vx * p.a1 - R.vy * p.a0;
  aa = pair_dir(R, p, g);
  const float* S = R.S;
  const float nsn = nx * (S[0] * nx + S[1] * ny + S[2] * nz) + ny * (S[3] * ny + S[4] * nz) + S[5] * nz * nz;
  return nsn <= aa;
}

// The tests of pair_cheap after the tangent-cone test (g holds a, aa = |a|^2).
template <int FILTER>
__device__ __forceinline__ bool pair_cheap_rest(const Record& R, const PairPixel& p, const Origin& O, const Opts& o,
                                                PairGeom& g, float aa) {
  g.rn = fast_rcp(aa);
  if (!pair_geom_rest(R, p, O, o.t_near, g)) return false;
  if (FILTER == 0) return g.D2 <= R.Lg;
  return g.D2 <= R.Lg * fmaf(g.tstar * g.tstar * p.cpix, R.kg, 1.f) * 1.0001f + 1e-6f;
}

template <int FILTER>
__device__ __forceinline__ bool pair_cheap(const Record& R, const PairPixel& p, const Origin& O, const Opts& o,
                                           PairGeom& g) {
  float aa;
  if (!pair_tangent(R, p, g, aa)) return false;
  return pair_cheap_rest<FILTER>(R, p, O, o, g, aa);
}

// Filtered response T of a pair that passed pair_cheap.  FILTER 0: centre ray (Eq. 3,
// C = 1); 1: anisotropic (Eq. 9); 2: isotropic in-plane covariance of the same trace.
// MARGINAL: floor composition by Eq. 12 (records with rho2 = 0 take the plain path).
// The footprint and floor state are left in f and fl for the backward.
template <int FILTER, bool MARGINAL, bool GEER>
__device__ __forceinline__ float pair_full_keep(const Record& R, const PairPixel& p, const PairGeom& g, PairFoot& f,
                                                PairFloor& fl, bool& filt) {
  // GEER: ray-integral backbone, C = 1 / (g_mean |W d|); R.sigma carries 1 / g_mean
  const float C = GEER ? fast_sqrt(g.rn) : 1.f;
  filt = true;
  if (FILTER == 0) return C * R.sigma * __expf(-0.5f * g.D2);
  pair_foot(R, p, g, f);
  fl.G11 = 1.f;
  fl.G12 = 0.f;
  fl.G22 = 1.f;
  fl.P11 = fl.P12 = fl.P22 = fl.dd = fl.rr = fl.lp = fl.lm = fl.gp = 0.f;
  if (MARGINAL && R.rho2 > 0.f) filt = floor_G(R, f, fl);
  if (!filt) return C * R.sigma * __expf(-0.5f * g.D2);
  const float G11 = fl.G11, G12 = fl.G12, G22 = fl.G22;
  if (FILTER == 2) {
    const float tau = (MARGINAL && R.rho2 > 0.f) ? (G11 * f.K11 + 2.f * G12 * f.K12 + G22 * f.K22) : (f.K11 + f.K22);
    const float s = 1.f + 0.5f * tau;
    const float is = fast_rcp(s);
    return C * R.sigma * is * __expf(-0.5f * g.D2 * is);
  }
  float det, quad;
  if (!(f.K11 + f.K22 <= kStableTrace)) {  // large whitened footprint
    float expo;
    const bool ok = (MARGINAL && R.rho2 > 0.f) ? foot_stable<true>(R, p, g, f, fl, det, expo)
                                               : foot_stable<false>(R, p, g, f, fl, det, expo);
    if (ok) return C * R.sigma * fast_rsq(det) * __expf(-0.5f * expo);
  }
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
  return C * R.sigma * fast_rsq(det) * __expf(-0.5f * (g.D2 - quad));
}

template <int FILTER, bool MARGINAL, bool GEER>
__device__ __forceinline__ float pair_full(const Record& R, const PairPixel& p, const PairGeom& g) {
  PairFoot f;
  PairFloor fl;
  bool filt;
  return pair_full_keep<FILTER, MARGINAL, GEER>(R, p, g, f, fl, filt);
}

// Both parts; false when the pair cannot reach alpha_min (T is then not set).
template <int FILTER, bool MARGINAL, bool GEER>
__device__ __forceinline__ bool pair_response(const Record& R, const PairPixel& p, const Origin& O, const Opts& o,
                                              float& T) {
  PairGeom g;
  if (!pair_cheap<FILTER>(R, p, O, o, g)) return false;
  T = pair_full<FILTER, MARGINAL, GEER>(R, p, g);
  return true;
}

}  // namespace cg
