// ConeGaussian FP64 CPU oracle.
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
// reference that the GPU renderer is checked against.  Only the test-suite, the
// smoke check and the benchmark's CPU-baseline leg may load it; the product path
// never does.  It shares no code, header, table or constant with the HIP library.
//
// Everything is computed in double precision from the float32 inputs (upcast
// exactly).  Each function names the passage of the paper it follows.  Where the
// paper is silent the chosen reading is stated next to the code:
//
//   * camera models (the paper names pinhole and fisheye only): OpenCV axes,
//     pinhole, equidistant Kannala-Brandt, equirectangular;
//   * pixel (i, j) of the crop window has centre (x0 + i + 1/2, y0 + j + 1/2);
//   * neighbour rays use the forward half-pixel offsets of Sec. 4.1, falling back
//     to the backward offset when the forward one leaves the camera's valid domain;
//   * backbone factor C[w] = 1 (max-response instance of Eq. 3);
//   * compositing order (Eq. 4): one key per Gaussian and view, the distance
//     |mu - o| (compared as its square) in double precision, ties broken by index.
//     Two composited Gaussians whose keys agree to within float rounding are an
//     order decision: a renderer that sorts a rounded key may take them the other
//     way round, and the result with the two swapped is kept as an alternative;
//   * cut-offs: alpha = min(T, alpha_max); skip if alpha < alpha_min; stop before
//     the Gaussian that would take transmittance below T_min; T = 0 if t* <= t_near.
//
// Build: g++ -O2 -fopenmp -ffp-contract=off -shared -fPIC (see build_oracle.py).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

// ----------------------------------------------------------------------------- types

struct orc_camera {
  int32_t model;  // 0 pinhole, 1 Kannala-Brandt fisheye, 2 equirectangular
  int32_t full_w, full_h;
  int32_t crop_x0, crop_y0, crop_w, crop_h;
  float fx, fy, cx, cy;
  float k[4];
  float R_c2w[9];  // row-major, columns are the camera axes in world coordinates
  float origin[3];
  float theta_max;
};

struct orc_gaussians {
  int64_t n;
  int32_t color_mode;  // 0: rgb[3][n]; 3: sh[48][n] (index 3*coef + channel)
  const float* means;          // [3][n]
  const float* log_scales;     // [3][n]
  const float* quats;          // [4][n]  (w, x, y, z), not necessarily unit
  const float* opacity_logits; // [n]
  const float* color;          // [3][n] or [48][n]
  const float* rho2;           // [n] or NULL (= 0)
};

struct orc_opts {
  int32_t filter_mode;   // 0 centre ray, 1 anisotropic footprint (Eq. 9), 2 isotropic
  int32_t use_floor;     // apply the floor of Eq. 10 with rho^2
  int32_t composition;   // 0 marginal (Eq. 12), 1 additive (floor + full footprint)
  float alpha_min, alpha_max, T_min, t_near;
  float bg[3];
  float footprint_scale; // multiplies the neighbour-ray differentials
  int32_t order_mode;    // 0 per-Gaussian key |mu - o|; 1 per-ray max-response depth t*
  int32_t backbone;      // 0 max response (w = delta(t - t*), C = 1); 1 ray integral (w = 1)
};

}  // extern "C"

namespace {

constexpr double kPi = 3.14159265358979323846;

// ----------------------------------------------------------------------------- 3-vectors

inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

inline void matvec(const double M[3][3], const double* x, double* y) {
  for (int i = 0; i < 3; ++i) y[i] = M[i][0] * x[0] + M[i][1] * x[1] + M[i][2] * x[2];
}

inline void matmul(const double A[3][3], const double B[3][3], double C[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[i][j] = A[i][0] * B[0][j] + A[i][1] * B[1][j] + A[i][2] * B[2][j];
}

inline void transpose(const double A[3][3], double T[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) T[i][j] = A[j][i];
}

inline double det3(const double A[3][3]) {
  return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
         A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

// Inverse by the adjugate (A is symmetric positive definite here).
inline void inv3(const double A[3][3], double I[3][3]) {
  const double d = det3(A);
  I[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / d;
  I[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / d;
  I[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / d;
  I[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / d;
  I[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / d;
  I[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / d;
  I[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / d;
  I[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / d;
  I[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / d;
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix: A = V diag(w) V^T.
void jacobi3(const double Ain[3][3], double w[3], double V[3][3]) {
  double A[3][3];
  std::memcpy(A, Ain, sizeof(A));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double diag = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-40 * diag || off == 0.0) break;
    for (int p = 0; p < 2; ++p) {
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {  // A <- A G (columns p, q)
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {  // A <- G^T A (rows p, q)
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
    }
  }
  for (int i = 0; i < 3; ++i) w[i] = A[i][i];
}

// ----------------------------------------------------------------------------- cameras
// Sec. 3: a pixel (x, y) of a central camera yields the world ray (o, d) through the
// inverse mapping; the paper gives no camera formulas, so the models below are the
// stated readings.  (x, y) are continuous coordinates of the full virtual image.

double kb_theta_d(const orc_camera& c, double th) {
  const double t2 = th * th;
  return th * (1.0 + c.k[0] * t2 + c.k[1] * t2 * t2 + c.k[2] * t2 * t2 * t2 + c.k[3] * t2 * t2 * t2 * t2);
}

double kb_theta_d_slope(const orc_camera& c, double th) {
  const double t2 = th * th;
  return 1.0 + 3.0 * c.k[0] * t2 + 5.0 * c.k[1] * t2 * t2 + 7.0 * c.k[2] * t2 * t2 * t2 +
         9.0 * c.k[3] * t2 * t2 * t2 * t2;
}

// Solve theta_d(theta) = thd on [0, theta_max]: bracketed Newton, bisection when a
// Newton step leaves the bracket.  Requires theta_d increasing on the interval.
double kb_solve(const orc_camera& c, double thd) {
  double lo = 0.0, hi = c.theta_max;
  double th = std::min(thd, hi);
  for (int it = 0; it < 200; ++it) {
    const double f = kb_theta_d(c, th) - thd;
    if (f > 0) hi = th; else lo = th;
    const double step = f / kb_theta_d_slope(c, th);
    double nt = th - step;
    if (!(nt > lo && nt < hi)) nt = 0.5 * (lo + hi);
    if (std::fabs(nt - th) < 1e-15 || hi - lo < 1e-15) { th = nt; break; }
    th = nt;
  }
  return th;
}

void to_world(const orc_camera& c, const double dc[3], double dw[3]) {
  for (int i = 0; i < 3; ++i)
    dw[i] = (double)c.R_c2w[3 * i + 0] * dc[0] + (double)c.R_c2w[3 * i + 1] * dc[1] + (double)c.R_c2w[3 * i + 2] * dc[2];
}

// World -> camera uses the exact inverse of the stored float32 rotation (which is
// orthonormal only to float32 rounding), so that Pi(Pi^{-1}(p)) = p holds in FP64.
void to_cam(const orc_camera& c, const double dw[3], double dc[3]) {
  double R[3][3], Ri[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[i][j] = c.R_c2w[3 * i + j];
  inv3(R, Ri);
  matvec(Ri, dw, dc);
}

// Inverse mapping Pi^{-1}: continuous pixel coordinate -> unit world direction.
// Returns false outside the camera's valid domain (KB: theta > theta_max).
bool unproject(const orc_camera& c, double x, double y, double d[3]) {
  double dc[3];
  if (c.model == 0) {
    const double mx = (x - c.cx) / c.fx, my = (y - c.cy) / c.fy;
    const double r = std::sqrt(mx * mx + my * my + 1.0);
    dc[0] = mx / r; dc[1] = my / r; dc[2] = 1.0 / r;
  } else if (c.model == 1) {
    const double mx = (x - c.cx) / c.fx, my = (y - c.cy) / c.fy;
    const double thd = std::sqrt(mx * mx + my * my);
    if (thd > kb_theta_d(c, c.theta_max)) return false;
    if (thd == 0.0) {
      dc[0] = 0.0; dc[1] = 0.0; dc[2] = 1.0;
    } else {
      const double th = kb_solve(c, thd);
      const double s = std::sin(th) / thd;
      dc[0] = s * mx; dc[1] = s * my; dc[2] = std::cos(th);
    }
  } else if (c.model == 2) {
    const double phi = 2.0 * kPi * (x / c.full_w - 0.5);
    const double lam = kPi * (0.5 - y / c.full_h);
    dc[0] = std::cos(lam) * std::sin(phi);
    dc[1] = -std::sin(lam);
    dc[2] = std::cos(lam) * std::cos(phi);
  } else {
    return false;
  }
  to_world(c, dc, d);
  return true;
}

// Forward mapping Pi: world direction -> continuous pixel coordinate of the full image.
bool project(const orc_camera& c, const double dw[3], double* x, double* y) {
  double dc[3];
  to_cam(c, dw, dc);
  if (c.model == 0) {
    if (dc[2] <= 0) return false;
    *x = c.fx * dc[0] / dc[2] + c.cx;
    *y = c.fy * dc[1] / dc[2] + c.cy;
    return true;
  } else if (c.model == 1) {
    const double rxy = std::sqrt(dc[0] * dc[0] + dc[1] * dc[1]);
    const double th = std::atan2(rxy, dc[2]);
    if (th > c.theta_max) return false;
    if (rxy == 0.0) { *x = c.cx; *y = c.cy; return true; }
    const double thd = kb_theta_d(c, th);
    *x = c.fx * thd * dc[0] / rxy + c.cx;
    *y = c.fy * thd * dc[1] / rxy + c.cy;
    return true;
  } else if (c.model == 2) {
    const double n = std::sqrt(dot3(dc, dc));
    const double phi = std::atan2(dc[0], dc[2]);
    const double lam = std::asin(std::max(-1.0, std::min(1.0, -dc[1] / n)));
    *x = c.full_w * (phi / (2.0 * kPi) + 0.5);
    *y = c.full_h * (0.5 - lam / kPi);
    return true;
  }
  return false;
}

// Centre ray and the two half-pixel edge rays of one pixel (Sec. 4.1, Eq. 6 setup).
struct PixelRays {
  bool valid;
  double d[3], dx[3], dy[3];
};

PixelRays pixel_rays(const orc_camera& c, double px, double py) {
  PixelRays r;
  r.valid = unproject(c, px, py, r.d);
  if (!r.valid) return r;
  if (!unproject(c, px + 0.5, py, r.dx) && !unproject(c, px - 0.5, py, r.dx))
    std::memcpy(r.dx, r.d, sizeof(r.d));
  if (!unproject(c, px, py + 0.5, r.dy) && !unproject(c, px, py - 0.5, r.dy))
    std::memcpy(r.dy, r.d, sizeof(r.d));
  return r;
}

// ----------------------------------------------------------------------------- colour
// Real spherical harmonics up to degree 3, orthonormal on the sphere, with the
// Condon-Shortley phase carried by the associated Legendre functions.  The
// constants come from the definition, not from a table:
//   Y_l^m = sqrt(2) K_l^|m| P_l^|m|(cos th) sin(|m| phi)  (m < 0)
//   Y_l^0 =          K_l^0  P_l^0(cos th)
//   Y_l^m = sqrt(2) K_l^m   P_l^m(cos th)  cos(m phi)    (m > 0)
//   K_l^m = sqrt((2l + 1) / (4 pi) * (l - m)! / (l + m)!)

double assoc_legendre(int l, int m, double x) {
  // P_m^m = (-1)^m (2m - 1)!! (1 - x^2)^{m/2}; upward recurrence in l.
  double pmm = 1.0;
  const double somx2 = std::sqrt(std::max(0.0, (1.0 - x) * (1.0 + x)));
  double fact = 1.0;
  for (int i = 1; i <= m; ++i) { pmm *= -fact * somx2; fact += 2.0; }
  if (l == m) return pmm;
  double pmmp1 = x * (2 * m + 1) * pmm;
  if (l == m + 1) return pmmp1;
  double pll = 0.0;
  for (int ll = m + 2; ll <= l; ++ll) {
    pll = ((2 * ll - 1) * x * pmmp1 - (ll + m - 1) * pmm) / (ll - m);
    pmm = pmmp1;
    pmmp1 = pll;
  }
  return pll;
}

double factorial(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

void sh_basis(const double dir[3], double Y[16]) {
  const double n = std::sqrt(dot3(dir, dir));
  const double x = dir[0] / n, y = dir[1] / n, z = dir[2] / n;
  const double th = std::acos(std::max(-1.0, std::min(1.0, z)));
  const double phi = std::atan2(y, x);
  int idx = 0;
  for (int l = 0; l <= 3; ++l) {
    for (int m = -l; m <= l; ++m) {
      const int am = m < 0 ? -m : m;
      const double K = std::sqrt((2.0 * l + 1.0) / (4.0 * kPi) * factorial(l - am) / factorial(l + am));
      const double P = assoc_legendre(l, am, std::cos(th));
      double v;
      if (m < 0) v = std::sqrt(2.0) * K * P * std::sin(am * phi);
      else if (m == 0) v = K * P;
      else v = std::sqrt(2.0) * K * P * std::cos(am * phi);
      Y[idx++] = v;
    }
  }
}

// ----------------------------------------------------------------------------- Gaussians
// Sec. 3: mean mu, Sigma = R S^2 R^T, opacity sigma; whitening W = S^{-1} R^T.
// Eq. 10: with the floor, s_i -> sqrt(s_i^2 + rho^2) and
// sigma_eff = sigma * prod_i s_i / sqrt(s_i^2 + rho^2); whitening then uses Sigma_eff.

struct GaussRaw {
  double mu[3], log_s[3], quat[4], logit;
};

struct GaussPre {
  double mu[3];
  double sp[3];        // effective scales s'
  double R[3][3];      // columns = principal axes
  double W[3][3];      // diag(1/s') R^T
  double Winv[3][3];   // R diag(s')
  double sigma;        // effective opacity
  double rho2;         // floor variance (0 when the floor is off)
};

GaussRaw raw_of(const orc_gaussians& g, int64_t i) {
  GaussRaw r;
  const int64_t n = g.n;
  for (int k = 0; k < 3; ++k) { r.mu[k] = g.means[k * n + i]; r.log_s[k] = g.log_scales[k * n + i]; }
  for (int k = 0; k < 4; ++k) r.quat[k] = g.quats[k * n + i];
  r.logit = g.opacity_logits[i];
  return r;
}

GaussPre preprocess(const GaussRaw& r, double rho2_in, bool use_floor) {
  GaussPre p;
  std::memcpy(p.mu, r.mu, sizeof(p.mu));
  const double qn = std::sqrt(r.quat[0] * r.quat[0] + r.quat[1] * r.quat[1] + r.quat[2] * r.quat[2] + r.quat[3] * r.quat[3]);
  const double w = r.quat[0] / qn, x = r.quat[1] / qn, y = r.quat[2] / qn, z = r.quat[3] / qn;
  p.R[0][0] = 1 - 2 * (y * y + z * z); p.R[0][1] = 2 * (x * y - w * z);     p.R[0][2] = 2 * (x * z + w * y);
  p.R[1][0] = 2 * (x * y + w * z);     p.R[1][1] = 1 - 2 * (x * x + z * z); p.R[1][2] = 2 * (y * z - w * x);
  p.R[2][0] = 2 * (x * z - w * y);     p.R[2][1] = 2 * (y * z + w * x);     p.R[2][2] = 1 - 2 * (x * x + y * y);
  const double sigma = 1.0 / (1.0 + std::exp(-r.logit));
  const double rho2 = use_floor ? rho2_in : 0.0;
  double ratio = 1.0;
  for (int k = 0; k < 3; ++k) {
    const double s = std::exp(r.log_s[k]);
    p.sp[k] = std::sqrt(s * s + rho2);
    ratio *= s / p.sp[k];
  }
  p.sigma = sigma * ratio;
  p.rho2 = rho2;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      p.W[i][j] = p.R[j][i] / p.sp[i];
      p.Winv[i][j] = p.R[i][j] * p.sp[j];
    }
  return p;
}

// View-dependent colour: RGB as given, or SH evaluated at the unit direction from the
// camera centre to the mean, offset by 1/2 and clamped at 0 per channel.
void gauss_color(const orc_gaussians& g, int64_t i, const double mu[3], const double o[3], double col[3],
                 double* Y_out = nullptr, bool* clamped = nullptr) {
  const int64_t n = g.n;
  if (g.color_mode == 0) {
    for (int c = 0; c < 3; ++c) col[c] = g.color[c * n + i];
    if (clamped) for (int c = 0; c < 3; ++c) clamped[c] = false;
    return;
  }
  double dir[3] = {mu[0] - o[0], mu[1] - o[1], mu[2] - o[2]};
  double Y[16];
  sh_basis(dir, Y);
  for (int c = 0; c < 3; ++c) {
    double s = 0.0;
    for (int k = 0; k < 16; ++k) s += (double)g.color[(3 * k + c) * n + i] * Y[k];
    s += 0.5;
    if (clamped) clamped[c] = s < 0.0;
    col[c] = s > 0.0 ? s : 0.0;
  }
  if (Y_out) std::memcpy(Y_out, Y, sizeof(Y));
}

// ----------------------------------------------------------------------------- pair response

struct PairResult {
  double T;       // response (0 when cut by t_near)
  double T_raw;   // response ignoring the t_near cut
  double tstar;
  double D2;
};

// The filtered ray response of one Gaussian for one pixel.
//   Eq. 1-2:  o_u = W (o - mu), d_u = W d, t* = -<o_u, d_u>/|d_u|^2, q = o_u + t* d_u, D^2 = |q|^2
//   Eq. 6:    e_i = t* M_perp W (d_i - d),  M_perp = I - d_u d_u^T / |d_u|^2
//   Eq. 8:    Sigma_fp^u = (e_x e_x^T + e_y e_y^T) / 3
//   Eq. 12:   Sigma_render^u = W [ W^{-1} Sigma_fp^u W^{-T} - rho^2 I ]_+ W^T   (floor on, marginal)
//   Eq. 9:    T = sigma / sqrt(det A) * exp(-q^T A^{-1} q / 2),  A = I + Sigma_render^u
// The PSD clamp of Eq. 12 is taken literally: eigen-decompose the symmetric 3x3
// matrix and zero its negative eigenvalues.  filter_mode 0 drops the footprint
// (Eq. 3 with C = 1); filter_mode 2 replaces the footprint by the isotropic
// in-plane covariance with the same trace.
// Longitudinal factor C[w] of the weighted ray response for w = 1 (the ray integral
// of Sec. 3): with G normalised as exp(-q^2/2) / (Z_G sqrt(det Sigma)), the integral of
// exp(-|o_u + t d_u|^2 / 2) over t is sqrt(2 pi) / |d_u| exp(-D^2 / 2), so
// C = sqrt(2 pi) / (Z_G sqrt(det Sigma) |d_u|).  Z_G is not given by the paper; the
// reading taken here is Z_G = sqrt(2 pi) det(Sigma)^(-1/3), the value for which an
// isotropic Gaussian's integral response equals its max response (C = 1).  Sigma is
// the effective covariance R S'^2 R^T.  nn = |d_u|^2.
double geer_factor(const GaussPre& G, double nn) {
  double WiT[3][3], Sig[3][3];
  transpose(G.Winv, WiT);
  matmul(G.Winv, WiT, Sig);
  const double detS = det3(Sig);
  const double ZG = std::sqrt(2.0 * kPi) * std::pow(detS, -1.0 / 3.0);
  return std::sqrt(2.0 * kPi) / (ZG * std::sqrt(detS) * std::sqrt(nn));
}

PairResult pair_response(const GaussPre& G, const double o[3], const double d[3], const double dx[3],
                         const double dy[3], const orc_opts& op) {
  PairResult res{0.0, 0.0, 0.0, 0.0};
  double om[3] = {o[0] - G.mu[0], o[1] - G.mu[1], o[2] - G.mu[2]};
  double ou[3], du[3];
  matvec(G.W, om, ou);
  matvec(G.W, d, du);
  const double nn = dot3(du, du);
  const double ts = -dot3(ou, du) / nn;
  double q[3] = {ou[0] + ts * du[0], ou[1] + ts * du[1], ou[2] + ts * du[2]};
  const double D2 = dot3(q, q);
  res.tstar = ts;
  res.D2 = D2;
  double T;
  if (op.filter_mode == 0) {
    T = G.sigma * std::exp(-0.5 * D2);
  } else {
    double Mp[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Mp[i][j] = (i == j ? 1.0 : 0.0) - du[i] * du[j] / nn;
    double e[2][3];
    const double* di[2] = {dx, dy};
    for (int k = 0; k < 2; ++k) {
      double dd[3] = {(di[k][0] - d[0]) * op.footprint_scale, (di[k][1] - d[1]) * op.footprint_scale,
                      (di[k][2] - d[2]) * op.footprint_scale};
      double wd[3], pw[3];
      matvec(G.W, dd, wd);
      matvec(Mp, wd, pw);
      for (int j = 0; j < 3; ++j) e[k][j] = ts * pw[j];
    }
    double S[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) S[i][j] = (e[0][i] * e[0][j] + e[1][i] * e[1][j]) / 3.0;
    if (op.use_floor && op.composition == 0 && G.rho2 > 0.0) {
      double WiT[3][3], tmp[3][3], B[3][3];
      transpose(G.Winv, WiT);
      matmul(G.Winv, S, tmp);
      matmul(tmp, WiT, B);
      for (int i = 0; i < 3; ++i) B[i][i] -= G.rho2;
      double w[3], V[3][3];
      jacobi3(B, w, V);
      double Bp[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double s = 0.0;
          for (int k = 0; k < 3; ++k) s += V[i][k] * std::max(w[k], 0.0) * V[j][k];
          Bp[i][j] = s;
        }
      double WT[3][3];
      transpose(G.W, WT);
      matmul(G.W, Bp, tmp);
      matmul(tmp, WT, S);
    }
    double A[3][3];
    if (op.filter_mode == 2) {
      const double tau = S[0][0] + S[1][1] + S[2][2];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i][j] = (i == j ? 1.0 : 0.0) + 0.5 * tau * Mp[i][j];
    } else {
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i][j] = (i == j ? 1.0 : 0.0) + S[i][j];
    }
    double Ai[3][3], Aq[3];
    inv3(A, Ai);
    matvec(Ai, q, Aq);
    T = G.sigma / std::sqrt(det3(A)) * std::exp(-0.5 * dot3(q, Aq));
  }
  if (op.backbone == 1) T *= geer_factor(G, nn);
  res.T_raw = T;
  res.T = (ts <= (double)op.t_near) ? 0.0 : T;
  return res;
}

// ----------------------------------------------------------------------------- depth order
// Eq. 4 composites front to back.  One key per Gaussian and view: the squared distance
// |mu - o|^2 of the mean from the camera centre, in double precision from the float32
// inputs (the differences and squares of float32 values are exact in double up to the
// last rounding).  Equal keys keep the index order.

double depth_key(const orc_gaussians& g, int64_t i, const float o[3]) {
  const int64_t n = g.n;
  double s = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double v = (double)g.means[k * n + i] - (double)o[k];
    s += v * v;
  }
  return s;
}

std::vector<int64_t> depth_order(const std::vector<double>& key) {
  std::vector<int64_t> idx(key.size());
  for (size_t i = 0; i < key.size(); ++i) idx[i] = (int64_t)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
  return idx;
}

// ----------------------------------------------------------------------------- view setup

struct ViewGauss {
  std::vector<GaussPre> pre;   // by Gaussian index
  std::vector<double> col;     // [n][3]
  std::vector<double> key;     // depth key |mu - o|^2 by Gaussian index
  std::vector<int64_t> order;  // compositing order
};

ViewGauss setup_view(const orc_gaussians& g, const orc_camera& c, const orc_opts& op) {
  ViewGauss v;
  v.pre.resize(g.n);
  v.col.resize(3 * g.n);
  const double o[3] = {c.origin[0], c.origin[1], c.origin[2]};
  for (int64_t i = 0; i < g.n; ++i) {
    const double rho2 = g.rho2 ? (double)g.rho2[i] : 0.0;
    v.pre[i] = preprocess(raw_of(g, i), rho2, op.use_floor != 0);
    gauss_color(g, i, v.pre[i].mu, o, &v.col[3 * i]);
  }
  v.key.resize(g.n);
  for (int64_t i = 0; i < g.n; ++i) v.key[i] = depth_key(g, i, c.origin);
  v.order = depth_order(v.key);
  return v;
}

// ----------------------------------------------------------------------------- compositing
// Eq. 4, front to back.  A "decision" is a comparison whose outcome could differ
// between this FP64 evaluation and an FP32 one because its operands are within a
// small relative band of the threshold.  The first few such decisions are recorded;
// `flip` forces the opposite outcome of one of them, giving the alternative result
// an FP32 renderer may legitimately produce.  With `key` given (the per-Gaussian
// order), two consecutive composited Gaussians whose keys lie within the band that
// float32 rounding of |mu - o|^2 can cross are an order decision too: their
// alternative is the composite with the two swapped in `cand`.

constexpr double kBandAlpha = 2e-4;  // relative band around alpha_min
constexpr double kBandTmin = 2e-4;   // relative band around T_min for T*(1 - alpha)
constexpr double kBandNear = 1e-5;   // relative band around t_near for t*
// relative band of the depth key: a float32 |mu - o|^2 (three rounded differences,
// three squares, two sums) is within about 5 units of 2^-24 of the exact value, so
// two keys can swap order only when they differ by less than about 6e-7 relative
constexpr double kBandKey = 1e-6;
constexpr int kMaxDecisions = 4;

// kind: 0 t_near, 1 alpha_min, 2 T_min, 3 key order (pa, pb: positions in cand)
struct Decision { int64_t k; int kind; int64_t pa, pb; };

struct CompositeOut {
  double rgba[4];
  int n_dec;
  Decision dec[kMaxDecisions];
  int64_t n_contrib;
};

template <class PairFn>
CompositeOut composite(const std::vector<int64_t>& cand, const ViewGauss& vg, const orc_opts& op, PairFn pair,
                       const double* key, int flip /* -1 none */) {
  CompositeOut out;
  out.n_dec = 0;
  out.n_contrib = 0;
  double Ttr = 1.0, C[3] = {0, 0, 0};
  int dec_counter = 0;
  auto decide = [&](bool outcome, bool near, int64_t k, int kind) {
    if (near) {
      const int id = dec_counter++;
      if (out.n_dec < kMaxDecisions) out.dec[out.n_dec++] = Decision{k, kind, -1, -1};
      if (id == flip) return !outcome;
    }
    return outcome;
  };
  const double amin = op.alpha_min, amax = op.alpha_max, tmin = op.T_min, tnear = op.t_near;
  int64_t prev = -1;  // position of the last composited pair
  for (int64_t pos = 0; pos < (int64_t)cand.size(); ++pos) {
    const int64_t k = cand[pos];
    const PairResult pr = pair(k);
    double T = pr.T_raw;
    // t_near cut: only a decision that matters when the uncut pair would contribute.
    const bool cut = pr.tstar <= tnear;
    const bool near_cut = std::fabs(pr.tstar - tnear) <= kBandNear * std::max(1.0, std::fabs(pr.tstar)) &&
                          std::min(T, amax) >= amin * (1.0 - kBandAlpha);
    if (decide(cut, near_cut, k, 0)) continue;
    const double alpha = std::min(T, amax);
    const bool skip = alpha < amin;
    const bool near_skip = std::fabs(alpha - amin) <= kBandAlpha * amin;
    if (decide(skip, near_skip, k, 1)) continue;
    if (key && prev >= 0) {
      const double ka = key[cand[prev]], kb = key[k];
      if (kb - ka <= kBandKey * std::max(ka, kb)) {
        const int id = dec_counter++;
        if (out.n_dec < kMaxDecisions) out.dec[out.n_dec++] = Decision{k, 3, prev, pos};
        (void)id;
      }
    }
    const double test = Ttr * (1.0 - alpha);
    const bool stop = test < tmin;
    const bool near_stop = std::fabs(test - tmin) <= kBandTmin * tmin;
    if (decide(stop, near_stop, k, 2)) break;
    const double* col = &vg.col[3 * k];
    for (int c = 0; c < 3; ++c) C[c] += Ttr * alpha * col[c];
    Ttr = test;
    prev = pos;
    out.n_contrib++;
  }
  for (int c = 0; c < 3; ++c) out.rgba[c] = C[c] + Ttr * (double)op.bg[c];
  out.rgba[3] = 1.0 - Ttr;
  return out;
}

// Per-ray compositing order (the front-to-back order of Eq. 4 by each pair's own
// max-response depth t* along this pixel's ray, Sec. 3): the candidates stably sorted
// by t*, so equal depths keep the per-Gaussian key order.  Two pairs that can both
// composite and whose t* lie within a small relative band are a decision: an FP32
// renderer may order them either way; swap_at[j] is the earlier one's position.
constexpr double kBandOrder = 1e-5;

struct RayOrder {
  std::vector<int64_t> list;
  int n_dec;
  int64_t swap_a[kMaxDecisions], swap_b[kMaxDecisions];
};

template <class PairFn>
RayOrder ray_order(const std::vector<int64_t>& cand, const orc_opts& op, PairFn pair) {
  struct Item { double t; int64_t k; bool live; };
  std::vector<Item> items;
  items.reserve(cand.size());
  for (int64_t k : cand) {
    const PairResult pr = pair(k);
    const bool live = pr.tstar > op.t_near * (1.0 - kBandNear) &&
                      std::min(pr.T_raw, (double)op.alpha_max) >= op.alpha_min * (1.0 - kBandAlpha);
    items.push_back(Item{pr.tstar, k, live});
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.t < b.t; });
  RayOrder ro;
  ro.n_dec = 0;
  ro.list.reserve(items.size());
  int64_t prev = -1;
  for (size_t q = 0; q < items.size(); ++q) {
    ro.list.push_back(items[q].k);
    if (!items[q].live) continue;
    if (prev >= 0 && ro.n_dec < kMaxDecisions &&
        std::fabs(items[q].t - items[prev].t) <= kBandOrder * std::max(1.0, std::fabs(items[q].t))) {
      ro.swap_a[ro.n_dec] = prev;
      ro.swap_b[ro.n_dec] = (int64_t)q;
      ro.n_dec++;
    }
    prev = (int64_t)q;
  }
  return ro;
}

// ----------------------------------------------------------------------------- culling grid
// Culled mode restricts each pixel's candidate list with a latitude-longitude grid of
// directions around the camera centre.  A Gaussian is entered in every cell that may
// hold a direction d with T >= alpha_min, using two facts about the filtered exponent
// Q = q^T A^{-1} q <= L = 2 ln(sigma_eff / alpha_min):
//  * the max-response point o + t* d is within rho of the mean, rho = s'_max sqrt(L (1 +
//    t*^2 c / s'_min^2)) with t* <= |v| + rho (c: largest pixel footprint coefficient
//    (|d_x - d|^2 + |d_y - d|^2) / 3 of the view), because |W^{-1} q| <= s'_max |q| and
//    lambda_max(A) <= 1 + tr Sigma_fp^u;
//  * Q is the ray's Mahalanobis distance to N(mu, Sigma_eff + footprint covariance), so
//    the perpendicular distance p of mu from the ray has p^2 <= L (s'_max^2 + t*^2 c).
// Rays meeting the ball B(mu, rho) at positive t lie in the cone asin(rho / |v|) when
// |v| > rho; the cone half-angle is asin(min(p, rho) / |v|).

struct Cone { double axis[3]; double half; bool all; };

Cone influence_cone(const GaussPre& G, const double o[3], double cmax, const orc_opts& op) {
  Cone cn;
  cn.all = false;
  double v[3] = {G.mu[0] - o[0], G.mu[1] - o[1], G.mu[2] - o[2]};
  const double dist = std::sqrt(dot3(v, v));
  for (int k = 0; k < 3; ++k) cn.axis[k] = dist > 0 ? v[k] / dist : 0.0;
  cn.half = kPi;
  const double smax = std::max(G.sp[0], std::max(G.sp[1], G.sp[2]));
  const double smin = std::min(G.sp[0], std::min(G.sp[1], G.sp[2]));
  // the ray-integral factor is at most s'_max / (geometric mean of s') (|d_u| >= 1/s'_max)
  const double sig_b = G.sigma * (op.backbone == 1 ? smax / std::cbrt(G.sp[0] * G.sp[1] * G.sp[2]) : 1.0);
  if (sig_b <= op.alpha_min) { cn.half = -1.0; return cn; }  // never reaches alpha_min
  if (dist <= 0) { cn.all = true; return cn; }
  const double L = 2.0 * std::log(sig_b / op.alpha_min);
  const double r = smax / smin;
  const double c = (op.filter_mode == 0) ? 0.0 : cmax;
  // Isotropic mode spreads the in-plane trace over both whitened directions, so its
  // world-space marginal variance is bounded by s'_max^2 (1 + tau/2) <= s'_max^2 + t*^2 c r^2 / 2.
  const double c_perp = (op.filter_mode == 2) ? c * r * r / 2.0 : c;
  const double a = L * smax * smax, k = c / (smin * smin), ak = a * k;
  if (ak >= 0.999) { cn.all = true; return cn; }
  const double rho = (ak * dist + std::sqrt(ak * dist * ak * dist + (1.0 - ak) * a * (1.0 + k * dist * dist))) /
                     (1.0 - ak) * (1.0 + 1e-9);
  if (dist + rho <= op.t_near) { cn.half = -1.0; return cn; }  // every t* <= t_near
  if (dist <= rho) { cn.all = true; return cn; }
  const double tmax = dist + rho;
  const double p = std::sqrt(L * (smax * smax + tmax * tmax * c_perp)) * (1.0 + 1e-9);
  cn.half = std::asin(std::min(p, rho) / dist);
  return cn;
}

struct LatLonGrid {
  int nlat, nlon;
  std::vector<std::vector<int64_t>> cells;  // per cell, candidate Gaussians in compositing order
  std::vector<int64_t> everywhere;          // Gaussians with no finite cone, in compositing order
  std::vector<int64_t> rank;                // position of each Gaussian in the compositing order
  // Candidates of the cell holding d: the cell's list merged with `everywhere` by rank.
  void candidates(const double d[3], std::vector<int64_t>& out) const {
    const std::vector<int64_t>& a = cells[cell_of(d)];
    out.clear();
    size_t i = 0, j = 0;
    while (i < a.size() || j < everywhere.size()) {
      if (j == everywhere.size() || (i < a.size() && rank[a[i]] < rank[everywhere[j]])) out.push_back(a[i++]);
      else out.push_back(everywhere[j++]);
    }
  }
  int cell_of(const double d[3]) const {
    const double lat = std::asin(std::max(-1.0, std::min(1.0, d[2])));
    double lon = std::atan2(d[1], d[0]);
    int a = (int)std::floor((lat + kPi / 2) / kPi * nlat);
    int b = (int)std::floor((lon + kPi) / (2 * kPi) * nlon);
    a = std::min(std::max(a, 0), nlat - 1);
    b = std::min(std::max(b, 0), nlon - 1);
    return a * nlon + b;
  }
};

LatLonGrid build_grid(const ViewGauss& vg, const orc_camera& cam, double cmax, const orc_opts& op, int nlat, int nlon) {
  LatLonGrid grid;
  grid.nlat = nlat;
  grid.nlon = nlon;
  grid.cells.assign((size_t)nlat * nlon, {});
  grid.rank.assign(vg.order.size(), 0);
  for (size_t r = 0; r < vg.order.size(); ++r) grid.rank[vg.order[r]] = (int64_t)r;
  const double o[3] = {cam.origin[0], cam.origin[1], cam.origin[2]};
  const double dlat = kPi / nlat, dlon = 2 * kPi / nlon;
  for (int64_t k : vg.order) {
    const Cone cn = influence_cone(vg.pre[k], o, cmax, op);
    if (cn.half < 0) continue;
    if (cn.all) {
      grid.everywhere.push_back(k);
      continue;
    }
    // Spherical cap -> enclosing latitude band and longitude interval (with a margin).
    const double margin = 1e-9;
    const double lat0 = std::asin(std::max(-1.0, std::min(1.0, cn.axis[2])));
    const double lon0 = std::atan2(cn.axis[1], cn.axis[0]);
    const double h = cn.half + margin;
    const double la = lat0 - h, lb = lat0 + h;
    int a0 = (int)std::floor((la + kPi / 2) / dlat), a1 = (int)std::floor((lb + kPi / 2) / dlat);
    a0 = std::max(a0, 0);
    a1 = std::min(a1, nlat - 1);
    bool all_lon = (la <= -kPi / 2) || (lb >= kPi / 2);
    double hw = kPi;
    if (!all_lon) {
      const double s = std::sin(h) / std::cos(lat0);
      if (s >= 1.0) all_lon = true; else hw = std::asin(s) + margin;
    }
    for (int a = a0; a <= a1; ++a) {
      if (all_lon) {
        for (int b = 0; b < nlon; ++b) grid.cells[(size_t)a * nlon + b].push_back(k);
        continue;
      }
      const int b0 = (int)std::floor((lon0 - hw + kPi) / dlon);
      const int b1 = (int)std::floor((lon0 + hw + kPi) / dlon);
      for (int bb = b0; bb <= b1; ++bb) {
        const int b = ((bb % nlon) + nlon) % nlon;
        auto& cell = grid.cells[(size_t)a * nlon + b];
        if (cell.empty() || cell.back() != k) cell.push_back(k);
      }
    }
  }
  return grid;
}

double view_max_footprint(const orc_camera& c, double fs) {
  double cmax = 0.0;
#pragma omp parallel for reduction(max : cmax) schedule(static)
  for (int j = 0; j < c.crop_h; ++j)
    for (int i = 0; i < c.crop_w; ++i) {
      const PixelRays r = pixel_rays(c, c.crop_x0 + i + 0.5, c.crop_y0 + j + 0.5);
      if (!r.valid) continue;
      double s = 0.0;
      for (int k = 0; k < 3; ++k) {
        s += (r.dx[k] - r.d[k]) * (r.dx[k] - r.d[k]);
        s += (r.dy[k] - r.d[k]) * (r.dy[k] - r.d[k]);
      }
      cmax = std::max(cmax, s * fs * fs / 3.0);
    }
  return cmax;
}

int num_threads_for(int req) {
#ifdef _OPENMP
  return req > 0 ? req : omp_get_max_threads();
#else
  (void)req;
  return 1;
#endif
}

}  // namespace

// ============================================================================= C entry points
extern "C" {

int orc_version(void) { return 1; }

// Pi^{-1} for n continuous pixel coordinates (px[i], py[i]) of the full image.
void orc_unproject(const orc_camera* cam, int64_t n, const double* px, const double* py, double* dirs /*[n][3]*/,
                   uint8_t* valid) {
  for (int64_t i = 0; i < n; ++i) {
    double d[3] = {0, 0, 0};
    const bool ok = unproject(*cam, px[i], py[i], d);
    valid[i] = ok ? 1 : 0;
    for (int k = 0; k < 3; ++k) dirs[3 * i + k] = ok ? d[k] : 0.0;
  }
}

// Pi for n world directions.
void orc_project(const orc_camera* cam, int64_t n, const double* dirs, double* px, double* py, uint8_t* valid) {
  for (int64_t i = 0; i < n; ++i) {
    double x = 0, y = 0;
    const bool ok = project(*cam, &dirs[3 * i], &x, &y);
    valid[i] = ok ? 1 : 0;
    px[i] = x;
    py[i] = y;
  }
}

// Centre and edge rays of the crop pixels: out [n_px][9] = d, d_x, d_y; valid [n_px].
void orc_pixel_rays(const orc_camera* cam, double* out, uint8_t* valid) {
  const orc_camera& c = *cam;
  for (int j = 0; j < c.crop_h; ++j)
    for (int i = 0; i < c.crop_w; ++i) {
      const int64_t p = (int64_t)j * c.crop_w + i;
      const PixelRays r = pixel_rays(c, c.crop_x0 + i + 0.5, c.crop_y0 + j + 0.5);
      valid[p] = r.valid;
      for (int k = 0; k < 3; ++k) {
        out[9 * p + k] = r.valid ? r.d[k] : 0.0;
        out[9 * p + 3 + k] = r.valid ? r.dx[k] : 0.0;
        out[9 * p + 6 + k] = r.valid ? r.dy[k] : 0.0;
      }
    }
}

// Real SH basis (16 values) at a direction.
void orc_sh_basis(const double* dir, double* Y) { sh_basis(dir, Y); }

// Per-Gaussian preprocessing for one camera centre: out [n][8] =
// (s'_0, s'_1, s'_2, sigma_eff, r, g, b, depth key |mu - o|^2), W [n][9] row-major.
void orc_preprocess(const orc_gaussians* g, const float* origin, const orc_opts* op, double* out, double* W) {
  const double o[3] = {origin[0], origin[1], origin[2]};
  for (int64_t i = 0; i < g->n; ++i) {
    const double rho2 = g->rho2 ? (double)g->rho2[i] : 0.0;
    const GaussPre p = preprocess(raw_of(*g, i), rho2, op->use_floor != 0);
    double col[3];
    gauss_color(*g, i, p.mu, o, col);
    out[8 * i + 0] = p.sp[0]; out[8 * i + 1] = p.sp[1]; out[8 * i + 2] = p.sp[2];
    out[8 * i + 3] = p.sigma;
    out[8 * i + 4] = col[0]; out[8 * i + 5] = col[1]; out[8 * i + 6] = col[2];
    out[8 * i + 7] = depth_key(*g, i, origin);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) W[9 * i + 3 * a + b] = p.W[a][b];
  }
}

// Response of Gaussian gi to n rays from origin: rays [n][9] = (d, d_x, d_y).
// out [n][4] = (T, T ignoring t_near, t*, D^2).
void orc_pair_batch(const orc_gaussians* g, int64_t gi, const double* origin, int64_t n, const double* rays,
                    const orc_opts* op, double* out) {
  const double rho2 = g->rho2 ? (double)g->rho2[gi] : 0.0;
  const GaussPre p = preprocess(raw_of(*g, gi), rho2, op->use_floor != 0);
  for (int64_t i = 0; i < n; ++i) {
    const PairResult r = pair_response(p, origin, &rays[9 * i], &rays[9 * i + 3], &rays[9 * i + 6], *op);
    out[4 * i + 0] = r.T;
    out[4 * i + 1] = r.T_raw;
    out[4 * i + 2] = r.tstar;
    out[4 * i + 3] = r.D2;
  }
}

// Full render of one view.
//   mode 0: brute force (every Gaussian for every pixel); mode 1: lat-long culled.
//   rgba [crop_h][crop_w][4]; n_dec [px] = number of near-threshold decisions seen;
//   alt [px][kMaxDecisions][4] = result with decision j flipped (j < min(n_dec, 4));
//   n_contrib [px] = contributing pairs.  alt / n_dec / n_contrib may be NULL.
//   skip_px [px] (may be NULL): set when the pixel's validity is itself ambiguous.
int orc_render(const orc_gaussians* g, const orc_camera* cam, const orc_opts* op, int mode, int n_threads,
               double* rgba, int32_t* n_dec, double* alt, int64_t* n_contrib, uint8_t* skip_px) {
  const orc_camera& c = *cam;
  const ViewGauss vg = setup_view(*g, c, *op);
  const double o[3] = {c.origin[0], c.origin[1], c.origin[2]};
  LatLonGrid grid;
  if (mode == 1) {
    const double cmax = view_max_footprint(c, op->footprint_scale) * 1.0001;
    grid = build_grid(vg, c, cmax, *op, 256, 512);
  }
  const int64_t npx = (int64_t)c.crop_w * c.crop_h;
  const double thd_max = (c.model == 1) ? kb_theta_d(c, c.theta_max) : 0.0;
#pragma omp parallel for schedule(dynamic, 4) num_threads(num_threads_for(n_threads))
  for (int j = 0; j < c.crop_h; ++j) {
    for (int i = 0; i < c.crop_w; ++i) {
      const int64_t p = (int64_t)j * c.crop_w + i;
      const double px = c.crop_x0 + i + 0.5, py = c.crop_y0 + j + 0.5;
      if (skip_px) {
        skip_px[p] = 0;
        if (c.model == 1) {
          const double mx = (px - c.cx) / c.fx, my = (py - c.cy) / c.fy;
          const double thd = std::sqrt(mx * mx + my * my);
          // centre or edge ray within a hair of the valid-domain boundary
          auto near_edge = [&](double x, double y) {
            const double ax = (x - c.cx) / c.fx, ay = (y - c.cy) / c.fy;
            return std::fabs(std::sqrt(ax * ax + ay * ay) - thd_max) <= 1e-9 * thd_max;
          };
          if (near_edge(px, py) || near_edge(px + 0.5, py) || near_edge(px, py + 0.5)) skip_px[p] = 1;
          (void)thd;
        }
      }
      const PixelRays r = pixel_rays(c, px, py);
      if (!r.valid) {
        for (int k = 0; k < 3; ++k) rgba[4 * p + k] = op->bg[k];
        rgba[4 * p + 3] = 0.0;
        if (n_dec) n_dec[p] = 0;
        if (n_contrib) n_contrib[p] = 0;
        continue;
      }
      auto pair = [&](int64_t k) { return pair_response(vg.pre[k], o, r.d, r.dx, r.dy, *op); };
      std::vector<int64_t> culled;
      if (mode == 1) grid.candidates(r.d, culled);
      const std::vector<int64_t>& keyed = (mode == 1) ? culled : vg.order;
      // order_mode 1: this ray's own t* order, with its near-ties as the first decisions
      RayOrder ro;
      ro.n_dec = 0;
      if (op->order_mode == 1) ro = ray_order(keyed, *op, pair);
      const std::vector<int64_t>& cand = (op->order_mode == 1) ? ro.list : keyed;
      const double* key = (op->order_mode == 0) ? vg.key.data() : nullptr;
      const CompositeOut co = composite(cand, vg, *op, pair, key, -1);
      const int n_all = std::min(kMaxDecisions, ro.n_dec + co.n_dec);
      for (int k = 0; k < 4; ++k) rgba[4 * p + k] = co.rgba[k];
      if (n_dec) n_dec[p] = n_all;
      if (n_contrib) n_contrib[p] = co.n_contrib;
      if (alt) {
        for (int f = 0; f < kMaxDecisions; ++f) {
          CompositeOut ca = co;
          if (f < ro.n_dec) {
            std::vector<int64_t> swapped = ro.list;
            std::swap(swapped[ro.swap_a[f]], swapped[ro.swap_b[f]]);
            ca = composite(swapped, vg, *op, pair, nullptr, -1);
          } else if (f < n_all) {
            const Decision& dd = co.dec[f - ro.n_dec];
            if (dd.kind == 3) {
              std::vector<int64_t> swapped = cand;
              std::swap(swapped[dd.pa], swapped[dd.pb]);
              ca = composite(swapped, vg, *op, pair, nullptr, -1);
            } else {
              ca = composite(cand, vg, *op, pair, key, f - ro.n_dec);
            }
          }
          for (int k = 0; k < 4; ++k) alt[(p * kMaxDecisions + f) * 4 + k] = ca.rgba[k];
        }
      }
    }
  }
  (void)npx;
  return 0;
}

// Eq. 5 reference: average of centre-ray renders (filter off, same floor) over
// sub-pixel offsets xi in [-1/2, 1/2]^2.  jitter [n_sub][2].  Sub-rays outside the
// valid domain contribute (bg, 0).
int orc_render_supersampled(const orc_gaussians* g, const orc_camera* cam, const orc_opts* op_in, int64_t n_sub,
                            const double* jitter, int n_threads, double* rgba) {
  const orc_camera& c = *cam;
  orc_opts op = *op_in;
  op.filter_mode = 0;
  const ViewGauss vg = setup_view(*g, c, op);
  const double o[3] = {c.origin[0], c.origin[1], c.origin[2]};
#pragma omp parallel for schedule(dynamic, 1) num_threads(num_threads_for(n_threads))
  for (int j = 0; j < c.crop_h; ++j) {
    for (int i = 0; i < c.crop_w; ++i) {
      const int64_t p = (int64_t)j * c.crop_w + i;
      double acc[4] = {0, 0, 0, 0};
      for (int64_t s = 0; s < n_sub; ++s) {
        double d[3];
        const double px = c.crop_x0 + i + 0.5 + jitter[2 * s], py = c.crop_y0 + j + 0.5 + jitter[2 * s + 1];
        if (!unproject(c, px, py, d)) {
          for (int k = 0; k < 3; ++k) acc[k] += op.bg[k];
          continue;
        }
        auto pair = [&](int64_t k) { return pair_response(vg.pre[k], o, d, d, d, op); };
        const CompositeOut co =
            composite(op.order_mode == 1 ? ray_order(vg.order, op, pair).list : vg.order, vg, op, pair, nullptr, -1);
        for (int k = 0; k < 4; ++k) acc[k] += co.rgba[k];
      }
      for (int k = 0; k < 4; ++k) rgba[4 * p + k] = acc[k] / (double)n_sub;
    }
  }
  return 0;
}

// Eq. 11: rho^2 = min over views in which the Gaussian is visible of half the trace
// of the world-space footprint covariance at the pixel the mean projects to.
//   e_i = t (I - d d^T)(d_i - d),  d = unit direction to the mean, t = |mu - o|,
//   d_i = Pi^{-1}(Pi(mu) + Delta_i) (backward offset if the forward one is invalid),
//   half trace = (|e_x|^2 + |e_y|^2) / 6.
// Visible: Pi(mu) valid and inside the full image, and t > t_near.  No visible view
// gives rho^2 = 0.
void orc_bake_rho2(const orc_gaussians* g, const orc_camera* cams, int32_t n_cams, float t_near, int n_threads,
                   double* rho2_out) {
#pragma omp parallel for schedule(static) num_threads(num_threads_for(n_threads))
  for (int64_t i = 0; i < g->n; ++i) {
    double best = -1.0;
    for (int v = 0; v < n_cams; ++v) {
      const orc_camera& c = cams[v];
      double vv[3];
      for (int k = 0; k < 3; ++k) vv[k] = (double)g->means[k * g->n + i] - (double)c.origin[k];
      const double t = std::sqrt(dot3(vv, vv));
      if (!(t > t_near)) continue;
      double d[3] = {vv[0] / t, vv[1] / t, vv[2] / t};
      double x, y;
      if (!project(c, d, &x, &y)) continue;
      if (!(x >= 0 && x < c.full_w && y >= 0 && y < c.full_h)) continue;
      double di[2][3];
      bool ok = true;
      const double offs[2][2] = {{0.5, 0.0}, {0.0, 0.5}};
      for (int a = 0; a < 2; ++a) {
        if (!unproject(c, x + offs[a][0], y + offs[a][1], di[a]) &&
            !unproject(c, x - offs[a][0], y - offs[a][1], di[a]))
          ok = false;
      }
      if (!ok) continue;
      double ht = 0.0;
      for (int a = 0; a < 2; ++a) {
        double dd[3] = {di[a][0] - d[0], di[a][1] - d[1], di[a][2] - d[2]};
        const double along = dot3(d, dd);
        double e[3];
        for (int k = 0; k < 3; ++k) e[k] = t * (dd[k] - along * d[k]);
        ht += dot3(e, e);
      }
      ht /= 6.0;
      if (best < 0 || ht < best) best = ht;
    }
    rho2_out[i] = best < 0 ? 0.0 : best;
  }
}

// Gradients of L = sum_px sum_ch grad_rgba * rgba with respect to the raw parameters
// (means, log-scales, quaternions, opacity logits, colour), one view.
// Compositing (Eq. 4) is differentiated exactly: with S_k the colour composited
// behind pair k, dL/dalpha_k = sum_ch G_ch (c_k T_k - (S_k + T_final bg) / (1 - alpha_k))
// + G_a T_final / (1 - alpha_k) and dL/dc_k = G alpha_k T_k.  The per-pair response
// T_k and the SH colour are differentiated by Richardson-extrapolated central
// differences of the FP64 functions above.  Outputs are ADDED to (accumulate views).
// skip_px [px] (may be NULL): pixels whose upstream gradient is ignored.
int orc_grad(const orc_gaussians* g, const orc_camera* cam, const orc_opts* op, const float* grad_rgba,
             const uint8_t* skip_px, int n_threads, double* d_means, double* d_log_scales, double* d_quats,
             double* d_opacity, double* d_color) {
  // the compositing derivative below follows the per-Gaussian key order only
  if (op->order_mode != 0) return -2;
  const orc_camera& c = *cam;
  const ViewGauss vg = setup_view(*g, c, *op);
  const double o[3] = {c.origin[0], c.origin[1], c.origin[2]};
  const int64_t n = g->n;
  const int ncol = g->color_mode == 0 ? 3 : 48;
  const int nthr = num_threads_for(n_threads);
  const int per = 11 + ncol;
  std::vector<double> acc((size_t)nthr * n * per, 0.0);

  auto raw_response = [&](const GaussRaw& r, int64_t k, const PixelRays& pr) {
    const double rho2 = g->rho2 ? (double)g->rho2[k] : 0.0;
    const GaussPre p = preprocess(r, rho2, op->use_floor != 0);
    return pair_response(p, o, pr.d, pr.dx, pr.dy, *op).T_raw;
  };
  auto raw_color = [&](const GaussRaw& r, int64_t k, double col[3]) { gauss_color(*g, k, r.mu, o, col); };

#pragma omp parallel for schedule(dynamic, 2) num_threads(nthr)
  for (int j = 0; j < c.crop_h; ++j) {
#ifdef _OPENMP
    const int tid = omp_get_thread_num();
#else
    const int tid = 0;
#endif
    double* A = &acc[(size_t)tid * n * per];
    for (int i = 0; i < c.crop_w; ++i) {
      const int64_t p = (int64_t)j * c.crop_w + i;
      if (skip_px && skip_px[p]) continue;
      const PixelRays r = pixel_rays(c, c.crop_x0 + i + 0.5, c.crop_y0 + j + 0.5);
      if (!r.valid) continue;
      const double G[4] = {grad_rgba[4 * p], grad_rgba[4 * p + 1], grad_rgba[4 * p + 2], grad_rgba[4 * p + 3]};
      // forward: contributing list
      struct Item { int64_t k; double T, alpha, Tk; bool clamped; };
      std::vector<Item> items;
      double Ttr = 1.0;
      for (int64_t k : vg.order) {
        const PairResult pr = pair_response(vg.pre[k], o, r.d, r.dx, r.dy, *op);
        if (pr.tstar <= op->t_near) continue;
        const double alpha = std::min(pr.T_raw, (double)op->alpha_max);
        if (alpha < op->alpha_min) continue;
        const double test = Ttr * (1.0 - alpha);
        if (test < op->T_min) break;
        items.push_back(Item{k, pr.T_raw, alpha, Ttr, pr.T_raw >= op->alpha_max});
        Ttr = test;
      }
      const double Tfin = Ttr;
      // suffix sums S_k of composited colour behind each item
      std::vector<double> S(3 * items.size() + 3, 0.0);
      for (int64_t m = (int64_t)items.size() - 1; m >= 0; --m) {
        const double* col = &vg.col[3 * items[m].k];
        for (int ch = 0; ch < 3; ++ch)
          S[3 * m + ch] = S[3 * (m + 1) + ch] + col[ch] * items[m].alpha * items[m].Tk;
      }
      for (size_t m = 0; m < items.size(); ++m) {
        const Item& it = items[m];
        const int64_t k = it.k;
        const double* col = &vg.col[3 * k];
        double dL_dalpha = G[3] * Tfin / (1.0 - it.alpha);
        for (int ch = 0; ch < 3; ++ch)
          dL_dalpha += G[ch] * (col[ch] * it.Tk - (S[3 * (m + 1) + ch] + Tfin * op->bg[ch]) / (1.0 - it.alpha));
        const double dL_dT = it.clamped ? 0.0 : dL_dalpha;
        double dL_dc[3];
        for (int ch = 0; ch < 3; ++ch) dL_dc[ch] = G[ch] * it.alpha * it.Tk;
        const GaussRaw base = raw_of(*g, k);
        double* Ak = &A[(size_t)k * per];
        // d T / d raw via Richardson-extrapolated central differences
        const double smin = std::exp(std::min(base.log_s[0], std::min(base.log_s[1], base.log_s[2])));
        const double rho2 = g->rho2 && op->use_floor ? (double)g->rho2[k] : 0.0;
        const double spmin = std::sqrt(smin * smin + rho2);
        const double qn = std::sqrt(base.quat[0] * base.quat[0] + base.quat[1] * base.quat[1] +
                                    base.quat[2] * base.quat[2] + base.quat[3] * base.quat[3]);
        for (int pidx = 0; pidx < 11; ++pidx) {
          double h;
          if (pidx < 3) h = 1e-3 * spmin;
          else if (pidx < 6) h = 1e-3;
          else if (pidx < 10) h = 1e-3 * qn;
          else h = 1e-3;
          auto f = [&](double delta) {
            GaussRaw rr = base;
            if (pidx < 3) rr.mu[pidx] += delta;
            else if (pidx < 6) rr.log_s[pidx - 3] += delta;
            else if (pidx < 10) rr.quat[pidx - 6] += delta;
            else rr.logit += delta;
            return raw_response(rr, k, r);
          };
          const double D1 = (f(h) - f(-h)) / (2 * h);
          const double D2 = (f(h / 2) - f(-h / 2)) / h;
          const double dT = (4 * D2 - D1) / 3;
          Ak[pidx] += dL_dT * dT;
        }
        // colour
        if (g->color_mode == 0) {
          for (int ch = 0; ch < 3; ++ch) Ak[11 + ch] += dL_dc[ch];
        } else {
          double Y[16];
          bool clamped[3];
          double colv[3];
          gauss_color(*g, k, base.mu, o, colv, Y, clamped);
          for (int ch = 0; ch < 3; ++ch) {
            if (clamped[ch]) continue;
            for (int cf = 0; cf < 16; ++cf) Ak[11 + 3 * cf + ch] += dL_dc[ch] * Y[cf];
          }
          // colour through the viewing direction (means)
          const double h = 1e-3 * spmin;
          for (int a = 0; a < 3; ++a) {
            auto fc = [&](double delta, double out3[3]) {
              GaussRaw rr = base;
              rr.mu[a] += delta;
              raw_color(rr, k, out3);
            };
            double cp[3], cm[3], cp2[3], cm2[3];
            fc(h, cp); fc(-h, cm); fc(h / 2, cp2); fc(-h / 2, cm2);
            for (int ch = 0; ch < 3; ++ch) {
              const double D1 = (cp[ch] - cm[ch]) / (2 * h);
              const double D2 = (cp2[ch] - cm2[ch]) / h;
              Ak[a] += dL_dc[ch] * (4 * D2 - D1) / 3;
            }
          }
        }
      }
    }
  }
  for (int t = 0; t < nthr; ++t) {
    const double* A = &acc[(size_t)t * n * per];
    for (int64_t k = 0; k < n; ++k) {
      const double* Ak = &A[(size_t)k * per];
      for (int a = 0; a < 3; ++a) d_means[a * n + k] += Ak[a];
      for (int a = 0; a < 3; ++a) d_log_scales[a * n + k] += Ak[3 + a];
      for (int a = 0; a < 4; ++a) d_quats[a * n + k] += Ak[6 + a];
      d_opacity[k] += Ak[10];
      for (int a = 0; a < ncol; ++a) d_color[a * n + k] += Ak[11 + a];
    }
  }
  return 0;
}

}  // extern "C"
