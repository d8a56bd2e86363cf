// Reverse mode of the per-pair filtered response (pair_math.hpp), used by the tile
// backward only.
#pragma once

#include "pair_math.hpp"

namespace cg {

// ---------------------------------------------------------------------------- backward
// Gradient of one pair's response T with respect to its record: dL/dT = dT is given;
// the result is written to g[0..15] = (dW[9], dmu[3], dsigma, dsp2[3]).  gm, ft, fl
// and filt are the forward intermediates left by pair_cheap and pair_full_keep for this
// pair; every step is differentiated in reverse order.  G = g(Phi) (the marginal
// composition) is differentiated in closed form: with both eigenvalues above rho^2,
// G = I - rho^2 Phi^{-1}; with one, G = g+ u u^T (u the leading eigenvector); at the
// clamp kink the clamped branch's (zero) derivative is used.
template <int FILTER, bool MARGINAL, bool GEER>
__device__ __forceinline__ void pair_grad(const Record& R, const PairPixel& p, const PairGeom& gm, const PairFoot& ft,
                                          const PairFloor& fl, bool filt, float dT, float T,
                                          float* __restrict__ g) {
  const float* W = R.W;
  const float wx = gm.wx, wy = gm.wy, wz = gm.wz;
  const float yx = gm.yx, yy = gm.yy, yz = gm.yz;
  const float ya = gm.ya;
  const float f = ya * gm.rn;

  // adjoints
  // reverse mode only: hardware reciprocals are accurate enough for the gradients
  float dsig = dT * T * fast_rcp(R.sigma);
  const float dlogT = dT * T;
  float dD2 = 0.f;
  float dq0 = 0.f, dq1 = 0.f, dq2 = 0.f;
  float dts = 0.f;
  float da0 = 0.f, da1 = 0.f, da2 = 0.f, drn = 0.f;
  float dW[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) dW[k] = 0.f;
  float dsp0 = 0.f, dsp1 = 0.f, dsp2 = 0.f;
  // ray-integral backbone: T carries sqrt(rn) = 1 / |a|
  if (GEER) drn += 0.5f * dlogT * fast_rcp(gm.rn);

  if (FILTER == 0) {
    dD2 = -0.5f * dlogT;
  } else {
    const float G11 = fl.G11, G12 = fl.G12, G22 = fl.G22;
    const float P11 = fl.P11, P12 = fl.P12, P22 = fl.P22, lp = fl.lp, rr = fl.rr, gp = fl.gp;
    float c2 = 0.f, s2 = 0.f, detP = 0.f;
    int gcase = 0;  // 0: no floor; 1: G = I - rho^2 Phi^-1; 2: G = g+ u u^T; 3: G = 0
    const bool floor_on = MARGINAL && R.rho2 > 0.f;
    if (floor_on) {
      if (!filt) {
        gcase = 3;
      } else if (fl.lm > R.rho2) {
        gcase = 1;
        detP = P11 * P22 - P12 * P12;
      } else {
        gcase = 2;
        const float irr = fast_rcp(rr);
        c2 = fl.dd * irr;
        s2 = P12 * irr;
      }
    }
    float dK11 = 0.f, dK12 = 0.f, dK22 = 0.f, dh1 = 0.f, dh2 = 0.f;
    float dG11 = 0.f, dG12 = 0.f, dG22 = 0.f;
    if (!filt) {
      dD2 = -0.5f * dlogT;
    } else if (FILTER == 2) {
      const float tau = floor_on ? (G11 * ft.K11 + 2.f * G12 * ft.K12 + G22 * ft.K22) : (ft.K11 + ft.K22);
      const float s = 1.f + 0.5f * tau;
      const float is = fast_rcp(s);
      dD2 = -0.5f * is * dlogT;
      const float ds = dlogT * (-is + 0.5f * gm.D2 * is * is);
      const float dtau = 0.5f * ds;
      if (floor_on) {
        dK11 += dtau * G11; dK12 += 2.f * dtau * G12; dK22 += dtau * G22;
        dG11 += dtau * ft.K11; dG12 += 2.f * dtau * ft.K12; dG22 += dtau * ft.K22;
      } else {
        dK11 += dtau; dK22 += dtau;
      }
    } else {
      // log T = log sigma - (log det M) / 2 - (D^2 - quad) / 2 with M = I + K G and
      // quad = h^T G M^{-1} h (Eq. 9 in the 2x2 form).  With w = M^{-1} h, z = G w and the
      // symmetric B = G M^{-1}, C = M^{-1} K:
      //   d log T / dK = -(B + z z^T) / 2,  d log T / dG = (w w^T - C) / 2,  d log T / dh = z,
      // where K12 and G12 each stand for both off-diagonal entries (counted twice).
      dD2 = -0.5f * dlogT;
      const float a = 0.5f * dlogT;
      if (floor_on) {
        const float M11 = 1.f + ft.K11 * G11 + ft.K12 * G12, M12 = ft.K11 * G12 + ft.K12 * G22;
        const float M21 = ft.K12 * G11 + ft.K22 * G12, M22 = 1.f + ft.K12 * G12 + ft.K22 * G22;
        const float idet = fast_rcp(M11 * M22 - M12 * M21);
        const float w1 = (M22 * ft.h1 - M12 * ft.h2) * idet, w2 = (M11 * ft.h2 - M21 * ft.h1) * idet;
        const float z1 = G11 * w1 + G12 * w2, z2 = G12 * w1 + G22 * w2;
        const float ai = a * idet;
        dK11 -= ai * (G11 * M22 - G12 * M21) + a * z1 * z1;
        dK12 -= 2.f * (ai * (G12 * M11 - G11 * M12) + a * z1 * z2);
        dK22 -= ai * (G22 * M11 - G12 * M12) + a * z2 * z2;
        dG11 += a * w1 * w1 - ai * (M22 * ft.K11 - M12 * ft.K12);
        dG12 += 2.f * (a * w1 * w2 - ai * (M22 * ft.K12 - M12 * ft.K22));
        dG22 += a * w2 * w2 - ai * (M11 * ft.K22 - M21 * ft.K12);
        dh1 += dlogT * z1;
        dh2 += dlogT * z2;
      } else {  // G = I: B = M^{-1}, z = w
        const float Q11 = 1.f + ft.K11, Q22 = 1.f + ft.K22, Q12 = ft.K12;
        const float idet = fast_rcp(Q11 * Q22 - Q12 * Q12);
        const float w1 = (Q22 * ft.h1 - Q12 * ft.h2) * idet, w2 = (Q11 * ft.h2 - Q12 * ft.h1) * idet;
        const float ai = a * idet;
        dK11 -= ai * Q22 + a * w1 * w1;
        dK12 += 2.f * (ai * Q12 - a * w1 * w2);
        dK22 -= ai * Q11 + a * w2 * w2;
        dh1 += dlogT * w1;
        dh2 += dlogT * w2;
      }
    }
    // G = g(Phi) -> Phi
    float dP11 = 0.f, dP12 = 0.f, dP22 = 0.f;
    if (gcase == 1) {
      // G11 = 1 - rho2 P22/det, G22 = 1 - rho2 P11/det, G12 = rho2 P12/det
      const float r2 = R.rho2, id = fast_rcp(detP);
      const float Gp11 = -r2 * P22 * id, Gp22 = -r2 * P11 * id, Gp12 = r2 * P12 * id;  // G - I
      // d(1/det) = -(P22 dP11 + P11 dP22 - 2 P12 dP12) / det^2
      const float s = dG11 * Gp11 + dG22 * Gp22 + dG12 * Gp12;  // sum dG * (G - I)
      dP11 += -dG22 * r2 * id - s * P22 * id;
      dP22 += -dG11 * r2 * id - s * P11 * id;
      dP12 += dG12 * r2 * id + 2.f * s * P12 * id;
    } else if (gcase == 2) {
      const float dgp = 0.5f * (dG11 * (1.f + c2) + dG22 * (1.f - c2) + dG12 * s2);
      const float dc2 = 0.5f * gp * (dG11 - dG22), ds2 = 0.5f * gp * dG12;
      const float ilp = fast_rcp(lp), irr = fast_rcp(rr);
      const float dlp = dgp * R.rho2 * ilp * ilp;
      float dm = dlp, drr = dlp;
      float ddd = dc2 * irr;
      drr += (-dc2 * c2 - ds2 * s2) * irr;
      float dpq = ds2 * irr;
      ddd += drr * c2;
      dpq += drr * s2;
      dP11 += 0.5f * (dm + ddd);
      dP22 += 0.5f * (dm - ddd);
      dP12 += dpq;
    }
    // Phi, K, h -> e_x, e_y, s'^2, q, with the factors 2/3, 1/3 and 1/sqrt 3 applied to
    // the coefficients once
    constexpr float third = 1.f / 3.f, two_thirds = 2.f / 3.f;
    constexpr float isq3 = 0.57735026918962576f;
    const float hx = dh1 * isq3, hy = dh2 * isq3;
    const float kxx = dK11 * two_thirds, kxy = dK12 * third, kyy = dK22 * two_thirds;
    // Phi = E^T S'^2 E / 3 adds the same terms weighted by s'^2 per component (dPhi is
    // zero unless the floor clamps, so these need no branch)
    const float pxx = dP11 * two_thirds, pxy = dP12 * third, pyy = dP22 * two_thirds;
    const float cxx0 = fmaf(pxx, R.sp2[0], kxx), cxx1 = fmaf(pxx, R.sp2[1], kxx), cxx2 = fmaf(pxx, R.sp2[2], kxx);
    const float cxy0 = fmaf(pxy, R.sp2[0], kxy), cxy1 = fmaf(pxy, R.sp2[1], kxy), cxy2 = fmaf(pxy, R.sp2[2], kxy);
    const float cyy0 = fmaf(pyy, R.sp2[0], kyy), cyy1 = fmaf(pyy, R.sp2[1], kyy), cyy2 = fmaf(pyy, R.sp2[2], kyy);
    const float qxx = dP11 * third, qyy = dP22 * third;
    dsp0 += ft.ex0 * (qxx * ft.ex0 + pxy * ft.ey0) + qyy * ft.ey0 * ft.ey0;
    dsp1 += ft.ex1 * (qxx * ft.ex1 + pxy * ft.ey1) + qyy * ft.ey1 * ft.ey1;
    dsp2 += ft.ex2 * (qxx * ft.ex2 + pxy * ft.ey2) + qyy * ft.ey2 * ft.ey2;
    const float dex0 = cxx0 * ft.ex0 + cxy0 * ft.ey0 + hx * gm.qx;
    const float dex1 = cxx1 * ft.ex1 + cxy1 * ft.ey1 + hx * gm.qy;
    const float dex2 = cxx2 * ft.ex2 + cxy2 * ft.ey2 + hx * gm.qz;
    const float dey0 = cyy0 * ft.ey0 + cxy0 * ft.ex0 + hy * gm.qx;
    const float dey1 = cyy1 * ft.ey1 + cxy1 * ft.ex1 + hy * gm.qy;
    const float dey2 = cyy2 * ft.ey2 + cxy2 * ft.ex2 + hy * gm.qz;
    dq0 += hx * ft.ex0 + hy * ft.ey0;
    dq1 += hx * ft.ex1 + hy * ft.ey1;
    dq2 += hx * ft.ex2 + hy * ft.ey2;
    // e_i = t* u_i with u_i = b_i - p_i a, p_i = (b_i . a) rn and b_i = W delta_i; the
    // forward recompute leaves e_i and b_i . a, so u_i = e_i / t* and b_i = u_i + p_i a
    const float t = gm.tstar, it = fast_rcp(t);
    const float bxa = ft.bxa, bya = ft.bya;
    const float px_ = bxa * gm.rn, py_ = bya * gm.rn;
    dts += (dex0 * ft.ex0 + dex1 * ft.ex1 + dex2 * ft.ex2 + dey0 * ft.ey0 + dey1 * ft.ey1 + dey2 * ft.ey2) * it;
    const float dux0 = t * dex0, dux1 = t * dex1, dux2 = t * dex2;
    const float duy0 = t * dey0, duy1 = t * dey1, duy2 = t * dey2;
    const float dpx = -(dux0 * gm.ax + dux1 * gm.ay + dux2 * gm.az);
    const float dpy = -(duy0 * gm.ax + duy1 * gm.ay + duy2 * gm.az);
    // (dpx b_x + dpy b_y) rn, with b_i = e_i / t* + p_i a
    const float ir = it * gm.rn, sa = (dpx * px_ + dpy * py_) * gm.rn;
    da0 += -px_ * dux0 - py_ * duy0 + (dpx * ft.ex0 + dpy * ft.ey0) * ir + sa * gm.ax;
    da1 += -px_ * dux1 - py_ * duy1 + (dpx * ft.ex1 + dpy * ft.ey1) * ir + sa * gm.ay;
    da2 += -px_ * dux2 - py_ * duy2 + (dpx * ft.ex2 + dpy * ft.ey2) * ir + sa * gm.az;
    drn += dpx * bxa + dpy * bya;
    const float dbx0 = dux0 + dpx * gm.rn * gm.ax, dbx1 = dux1 + dpx * gm.rn * gm.ay, dbx2 = dux2 + dpx * gm.rn * gm.az;
    const float dby0 = duy0 + dpy * gm.rn * gm.ax, dby1 = duy1 + dpy * gm.rn * gm.ay, dby2 = duy2 + dpy * gm.rn * gm.az;
    dW[0] += dbx0 * p.x0 + dby0 * p.y0; dW[1] += dbx0 * p.x1 + dby0 * p.y1; dW[2] += dbx0 * p.x2 + dby0 * p.y2;
    dW[3] += dbx1 * p.x0 + dby1 * p.y0; dW[4] += dbx1 * p.x1 + dby1 * p.y1; dW[5] += dbx1 * p.x2 + dby1 * p.y2;
    dW[6] += dbx2 * p.x0 + dby2 * p.y0; dW[7] += dbx2 * p.x1 + dby2 * p.y1; dW[8] += dbx2 * p.x2 + dby2 * p.y2;
  }
  // D^2 = |q|^2
  dq0 += 2.f * dD2 * gm.qx;
  dq1 += 2.f * dD2 * gm.qy;
  dq2 += 2.f * dD2 * gm.qz;
  // q = y - f a
  float dy0 = dq0, dy1 = dq1, dy2 = dq2;
  float df = -(dq0 * gm.ax + dq1 * gm.ay + dq2 * gm.az);
  da0 += -f * dq0;
  da1 += -f * dq1;
  da2 += -f * dq2;
  // t* = t_e - f
  const float dte = dts;
  df += -dts;
  // f = (y . a) rn
  dy0 += df * gm.rn * gm.ax;
  dy1 += df * gm.rn * gm.ay;
  dy2 += df * gm.rn * gm.az;
  da0 += df * gm.rn * yx;
  da1 += df * gm.rn * yy;
  da2 += df * gm.rn * yz;
  drn += df * ya;
  // rn = 1 / |a|^2
  const float dn = -drn * gm.rn * gm.rn;
  da0 += 2.f * dn * gm.ax;
  da1 += 2.f * dn * gm.ay;
  da2 += 2.f * dn * gm.az;
  // y = -W w
  dW[0] -= dy0 * wx; dW[1] -= dy0 * wy; dW[2] -= dy0 * wz;
  dW[3] -= dy1 * wx; dW[4] -= dy1 * wy; dW[5] -= dy1 * wz;
  dW[6] -= dy2 * wx; dW[7] -= dy2 * wy; dW[8] -= dy2 * wz;
  const float dw0 = -(W[0] * dy0 + W[3] * dy1 + W[6] * dy2);
  const float dw1 = -(W[1] * dy0 + W[4] * dy1 + W[7] * dy2);
  const float dw2 = -(W[2] * dy0 + W[5] * dy1 + W[8] * dy2);
  // a = W d
  dW[0] += da0 * p.a0; dW[1] += da0 * p.a1; dW[2] += da0 * p.a2;
  dW[3] += da1 * p.a0; dW[4] += da1 * p.a1; dW[5] += da1 * p.a2;
  dW[6] += da2 * p.a0; dW[7] += da2 * p.a1; dW[8] += da2 * p.a2;
  // w = (I - d d^T)(mu - o), t_e = d . (mu - o)
  const float dwd = dw0 * p.a0 + dw1 * p.a1 + dw2 * p.a2;
  const float dmu0 = dw0 - dwd * p.a0 + dte * p.a0;
  const float dmu1 = dw1 - dwd * p.a1 + dte * p.a1;
  const float dmu2 = dw2 - dwd * p.a2 + dte * p.a2;
#pragma unroll
  for (int k = 0; k < 9; ++k) g[k] = dW[k];
  g[9] = dmu0;
  g[10] = dmu1;
  g[11] = dmu2;
  g[12] = dsig;
  g[13] = dsp0;
  g[14] = dsp1;
  g[15] = dsp2;
}

}  // namespace cg
