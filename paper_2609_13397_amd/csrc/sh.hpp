// Real spherical harmonics of degree <= 3 and their vector-Jacobian product.
#pragma once

#include <hip/hip_runtime.h>

namespace cg {

// Real spherical harmonics of degree <= 3 at a unit direction (x, y, z): orthonormal
// on the sphere, Condon-Shortley phase, (l, m) order with m = -l..l.  Each constant is
// the normalisation sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (times sqrt 2 for m != 0)
// multiplied by the integer factor of the associated Legendre function written as a
// polynomial in x, y, z.
__device__ __forceinline__ void sh_basis3(float x, float y, float z, float Y[16]) {
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[0] = 0.28209479177387814f;                        // 1 / (2 sqrt(pi))
  Y[1] = -0.4886025119029199f * y;                    // sqrt(3 / (4 pi))
  Y[2] = 0.4886025119029199f * z;
  Y[3] = -0.4886025119029199f * x;
  Y[4] = 1.0925484305920792f * x * y;                 // (1/2) sqrt(15 / pi)
  Y[5] = -1.0925484305920792f * y * z;
  Y[6] = 0.31539156525252005f * (3.f * zz - 1.f);     // (1/4) sqrt(5 / pi)
  Y[7] = -1.0925484305920792f * x * z;
  Y[8] = 0.5462742152960396f * (xx - yy);             // (1/4) sqrt(15 / pi)
  Y[9] = -0.5900435899266435f * y * (3.f * xx - yy);  // (1/4) sqrt(35 / (2 pi))
  Y[10] = 2.890611442640554f * x * y * z;             // (1/2) sqrt(105 / pi)
  Y[11] = -0.4570457994644658f * y * (5.f * zz - 1.f);  // (1/4) sqrt(21 / (2 pi))
  Y[12] = 0.3731763325901154f * z * (5.f * zz - 3.f);   // (1/4) sqrt(7 / pi)
  Y[13] = -0.4570457994644658f * x * (5.f * zz - 1.f);
  Y[14] = 1.445305721320277f * z * (xx - yy);           // (1/4) sqrt(105 / pi)
  Y[15] = -0.5900435899266435f * x * (xx - 3.f * yy);
}

// g = sum_k a_k grad Y_k(x, y, z): the derivatives of the polynomials above with
// respect to the (unnormalised) direction components, contracted with a[16].
__device__ __forceinline__ void sh_basis3_vjp(float x, float y, float z, const float a[16], float g[3]) {
  constexpr float c1 = 0.4886025119029199f, c2a = 1.0925484305920792f, c2b = 0.31539156525252005f,
                  c2c = 0.5462742152960396f, c3a = 0.5900435899266435f, c3b = 2.890611442640554f,
                  c3c = 0.4570457994644658f, c3d = 0.3731763325901154f, c3e = 1.445305721320277f;
  const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
  const float p5 = 5.f * zz - 1.f, dxy3 = 3.f * xx - 3.f * yy;
  g[0] = -c1 * a[3] + c2a * (y * a[4] - z * a[7]) + 2.f * c2c * x * a[8] - 6.f * c3a * xy * a[9] +
         c3b * yz * a[10] - c3c * p5 * a[13] + 2.f * c3e * xz * a[14] - c3a * dxy3 * a[15];
  g[1] = -c1 * a[1] + c2a * (x * a[4] - z * a[5]) - 2.f * c2c * y * a[8] - c3a * dxy3 * a[9] +
         c3b * xz * a[10] - c3c * p5 * a[11] - 2.f * c3e * yz * a[14] + 6.f * c3a * xy * a[15];
  g[2] = c1 * a[2] - c2a * (y * a[5] + x * a[7]) + 6.f * c2b * z * a[6] + c3b * xy * a[10] -
         10.f * c3c * (yz * a[11] + xz * a[13]) + c3d * (15.f * zz - 3.f) * a[12] + c3e * (xx - yy) * a[14];
}

}  // namespace cg
