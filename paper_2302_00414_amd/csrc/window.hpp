// Kaiser-Bessel window on the device, normalised to avoid overflow.
//
// In grid units the window is phi(t) = (1/pi) sinh(b z)/z with
// z = sqrt(m^2 - t^2), |t| <= m, b = pi (2 - 1/sigma). The device evaluates
//     psi(t) = pi e^{-b m} phi(t) = e^{b (z - m)} (1 - e^{-2 b z}) / (2 z),
// with z - m = -t^2 / (z + m) so that the exponent is formed without
// cancellation, and z^2 = (m - t)(m + t). The constant pi e^{-b m} per
// dimension is removed again by the deconvolution factors, which the host
// tabulates as e^{b m} / (pi * M_sigma * hat phi(k)) including the sign
// (-1)^k of the half-grid shift.
#pragma once

#include "common.hpp"

namespace nfft {

__device__ __forceinline__ double kb_psi(double t, double b, double m) {
  double z2 = (m - t) * (m + t);
  z2 = z2 > 0.0 ? z2 : 0.0;
  double z = sqrt(z2);
  double e1 = exp(-b * t * t / (z + m));
  double s = (z > 0.0) ? (-expm1(-2.0 * b * z) / (2.0 * z)) : b;
  return e1 * s;
}

__device__ __forceinline__ float kb_psi(float t, float b, float m) {
  float z2 = (m - t) * (m + t);
  z2 = z2 > 0.0f ? z2 : 0.0f;
  float z = sqrtf(z2);
  float e1 = __expf(-b * t * t / (z + m));
  float bz = b * z;
  // (1 - e^{-2bz}) / (2z): series near z = 0 (only edge cells, whose values
  // are ~e^{-bm} of the peak), exponential form elsewhere.
  float s = (bz < 1e-3f) ? b * (1.0f - bz) : (1.0f - __expf(-2.0f * bz)) / (2.0f * z);
  return e1 * s;
}

// Degree of the per-cell window polynomials (see kb_poly).
template <typename R> struct PolyDeg;
template <> struct PolyDeg<double> { static constexpr int value = 16; };
template <> struct PolyDeg<float> { static constexpr int value = 10; };

// Window factors of one node from per-cell polynomials, for its D offsets
// at once: for cell i = 0..2m-1 (offset t = frac + m - 1 - i) the host fits
// psi(t) ~ sum_p coef[i][p] y^p with y = 2 frac - 1 in [-1, 1] (Chebyshev
// interpolation, converted to monomials, error checked at plan time); each
// coefficient is read once and feeds the D Horner evaluations. psi[t][0] is
// the extra closed-edge cell of a node on a grid line of dimension t.
template <typename R, int MW, int D>
__device__ __forceinline__ void kb_poly(const R* y, const bool* edge, R edge_val,
                                        const R* __restrict__ coef, R (*psi)[2 * MW + 1]) {
  constexpr int DEG = PolyDeg<R>::value;
#pragma unroll
  for (int t = 0; t < D; ++t) psi[t][0] = edge[t] ? edge_val : (R)0;
#pragma unroll
  for (int i = 0; i < 2 * MW; ++i) {
    const R* c = coef + i * (DEG + 1);
    R v[D];
#pragma unroll
    for (int t = 0; t < D; ++t) v[t] = c[DEG];
#pragma unroll
    for (int p = DEG - 1; p >= 0; --p)
#pragma unroll
      for (int t = 0; t < D; ++t) v[t] = v[t] * y[t] + c[p];
#pragma unroll
    for (int t = 0; t < D; ++t) psi[t][1 + i] = v[t];
  }
}

}  // namespace nfft
