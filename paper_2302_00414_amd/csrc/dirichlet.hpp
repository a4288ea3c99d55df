// The sum over one dimension of I_M of e^{2 pi i k s}, k = -M/2 .. M/2-1:
//   D_{M/2-1}(s) + e^{-M pi i s},  D_{M/2-1}(s) = sin((M-1) pi s) / sin(pi s)
// (the Dirichlet-kernel form of (4.13)); at integer s the kernel takes its
// limit (M-1) cos((M-1) pi s) / cos(pi s).
#pragma once

#include <hip/hip_runtime.h>

namespace nfft {

__device__ __forceinline__ void dirichlet_term(int M, double s, double* re, double* im) {
  double sn, cs;
  sincospi(s, &sn, &cs);
  double s2, c2;
  sincospi((double)(M - 1) * s, &s2, &c2);
  const double dk = fabs(sn) < 1e-12 ? (double)(M - 1) * c2 / cs : s2 / sn;
  double sm, cm;
  sincospi((double)M * s, &sm, &cm);
  *re = dk + cm;
  *im = -sm;
}

}  // namespace nfft
