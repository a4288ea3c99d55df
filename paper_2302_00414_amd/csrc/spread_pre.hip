// Spreading with window factors precomputed at plan time (d = 2), and the
// plan-time kernel that computes them.
//
// The nodes of a plan are fixed, so the 2m window factors per dimension that
// the group kernel would otherwise evaluate on every call (two polynomials of
// the per-cell fit per lane and node, plus the broadcasts of the row factors)
// can be evaluated once. The table holds, in the plan's tile order, for every
// node and footprint cell c = 0..2m-1 the pair (factor of dimension 0,
// factor of dimension 1): 16 m bytes per node in float32, 32 m in float64.
// Lane c of a spreading group loads its pair (the row factor it broadcasts
// to the group and its own column factor), one 8- or 16-byte load. The table
// is computed with the same polynomials and the same arithmetic as the lanes
// of the group kernel, so both spreading paths use identical factors.
#include <type_traits>

#include "spread_group.hpp"

namespace nfft {

template <typename R, int MW>
__global__ __launch_bounds__(256) void psi_kernel(const R* frac, int64_t N, const R* coef, R* psi) {
  constexpr int K2 = 2 * MW;
  constexpr int DEG = PolyDeg<R>::value;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= 2 * N) return;
  const int64_t i = j >> 1;   // node (tile order)
  const int t = (int)(j & 1);  // dimension
  const R y = (R)2 * frac[t * N + i] - (R)1;
  R* out = psi + i * (2 * K2) + t;
#pragma unroll
  for (int c = 0; c < K2; ++c) out[2 * c] = horner<R>(coef + c * (DEG + 1), y);
}

template <typename R, int MW>
static hipError_t psi_m(const R* frac, int64_t N, const R* coef, R* psi, hipStream_t s) {
  const int64_t jobs = 2 * N;
  const unsigned blocks = (unsigned)((jobs + 255) / 256);
  hipLaunchKernelGGL((psi_kernel<R, MW>), dim3(blocks), dim3(256), 0, s, frac, N, coef, psi);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_psi(const R* frac, int64_t N, int m, const R* coef, R* psi, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  switch (m) {
    case 1: return psi_m<R, 1>(frac, N, coef, psi, s);
    case 2: return psi_m<R, 2>(frac, N, coef, psi, s);
    case 3: return psi_m<R, 3>(frac, N, coef, psi, s);
    case 4: return psi_m<R, 4>(frac, N, coef, psi, s);
    case 5: return psi_m<R, 5>(frac, N, coef, psi, s);
    case 6: return psi_m<R, 6>(frac, N, coef, psi, s);
    case 7: return psi_m<R, 7>(frac, N, coef, psi, s);
    case 8: return psi_m<R, 8>(frac, N, coef, psi, s);
    default: return hipErrorInvalidValue;
  }
}

// float32: private group tiles (64 / 128 / 256 threads, complex or component
// planes); float64: 256 threads sharing one tile
template <typename R, int MW>
static hipError_t spread_pre_m(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  if constexpr (std::is_same<R, float>::value) {
    if (a.planes == 2) {
      if (a.nt == 64) return spread_group_nt<R, 2, MW, 64, true, 1>(a, nrhs, s);
      if (a.nt == 256) return spread_group_nt<R, 2, MW, 256, true, 1>(a, nrhs, s);
      return spread_group_nt<R, 2, MW, 128, true, 1>(a, nrhs, s);
    }
    if (a.nt == 64) return spread_group_nt<R, 2, MW, 64, false, 1>(a, nrhs, s);
    if (a.nt == 256) return spread_group_nt<R, 2, MW, 256, false, 1>(a, nrhs, s);
    return spread_group_nt<R, 2, MW, 128, false, 1>(a, nrhs, s);
  } else {
    return spread_group_nt<R, 2, MW, 256, false, 1>(a, nrhs, s);
  }
}

template <typename R>
hipError_t launch_spread_pre(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  if (a.g.d != 2 || !a.psi) return hipErrorInvalidValue;
  if (a.g.nsub == 0) return hipSuccess;
  switch (a.g.m) {
    case 1: return spread_pre_m<R, 1>(a, nrhs, s);
    case 2: return spread_pre_m<R, 2>(a, nrhs, s);
    case 3: return spread_pre_m<R, 3>(a, nrhs, s);
    case 4: return spread_pre_m<R, 4>(a, nrhs, s);
    case 5: return spread_pre_m<R, 5>(a, nrhs, s);
    case 6: return spread_pre_m<R, 6>(a, nrhs, s);
    case 7: return spread_pre_m<R, 7>(a, nrhs, s);
    case 8: return spread_pre_m<R, 8>(a, nrhs, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_psi<float>(const float*, int64_t, int, const float*, float*, hipStream_t);
template hipError_t launch_psi<double>(const double*, int64_t, int, const double*, double*,
                                       hipStream_t);
template hipError_t launch_spread_pre<float>(const SpreadArgs<float>&, int, hipStream_t);
template hipError_t launch_spread_pre<double>(const SpreadArgs<double>&, int, hipStream_t);

}  // namespace nfft
