// Spreading for d = 2 with the window evaluated late (spread mode 4): the
// structure of the table path (node offsets and cell words loaded from device
// memory two nodes ahead, only c_j staged in LDS, row factors broadcast in
// the group), with the two window polynomials of a lane evaluated in the step
// from the offsets instead of read from a table. Same values as the other
// paths, no per-node-set memory beyond the plan's.
#include <type_traits>

#include "spread_group.hpp"

namespace nfft {

// float32: private group tiles (64 / 128 / 256 threads, complex or component
// planes); float64: 256 threads sharing one tile
template <typename R, int MW>
static hipError_t spread_late_m(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  if constexpr (std::is_same<R, float>::value) {
    if (a.planes == 2) {
      if (a.nt == 64) return spread_group_nt<R, 2, MW, 64, true, 2>(a, nrhs, s);
      if (a.nt == 256) return spread_group_nt<R, 2, MW, 256, true, 2>(a, nrhs, s);
      return spread_group_nt<R, 2, MW, 128, true, 2>(a, nrhs, s);
    }
    if (a.nt == 64) return spread_group_nt<R, 2, MW, 64, false, 2>(a, nrhs, s);
    if (a.nt == 256) return spread_group_nt<R, 2, MW, 256, false, 2>(a, nrhs, s);
    return spread_group_nt<R, 2, MW, 128, false, 2>(a, nrhs, s);
  } else {
    return spread_group_nt<R, 2, MW, 256, false, 2>(a, nrhs, s);
  }
}

template <typename R>
hipError_t launch_spread_late(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  if (a.g.d != 2) return hipErrorInvalidValue;
  if (a.g.nsub == 0) return hipSuccess;
  switch (a.g.m) {
    case 1: return spread_late_m<R, 1>(a, nrhs, s);
    case 2: return spread_late_m<R, 2>(a, nrhs, s);
    case 3: return spread_late_m<R, 3>(a, nrhs, s);
    case 4: return spread_late_m<R, 4>(a, nrhs, s);
    case 5: return spread_late_m<R, 5>(a, nrhs, s);
    case 6: return spread_late_m<R, 6>(a, nrhs, s);
    case 7: return spread_late_m<R, 7>(a, nrhs, s);
    case 8: return spread_late_m<R, 8>(a, nrhs, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_spread_late<float>(const SpreadArgs<float>&, int, hipStream_t);
template hipError_t launch_spread_late<double>(const SpreadArgs<double>&, int, hipStream_t);

}  // namespace nfft
