// Spreading of several right-hand sides per work-group (d <= 2).
//
// Right-hand sides that share one node set (coils, slices) share everything
// but the samples: the node's cell, its window factors and its weight. A
// work-group here takes one work item and NR right-hand sides; every node is
// loaded and its window polynomials evaluated once, then its NR values
// c_j^(r) = w_j f_j^(r) are spread with the same factors. The NR padded tiles
// are shared by all lane groups of the work-group and updated with float64
// LDS atomics (private tiles per group and right-hand side would not fit in
// LDS); the float32 path therefore also accumulates in float64 and rounds
// once when the tile is written out. Group layout, row broadcasts and the
// closed-edge cells are those of the single right-hand-side kernel.
#include <algorithm>
#include <type_traits>

#include "spread_common.hpp"

namespace nfft {

template <typename R, int D, int MW, int NT, int TT, int NR>
__global__ __launch_bounds__(NT) void spread_multi_kernel(SpreadArgs<R> a, int nrhs) {
  static_assert(D <= 2 && 2 * MW <= 16, "group spreading covers d <= 2, m <= 8");
  constexpr int DEG = PolyDeg<R>::value;
  constexpr int NG = NT / 16;
  constexpr int K2 = 2 * MW;
  extern __shared__ double lds_d[];
  const int item = blockIdx.x;
  const int r0 = blockIdx.y * NR;
  const int nr = (nrhs - r0) < NR ? (nrhs - r0) : NR;
  const int P = TT > 0 ? TT + 2 * MW : a.g.P;
  const int Ptot = a.g.Ptot;
  const int tid = threadIdx.x;
  const int grp = tid >> 4;
  const int k = tid & 15;

  // LDS: NR tiles of (real, imaginary) float64 planes, then the staging area
  double* planes = lds_d;
  R* st_y0 = reinterpret_cast<R*>(lds_d + (size_t)NR * 2 * Ptot);
  R* st_y1 = st_y0 + NT;
  R* st_c = st_y1 + NT;  // [NR][re, im][NT]
  uint32_t* st_loc = reinterpret_cast<uint32_t*>(st_c + 2 * NR * NT);
  for (int i = tid; i < NR * 2 * Ptot; i += NT) lds_d[i] = 0.0;
  auto add = [&](int r, int cell, R x, R y) {
    lds_add(planes + (size_t)(2 * r) * Ptot + cell, (double)x);
    lds_add(planes + (size_t)(2 * r + 1) * Ptot + cell, (double)y);
  };

  R cf[DEG + 1];
  {
    const int kk = k < K2 ? k : 0;
#pragma unroll
    for (int p = 0; p <= DEG; ++p) cf[p] = a.coef[kk * (DEG + 1) + p];
  }
  const R edge = a.edge;
  __syncthreads();

  const int64_t N = a.g.N;
  const int start = a.item_start[item];
  const int cnt = a.item_count[item];
  // one node per thread loaded one batch ahead (see the single-rhs kernel)
  R pf0 = 0, pf1 = 0;
  uint32_t pfl = 0;
  cplx<R> pfw = mkc<R>(0, 0);
  cplx<R> pfs[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) pfs[r] = mkc<R>(0, 0);
  auto issue = [&](int b) {
    if (b + tid < cnt) {
      const int i = start + b + tid;
      pf0 = a.frac[i];
      pf1 = D > 1 ? a.frac[N + i] : (R)0;
      pfl = a.loc[i];
      pfw = a.w[i];
      const int j = a.perm[i];
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (r < nr) pfs[r] = a.f[(int64_t)(r0 + r) * a.f_rs + j];
    }
  };
  issue(0);
  for (int b0 = 0; b0 < cnt; b0 += NT) {
    const int nb = (cnt - b0) < NT ? (cnt - b0) : NT;
    if (tid < nb) {
      st_y0[tid] = (R)2 * pf0 - (R)1;
      st_y1[tid] = (R)2 * pf1 - (R)1;
      st_loc[tid] = pfl;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const cplx<R> c = cmul<R>(pfw, pfs[r]);
        st_c[(2 * r) * NT + tid] = c.x;
        st_c[(2 * r + 1) * NT + tid] = c.y;
      }
    }
    if (b0 + NT < cnt) issue(b0 + NT);
    __syncthreads();
    for (int n = grp; n < nb; n += NG) {
      // window factors only (c = 1): vx = the lane's column factor
      NodePrep<R, K2> h;
      prep_node<R, D, K2>(h, st_y0[n], st_y1[n], (R)1, (R)0, st_loc[n], cf);
      R cx[NR], cy[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        cx[r] = st_c[(2 * r) * NT + n];
        cy[r] = st_c[(2 * r + 1) * NT + n];
      }
      if constexpr (D == 1) {
        if (k < K2) {
#pragma unroll
          for (int r = 0; r < NR; ++r)
            if (r < nr) add(r, h.l0 + 1 + k, cx[r] * h.vx, cy[r] * h.vx);
        }
        if (h.e0 && k == 0) {
#pragma unroll
          for (int r = 0; r < NR; ++r)
            if (r < nr) add(r, h.l0, cx[r] * edge, cy[r] * edge);
        }
      } else {
        const int col = h.l1 + 1 + k;
        if (k < K2) {
#pragma unroll
          for (int i = 0; i < K2; ++i) {
            const R wgt = h.vx * h.rw[i];
            const int cell = (h.l0 + 1 + i) * P + col;
#pragma unroll
            for (int r = 0; r < NR; ++r)
              if (r < nr) add(r, cell, cx[r] * wgt, cy[r] * wgt);
          }
        }
        if (h.e0 | h.e1) {
          // closed-edge cells of a node on a grid line: row 0 and column 0
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            if (r >= nr) continue;
            if (h.e0 && k < K2) add(r, h.l0 * P + col, cx[r] * h.vx * edge, cy[r] * h.vx * edge);
            if (h.e1 && k < K2)
              add(r, (h.l0 + 1 + k) * P + h.l1, cx[r] * h.p0 * edge, cy[r] * h.p0 * edge);
            if (h.e0 && h.e1 && k == 0)
              add(r, h.l0 * P + h.l1, cx[r] * edge * edge, cy[r] * edge * edge);
          }
        }
      }
    }
    __syncthreads();
  }

  const int slot = a.item_slot[item];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= nr) break;
    cplx<R>* out = slot < 0 ? a.tilep + (r0 + r) * a.tile_rs + (int64_t)a.item_bin[item] * Ptot
                            : a.itemp + (r0 + r) * a.item_rs + (int64_t)slot * Ptot;
    const double* re = planes + (size_t)(2 * r) * Ptot;
    const double* im = re + Ptot;
    for (int i = tid; i < Ptot; i += NT) out[i] = mkc<R>((R)re[i], (R)im[i]);
  }
}

namespace {

constexpr int kMultiThreads = 256;

template <typename R, int NR>
size_t multi_lds(int Ptot) {
  return (size_t)NR * 2 * Ptot * sizeof(double) +
         (size_t)kMultiThreads * ((2 + 2 * NR) * sizeof(R) + sizeof(uint32_t));
}

template <typename R, int D, int MW, int NR>
hipError_t multi_nr(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  constexpr int NT = kMultiThreads;
  const dim3 grid(a.g.nsub, (nrhs + NR - 1) / NR);
  const size_t lds = multi_lds<R, NR>(a.g.Ptot);
  if constexpr (D == 2) {
    if (a.g.T == 16) {
      hipLaunchKernelGGL((spread_multi_kernel<R, D, MW, NT, 16, NR>), grid, dim3(NT), lds, s, a, nrhs);
      return hipGetLastError();
    }
    if (a.g.T == 8) {
      hipLaunchKernelGGL((spread_multi_kernel<R, D, MW, NT, 8, NR>), grid, dim3(NT), lds, s, a, nrhs);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((spread_multi_kernel<R, D, MW, NT, 0, NR>), grid, dim3(NT), lds, s, a, nrhs);
  return hipGetLastError();
}

template <typename R, int D, int MW>
hipError_t multi_dm(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  switch (a.nr) {
    case 2: return multi_nr<R, D, MW, 2>(a, nrhs, s);
    case 4: return multi_nr<R, D, MW, 4>(a, nrhs, s);
    case 8: return multi_nr<R, D, MW, 8>(a, nrhs, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename R, int D>
hipError_t multi_d(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  switch (a.g.m) {
    case 1: return multi_dm<R, D, 1>(a, nrhs, s);
    case 2: return multi_dm<R, D, 2>(a, nrhs, s);
    case 3: return multi_dm<R, D, 3>(a, nrhs, s);
    case 4: return multi_dm<R, D, 4>(a, nrhs, s);
    case 5: return multi_dm<R, D, 5>(a, nrhs, s);
    case 6: return multi_dm<R, D, 6>(a, nrhs, s);
    case 7: return multi_dm<R, D, 7>(a, nrhs, s);
    case 8: return multi_dm<R, D, 8>(a, nrhs, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

template <typename R>
hipError_t launch_spread_multi(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  if (a.g.nsub == 0) return hipSuccess;
  switch (a.g.d) {
    case 1: return multi_d<R, 1>(a, nrhs, s);
    case 2: return multi_d<R, 2>(a, nrhs, s);
    default: return hipErrorInvalidValue;
  }
}

size_t spread_multi_lds_bytes(bool f64, int Ptot, int nr) {
  switch (nr) {
    case 2: return f64 ? multi_lds<double, 2>(Ptot) : multi_lds<float, 2>(Ptot);
    case 4: return f64 ? multi_lds<double, 4>(Ptot) : multi_lds<float, 4>(Ptot);
    case 8: return f64 ? multi_lds<double, 8>(Ptot) : multi_lds<float, 8>(Ptot);
    default: return 0;
  }
}

template hipError_t launch_spread_multi<float>(const SpreadArgs<float>&, int, hipStream_t);
template hipError_t launch_spread_multi<double>(const SpreadArgs<double>&, int, hipStream_t);

}  // namespace nfft
