// Spreading for d = 2 by a register row sweep.
//
// The nodes of a tile are sorted by tile row at plan time, so a work item is
// a run of nodes whose rows never decrease. One wave takes one work item; its
// four 16-lane groups each take one node at a time, all four from the same
// tile row. Lane k of a group owns the absolute padded-tile columns k and
// k + 16 and keeps, in registers, the 2m + 1 padded rows r0 .. r0 + 2m that
// nodes of tile row r0 reach (row r0 is the closed-edge row of a node on a
// grid line). A node adds c_j * psi_0(row) * psi_1(column) to that window:
// the row factors come from lanes 0..2m-1 of the group by DPP row broadcast
// (lane i evaluates window polynomial i), the column factors by a lane
// permutation of the same lanes' second-dimension values. When the sweep
// moves to a later tile row, the rows that leave the window are final: the
// four groups' copies are summed across the wave and the row is written to
// the item's padded-tile slot in device memory. No LDS accumulation, no
// atomics; every padded row is written exactly once, so the result does not
// depend on timing.
#include <type_traits>

#include "spread_common.hpp"

namespace nfft {

template <typename T>
__device__ __forceinline__ T lane_read(T v, int src_lane);
template <>
__device__ __forceinline__ float lane_read<float>(float v, int src_lane) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}
template <>
__device__ __forceinline__ double lane_read<double>(double v, int src_lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(src_lane << 2, (int)(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_ds_bpermute(src_lane << 2, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// sum over the four 16-lane groups of the wave (every lane gets the total)
template <typename T>
__device__ __forceinline__ T group_sum(T v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

template <typename R, int MW, int TT, int NR>
__global__ __launch_bounds__(64) void spread_rows_kernel(SpreadArgs<R> a, int nrhs) {
  constexpr int DEG = PolyDeg<R>::value;
  constexpr int K2 = 2 * MW;
  constexpr int W = K2 + 1;  // window rows
  constexpr int C = 2;       // columns per lane: padded edge <= 32
  constexpr int SB = 64;     // nodes staged per batch
  __shared__ R st_y0[SB], st_y1[SB], st_cx[NR][SB], st_cy[NR][SB];
  __shared__ uint32_t st_loc[SB];
  const int item = blockIdx.x;
  // NR right-hand sides per wave share every node's window factors
  const int r0 = blockIdx.y * NR;
  const int nr = (nrhs - r0) < NR ? (nrhs - r0) : NR;
  const int P = TT > 0 ? TT + K2 : a.g.P;
  const int lane = threadIdx.x;
  const int g = lane >> 4;
  const int k = lane & 15;

  R cf[DEG + 1];
  {
    const int kk = k < K2 ? k : 0;
#pragma unroll
    for (int p = 0; p <= DEG; ++p) cf[p] = a.coef[kk * (DEG + 1) + p];
  }
  const R edge = a.edge;
  const int64_t N = a.g.N;
  const int start = a.item_start[item];
  const int cnt = a.item_count[item];
  const int slot = a.item_slot[item];
  cplx<R>* outs[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int rhs = r0 + (q < nr ? q : 0);
    outs[q] = slot < 0 ? a.tilep + rhs * a.tile_rs + (int64_t)a.item_bin[item] * a.g.Ptot
                       : a.itemp + rhs * a.item_rs + (int64_t)slot * a.g.Ptot;
  }

  R ax[NR][W][C], ay[NR][W][C];
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int r = 0; r < W; ++r)
#pragma unroll
      for (int s = 0; s < C; ++s) ax[q][r][s] = ay[q][r][s] = (R)0;
  int row = 0;      // padded row held in window slot 0
  int maxrow = -1;  // last padded row any node has reached

  // write padded row `row` and move the window down by one row
  auto flush = [&]() {
    if (row > maxrow) {
      // no node reached this row: the whole window is zero
      if (g == 0) {
#pragma unroll
        for (int q = 0; q < NR; ++q) {
          if (q >= nr) break;
#pragma unroll
          for (int s = 0; s < C; ++s) {
            const int col = k + 16 * s;
            if (col < P) outs[q][row * P + col] = mkc<R>((R)0, (R)0);
          }
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < NR; ++q) {
#pragma unroll
        for (int s = 0; s < C; ++s) {
          const R x = group_sum(ax[q][0][s]);
          const R y = group_sum(ay[q][0][s]);
          const int col = k + 16 * s;
          if (q < nr && g == 0 && col < P) outs[q][row * P + col] = mkc<R>(x, y);
        }
#pragma unroll
        for (int r = 0; r + 1 < W; ++r)
#pragma unroll
          for (int s = 0; s < C; ++s) {
            ax[q][r][s] = ax[q][r + 1][s];
            ay[q][r][s] = ay[q][r + 1][s];
          }
#pragma unroll
        for (int s = 0; s < C; ++s) ax[q][W - 1][s] = ay[q][W - 1][s] = (R)0;
      }
    }
    ++row;
  };

  // node data of the next batch, one node per lane, loaded a batch ahead
  R pf0 = 0, pf1 = 0;
  uint32_t pfl = 0;
  cplx<R> pfw = mkc<R>(0, 0), pfs[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) pfs[q] = mkc<R>(0, 0);
  auto issue = [&](int b) {
    if (b + lane < cnt) {
      const int i = start + b + lane;
      pf0 = a.frac[i];
      pf1 = a.frac[N + i];
      pfl = a.loc[i];
      pfw = a.w[i];
      const int jj = a.perm[i];
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (q < nr) pfs[q] = a.f[(int64_t)(r0 + q) * a.f_rs + jj];
    }
  };
  issue(0);
  for (int b0 = 0; b0 < cnt; b0 += SB) {
    const int nb = (cnt - b0) < SB ? (cnt - b0) : SB;
    __syncthreads();  // previous batch consumed
    if (lane < nb) {
      st_y0[lane] = (R)2 * pf0 - (R)1;
      st_y1[lane] = (R)2 * pf1 - (R)1;
      st_loc[lane] = pfl;
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const cplx<R> c = cmul<R>(pfw, pfs[q]);
        st_cx[q][lane] = c.x;
        st_cy[q][lane] = c.y;
      }
    }
    if (b0 + SB < cnt) issue(b0 + SB);
    __syncthreads();
    int i = 0;
    while (i < nb) {
      const int r0 = (int)(st_loc[i] & kLocMask);  // tile row of the next node
      while (row < r0) flush();
      if (r0 + K2 > maxrow) maxrow = r0 + K2;
      // group g takes node i + g if it lies in the same tile row; rows never
      // decrease, so the groups that take a node are a prefix
      const int j = i + g;
      const uint32_t L = j < nb ? st_loc[j] : 0u;
      const bool take = j < nb && (int)(L & kLocMask) == r0;
      const uint64_t bal = __ballot(take);
      const int used = (int)((bal & 1ull) + ((bal >> 16) & 1ull) + ((bal >> 32) & 1ull) +
                             ((bal >> 48) & 1ull));
      if (take) {
        const R p0 = horner<R>(cf, st_y0[j]);
        const R p1 = horner<R>(cf, st_y1[j]);
        const int l1 = (int)((L >> kLocBits) & kLocMask);
        const bool e0 = (L >> kEdgeShift) & 1u;
        const bool e1 = (L >> (kEdgeShift + 1)) & 1u;
        // column factors of this lane's columns (footprint column jc = col - l1 - 1;
        // jc = -1 is the closed-edge column)
        R cw[C];
#pragma unroll
        for (int s = 0; s < C; ++s) {
          const int jc = k + 16 * s - l1 - 1;
          const R v = lane_read<R>(p1, (g << 4) | (jc & 15));
          cw[s] = (jc >= 0 && jc < K2) ? v : ((jc == -1 && e1) ? edge : (R)0);
        }
        R vx[NR][C], vy[NR][C];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
          const R cx = st_cx[q][j], cy = st_cy[q][j];
#pragma unroll
          for (int s = 0; s < C; ++s) {
            vx[q][s] = cx * cw[s];
            vy[q][s] = cy * cw[s];
          }
        }
        // window slot 0: closed-edge row; slot 1 + i: footprint row i
        const R w0 = e0 ? edge : (R)0;
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
          for (int s = 0; s < C; ++s) {
            ax[q][0][s] += vx[q][s] * w0;
            ay[q][0][s] += vy[q][s] * w0;
          }
        static_for<0, K2>([&](auto ic) {
          constexpr int I = decltype(ic)::value;
          const R rw = row_bcast<I>(p0);
#pragma unroll
          for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int s = 0; s < C; ++s) {
              ax[q][1 + I][s] += vx[q][s] * rw;
              ay[q][1 + I][s] += vy[q][s] * rw;
            }
        });
      }
      i += used;
    }
  }
  while (row < P) flush();
}

namespace {

template <typename R, int MW, int NR>
hipError_t rows_nr(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  const dim3 grid(a.g.nsub, (nrhs + NR - 1) / NR);
  if (a.g.T == 16)
    hipLaunchKernelGGL((spread_rows_kernel<R, MW, 16, NR>), grid, dim3(64), 0, s, a, nrhs);
  else
    hipLaunchKernelGGL((spread_rows_kernel<R, MW, 0, NR>), grid, dim3(64), 0, s, a, nrhs);
  return hipGetLastError();
}

// float32: two right-hand sides per wave when a call has several (the
// window work is shared); float64 keeps one (register budget)
template <typename R, int MW>
hipError_t rows_m(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  if constexpr (std::is_same<R, float>::value) {
    if (nrhs > 1 && a.nr >= 2) return rows_nr<R, MW, 2>(a, nrhs, s);
  }
  return rows_nr<R, MW, 1>(a, nrhs, s);
}

}  // namespace

bool spread_rows_supported(int d, int P) { return d == 2 && P <= 32; }

template <typename R>
hipError_t launch_spread_rows(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  if (a.g.nsub == 0) return hipSuccess;
  if (!spread_rows_supported(a.g.d, a.g.P)) return hipErrorInvalidValue;
  switch (a.g.m) {
    case 1: return rows_m<R, 1>(a, nrhs, s);
    case 2: return rows_m<R, 2>(a, nrhs, s);
    case 3: return rows_m<R, 3>(a, nrhs, s);
    case 4: return rows_m<R, 4>(a, nrhs, s);
    case 5: return rows_m<R, 5>(a, nrhs, s);
    case 6: return rows_m<R, 6>(a, nrhs, s);
    case 7: return rows_m<R, 7>(a, nrhs, s);
    case 8: return rows_m<R, 8>(a, nrhs, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_spread_rows<float>(const SpreadArgs<float>&, int, hipStream_t);
template hipError_t launch_spread_rows<double>(const SpreadArgs<double>&, int, hipStream_t);

}  // namespace nfft
