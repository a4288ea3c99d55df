// Spreading (adjoint NFFT step 1) and window sums (NFFT step 3).
//
// Work decomposition: the oversampled grid is cut into tiles of T^d cells;
// the nodes, sorted by tile at plan time, form work items of at most a few
// hundred nodes of one tile. A work-group owns one work item and one
// right-hand side. Its nodes touch only the padded tile of (T + 2m)^d cells
// around the tile, which lives in LDS:
//   spread : every thread takes nodes, forms c_j = w_j f_j and the d window
//            factor vectors, and adds c_j * prod_t psi_t into the LDS tile;
//            the finished padded tile is written out whole, and the tile
//            sums are merged into grid cells by the first FFT pass.
//   sums   : the padded tile is gathered from the grid (periodically
//            wrapped) into LDS, and every thread evaluates its nodes' sums.
// Nodes exactly on a grid line (offset zero) get the extra closed-edge cell;
// a wave takes the (2m+1)-wide loop only when one of its lanes needs it.
#include "internal.hpp"
#include "window.hpp"

namespace nfft {

template <typename R>
__device__ __forceinline__ void lds_add(R* p, R v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Window factors of one node in one dimension: psi[0] is the extra edge
// cell (zero unless the node lies on a grid line), psi[1 + i] the value at
// offset t = frac + m - 1 - i, i = 0..2m-1.
template <typename R, int MW>
__device__ __forceinline__ void node_window(R fr, bool edge, R b, R mr, R edge_val, R* psi) {
  psi[0] = edge ? edge_val : (R)0;
#pragma unroll
  for (int i = 0; i < 2 * MW; ++i) psi[1 + i] = kb_psi(fr + (R)(MW - 1 - i), b, mr);
}

template <typename R, int D, int MW, bool EDGE>
__device__ __forceinline__ void add_node(cplx<R>* tile, int P, const int* l, cplx<R> c,
                                         const R (*psi)[2 * MW + 1]) {
  constexpr int K0 = EDGE ? 0 : 1;
  constexpr int KE = 2 * MW + 1;
  if constexpr (D == 1) {
#pragma unroll
    for (int i0 = K0; i0 < KE; ++i0) {
      cplx<R>* p = tile + (l[0] + i0);
      lds_add(&p->x, c.x * psi[0][i0]);
      lds_add(&p->y, c.y * psi[0][i0]);
    }
  } else if constexpr (D == 2) {
#pragma unroll
    for (int i0 = K0; i0 < KE; ++i0) {
      const R a = psi[0][i0];
      const cplx<R> c0 = mkc<R>(c.x * a, c.y * a);
      cplx<R>* row = tile + (l[0] + i0) * P + l[1];
#pragma unroll
      for (int i1 = K0; i1 < KE; ++i1) {
        lds_add(&row[i1].x, c0.x * psi[1][i1]);
        lds_add(&row[i1].y, c0.y * psi[1][i1]);
      }
    }
  } else {
#pragma unroll
    for (int i0 = K0; i0 < KE; ++i0) {
      const R a = psi[0][i0];
      const cplx<R> c0 = mkc<R>(c.x * a, c.y * a);
#pragma unroll
      for (int i1 = K0; i1 < KE; ++i1) {
        const R a1 = psi[1][i1];
        const cplx<R> c1 = mkc<R>(c0.x * a1, c0.y * a1);
        cplx<R>* row = tile + ((l[0] + i0) * P + (l[1] + i1)) * P + l[2];
#pragma unroll
        for (int i2 = K0; i2 < KE; ++i2) {
          lds_add(&row[i2].x, c1.x * psi[2][i2]);
          lds_add(&row[i2].y, c1.y * psi[2][i2]);
        }
      }
    }
  }
}

template <typename R, int D, int MW>
__global__ __launch_bounds__(256) void spread_kernel(SpreadArgs<R> a) {
  extern __shared__ unsigned char smem_raw[];
  cplx<R>* tile = reinterpret_cast<cplx<R>*>(smem_raw);
  const int item = blockIdx.x;
  const int rhs = blockIdx.y;
  const int P = a.g.P;
  const int Ptot = a.g.Ptot;
  for (int i = threadIdx.x; i < Ptot; i += blockDim.x) tile[i] = mkc<R>(0, 0);
  __syncthreads();

  const int64_t N = a.g.N;
  const int start = a.item_start[item];
  const int cnt = a.item_count[item];
  const cplx<R>* f = a.f + rhs * a.f_rs;
  for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
    const int i = start + k;
    const uint32_t L = a.loc[i];
    int l[D];
    R psi[D][2 * MW + 1];
    bool any_edge = false;
#pragma unroll
    for (int t = 0; t < D; ++t) {
      l[t] = (int)((L >> (kLocBits * t)) & kLocMask);
      const bool e = (L >> (kEdgeShift + t)) & 1u;
      any_edge |= e;
      node_window<R, MW>(a.frac[t * N + i], e, a.b, a.mr, a.edge, psi[t]);
    }
    const cplx<R> c = cmul<R>(a.w[i], f[a.perm[i]]);
    if (__any(any_edge))
      add_node<R, D, MW, true>(tile, P, l, c, psi);
    else
      add_node<R, D, MW, false>(tile, P, l, c, psi);
  }
  __syncthreads();
  cplx<R>* out = a.sub + rhs * a.sub_rs + (int64_t)item * Ptot;
  for (int i = threadIdx.x; i < Ptot; i += blockDim.x) out[i] = tile[i];
}

template <typename R, int D, int MW, bool EDGE>
__device__ __forceinline__ cplx<R> sum_node(const cplx<R>* tile, int P, const int* l,
                                            const R (*psi)[2 * MW + 1]) {
  constexpr int K0 = EDGE ? 0 : 1;
  constexpr int KE = 2 * MW + 1;
  R sx = 0, sy = 0;
  if constexpr (D == 1) {
#pragma unroll
    for (int i0 = K0; i0 < KE; ++i0) {
      const cplx<R> v = tile[l[0] + i0];
      sx += v.x * psi[0][i0];
      sy += v.y * psi[0][i0];
    }
  } else if constexpr (D == 2) {
#pragma unroll
    for (int i0 = K0; i0 < KE; ++i0) {
      const cplx<R>* row = tile + (l[0] + i0) * P + l[1];
      R rx = 0, ry = 0;
#pragma unroll
      for (int i1 = K0; i1 < KE; ++i1) {
        const cplx<R> v = row[i1];
        rx += v.x * psi[1][i1];
        ry += v.y * psi[1][i1];
      }
      sx += rx * psi[0][i0];
      sy += ry * psi[0][i0];
    }
  } else {
#pragma unroll
    for (int i0 = K0; i0 < KE; ++i0) {
      R px = 0, py = 0;
#pragma unroll
      for (int i1 = K0; i1 < KE; ++i1) {
        const cplx<R>* row = tile + ((l[0] + i0) * P + (l[1] + i1)) * P + l[2];
        R rx = 0, ry = 0;
#pragma unroll
        for (int i2 = K0; i2 < KE; ++i2) {
          const cplx<R> v = row[i2];
          rx += v.x * psi[2][i2];
          ry += v.y * psi[2][i2];
        }
        px += rx * psi[1][i1];
        py += ry * psi[1][i1];
      }
      sx += px * psi[0][i0];
      sy += py * psi[0][i0];
    }
  }
  return mkc<R>(sx, sy);
}

template <typename R, int D, int MW>
__global__ __launch_bounds__(256) void interp_kernel(InterpArgs<R> a) {
  extern __shared__ unsigned char smem_raw[];
  cplx<R>* tile = reinterpret_cast<cplx<R>*>(smem_raw);
  const int item = blockIdx.x;
  const int rhs = blockIdx.y;
  const int P = a.g.P;
  const int Ptot = a.g.Ptot;
  const int Ms = a.g.Ms;
  const int nb = a.g.nb;
  // tile origin (in cells) of this work item's tile, per dimension
  int org[3] = {0, 0, 0};
  {
    int bb = a.item_bin[item];
    for (int t = D - 1; t >= 0; --t) {
      org[t] = (bb % nb) * a.g.T - a.g.m;
      bb /= nb;
    }
  }
  const cplx<R>* grid = a.grid + rhs * a.grid_rs;
  for (int i = threadIdx.x; i < Ptot; i += blockDim.x) {
    int rem = i;
    int64_t lin = 0;
    int p[3] = {0, 0, 0};
    for (int t = D - 1; t >= 0; --t) {
      p[t] = rem % P;
      rem /= P;
    }
    for (int t = 0; t < D; ++t) {
      int c = org[t] + p[t];
      c = (c % Ms + Ms) % Ms;
      lin = lin * Ms + c;
    }
    tile[i] = grid[lin];
  }
  __syncthreads();

  const int64_t N = a.g.N;
  const int start = a.item_start[item];
  const int cnt = a.item_count[item];
  cplx<R>* f = a.f + rhs * a.f_rs;
  for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
    const int i = start + k;
    const uint32_t L = a.loc[i];
    int l[D];
    R psi[D][2 * MW + 1];
    bool any_edge = false;
#pragma unroll
    for (int t = 0; t < D; ++t) {
      l[t] = (int)((L >> (kLocBits * t)) & kLocMask);
      const bool e = (L >> (kEdgeShift + t)) & 1u;
      any_edge |= e;
      node_window<R, MW>(a.frac[t * N + i], e, a.b, a.mr, a.edge, psi[t]);
    }
    cplx<R> v;
    if (__any(any_edge))
      v = sum_node<R, D, MW, true>(tile, P, l, psi);
    else
      v = sum_node<R, D, MW, false>(tile, P, l, psi);
    f[a.perm[i]] = v;
  }
}

template <typename R, int D, int MW>
static hipError_t spread_dm(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  size_t lds = (size_t)a.g.Ptot * sizeof(cplx<R>);
  hipLaunchKernelGGL((spread_kernel<R, D, MW>), dim3(a.g.nsub, nrhs), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <typename R, int D, int MW>
static hipError_t interp_dm(const InterpArgs<R>& a, int nrhs, hipStream_t s) {
  size_t lds = (size_t)a.g.Ptot * sizeof(cplx<R>);
  hipLaunchKernelGGL((interp_kernel<R, D, MW>), dim3(a.g.nsub, nrhs), dim3(256), lds, s, a);
  return hipGetLastError();
}

#define NFFT_DISPATCH_M(FN, R, D, ARGS, NRHS, S)   \
  switch (ARGS.g.m) {                              \
    case 1: return FN<R, D, 1>(ARGS, NRHS, S);     \
    case 2: return FN<R, D, 2>(ARGS, NRHS, S);     \
    case 3: return FN<R, D, 3>(ARGS, NRHS, S);     \
    case 4: return FN<R, D, 4>(ARGS, NRHS, S);     \
    case 5: return FN<R, D, 5>(ARGS, NRHS, S);     \
    case 6: return FN<R, D, 6>(ARGS, NRHS, S);     \
    case 7: return FN<R, D, 7>(ARGS, NRHS, S);     \
    case 8: return FN<R, D, 8>(ARGS, NRHS, S);     \
    default: return hipErrorInvalidValue;          \
  }

template <typename R>
hipError_t launch_spread(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  if (a.g.nsub == 0) return hipSuccess;
  switch (a.g.d) {
    case 1: NFFT_DISPATCH_M(spread_dm, R, 1, a, nrhs, s)
    case 2: NFFT_DISPATCH_M(spread_dm, R, 2, a, nrhs, s)
    case 3: NFFT_DISPATCH_M(spread_dm, R, 3, a, nrhs, s)
    default: return hipErrorInvalidValue;
  }
}

template <typename R>
hipError_t launch_interp(const InterpArgs<R>& a, int nrhs, hipStream_t s) {
  if (a.g.nsub == 0) return hipSuccess;
  switch (a.g.d) {
    case 1: NFFT_DISPATCH_M(interp_dm, R, 1, a, nrhs, s)
    case 2: NFFT_DISPATCH_M(interp_dm, R, 2, a, nrhs, s)
    case 3: NFFT_DISPATCH_M(interp_dm, R, 3, a, nrhs, s)
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_spread<float>(const SpreadArgs<float>&, int, hipStream_t);
template hipError_t launch_spread<double>(const SpreadArgs<double>&, int, hipStream_t);
template hipError_t launch_interp<float>(const InterpArgs<float>&, int, hipStream_t);
template hipError_t launch_interp<double>(const InterpArgs<double>&, int, hipStream_t);

}  // namespace nfft
