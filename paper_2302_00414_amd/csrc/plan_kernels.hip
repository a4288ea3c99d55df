// Plan-time kernels: node encoding and the stable bucket sort into tiles.
//
// The sort is a counting sort that keeps, inside every tile, the caller's
// node order: ranks are computed per chunk of kRankChunk nodes (a node's rank
// counts the earlier nodes of its chunk in the same tile), chunk counts are
// prefix-summed per tile, and the scatter writes each node once.
#include <cmath>

#include "internal.hpp"

namespace nfft {

__global__ void encode_kernel(const double* __restrict__ nodes, int64_t N, Geom g,
                              int32_t* __restrict__ bin, uint32_t* __restrict__ loc,
                              double* __restrict__ frac, int* __restrict__ err) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= N) return;
  const double Ms = (double)g.Ms;
  int32_t b = 0;
  uint32_t packed = 0;
  for (int t = 0; t < g.d; ++t) {
    double x = nodes[j * g.d + t];
    if (!isfinite(x)) {
      atomicOr(err, 1);
      x = 0.0;
    }
    // wrap onto [-1/2, 1/2): the transform is 1-periodic in every coordinate
    double xw = x - floor(x + 0.5);
    if (xw >= 0.5) xw -= 1.0;
    // grid units with the cell of l = -M_s/2 at index 0
    double u = xw * Ms + 0.5 * Ms;
    if (u >= Ms) u -= Ms;
    if (u < 0.0) u += Ms;
    double fl = floor(u);
    int cell = (int)fl;
    if (cell >= g.Ms) cell = g.Ms - 1;
    double fr = u - fl;
    int tb = cell / g.T;
    b = b * g.nb + tb;
    packed |= (uint32_t)(cell - tb * g.T) << (kLocBits * t);
    if (fr == 0.0) packed |= 1u << (kEdgeShift + t);
    frac[t * N + j] = fr;
  }
  bin[j] = b;
  loc[j] = packed;
}

__global__ void count_kernel(const int32_t* __restrict__ bin, int64_t N, int32_t* counts) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < N) atomicAdd(&counts[bin[j]], 1);
}

__global__ __launch_bounds__(kRankChunk) void rank_kernel(const int32_t* __restrict__ bin,
                                                          int64_t N, int nbins,
                                                          int32_t* __restrict__ rank,
                                                          int32_t* __restrict__ chunk_count) {
  __shared__ int32_t sb[kRankChunk];
  const int64_t base = (int64_t)blockIdx.x * kRankChunk;
  const int tid = threadIdx.x;
  const int64_t j = base + tid;
  const int n = (int)((N - base) < kRankChunk ? (N - base) : kRankChunk);
  sb[tid] = (tid < n) ? bin[j] : -1;
  __syncthreads();
  if (tid >= n) return;
  const int mine = sb[tid];
  int r = 0;
  for (int i = 0; i < tid; ++i) r += (sb[i] == mine);
  bool last = true;
  for (int i = tid + 1; i < n; ++i)
    if (sb[i] == mine) { last = false; break; }
  rank[j] = r;
  if (last) chunk_count[(int64_t)blockIdx.x * nbins + mine] = r + 1;
}

__global__ void chunk_offsets_kernel(const int32_t* __restrict__ chunk_count,
                                     const int32_t* __restrict__ bin_start, int64_t nchunks,
                                     int nbins, int32_t* __restrict__ offsets) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  int32_t acc = bin_start[b];
  for (int64_t c = 0; c < nchunks; ++c) {
    offsets[c * nbins + b] = acc;
    acc += chunk_count[c * nbins + b];
  }
}

template <typename R>
__device__ __forceinline__ R round_frac(double fr);
template <>
__device__ __forceinline__ double round_frac<double>(double fr) { return fr; }
template <>
__device__ __forceinline__ float round_frac<float>(double fr) {
  // keep the offset strictly below one cell after rounding
  float f = (float)fr;
  return f < 1.0f ? f : 0x1.fffffep-1f;
}

template <typename R>
__global__ void scatter_kernel(const int32_t* __restrict__ bin, const int32_t* __restrict__ rank,
                               const int32_t* __restrict__ offsets,
                               const uint32_t* __restrict__ loc_u,
                               const double* __restrict__ frac_u, int64_t N, int d, int nbins,
                               int32_t* __restrict__ perm, uint32_t* __restrict__ loc,
                               R* __restrict__ frac) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= N) return;
  int64_t c = j / kRankChunk;
  int32_t dest = offsets[c * nbins + bin[j]] + rank[j];
  perm[dest] = (int32_t)j;
  loc[dest] = loc_u[j];
  for (int t = 0; t < d; ++t) frac[t * N + dest] = round_frac<R>(frac_u[t * N + j]);
}

// Stable sort of every tile's nodes by their tile-local cell in dimension 0
// (the tile row), one work-group per tile: row counts, their prefix sums,
// then chunks of 256 nodes scattered with in-chunk ranks counted in order.
template <typename R>
__global__ __launch_bounds__(256) void row_sort_kernel(const int32_t* __restrict__ bstart, int T,
                                                       int64_t N, int d,
                                                       const int32_t* __restrict__ perm,
                                                       const uint32_t* __restrict__ loc,
                                                       const R* __restrict__ frac,
                                                       int32_t* __restrict__ perm2,
                                                       uint32_t* __restrict__ loc2,
                                                       R* __restrict__ frac2) {
  __shared__ int start[257];  // T <= 256
  __shared__ int rows[256];
  const int tid = threadIdx.x;
  const int s = bstart[blockIdx.x], e = bstart[blockIdx.x + 1];
  if (s == e) return;
  for (int r = tid; r <= T; r += 256) start[r] = 0;
  __syncthreads();
  for (int i = s + tid; i < e; i += 256) atomicAdd(&start[(int)(loc[i] & kLocMask) + 1], 1);
  __syncthreads();
  if (tid == 0)
    for (int r = 1; r <= T; ++r) start[r] += start[r - 1];
  __syncthreads();
  for (int c0 = s; c0 < e; c0 += 256) {
    const int i = c0 + tid;
    const int r = i < e ? (int)(loc[i] & kLocMask) : -1;
    rows[tid] = r;
    __syncthreads();
    if (i < e) {
      int rank = 0;
      for (int t = 0; t < tid; ++t) rank += rows[t] == r;
      const int dst = s + start[r] + rank;
      perm2[dst] = perm[i];
      loc2[dst] = loc[i];
      for (int t = 0; t < d; ++t) frac2[t * N + dst] = frac[t * N + i];
    }
    __syncthreads();
    if (tid < T) {
      int c = 0;
      for (int t = 0; t < 256; ++t) c += rows[t] == tid;
      start[tid] += c;
    }
    __syncthreads();
  }
}

template <typename R>
__global__ void permute_weights_kernel(const double* __restrict__ w,
                                       const int32_t* __restrict__ perm, int64_t N,
                                       cplx<R>* __restrict__ ws) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  int64_t j = perm[i];
  ws[i] = mkc<R>((R)w[2 * j], (R)w[2 * j + 1]);
}

static inline unsigned grid1(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_encode(const double* nodes, int64_t N, const Geom& g, int32_t* bin,
                         uint32_t* loc, double* frac, int* err, hipStream_t s) {
  hipLaunchKernelGGL(encode_kernel, dim3(grid1(N, 256)), dim3(256), 0, s, nodes, N, g, bin, loc,
                     frac, err);
  return hipGetLastError();
}

hipError_t launch_count(const int32_t* bin, int64_t N, int32_t* counts, hipStream_t s) {
  hipLaunchKernelGGL(count_kernel, dim3(grid1(N, 256)), dim3(256), 0, s, bin, N, counts);
  return hipGetLastError();
}

hipError_t launch_rank(const int32_t* bin, int64_t N, int nbins, int32_t* rank,
                       int32_t* chunk_count, hipStream_t s) {
  hipLaunchKernelGGL(rank_kernel, dim3(grid1(N, kRankChunk)), dim3(kRankChunk), 0, s, bin, N,
                     nbins, rank, chunk_count);
  return hipGetLastError();
}

hipError_t launch_chunk_offsets(const int32_t* chunk_count, const int32_t* bin_start,
                                int64_t nchunks, int nbins, int32_t* offsets, hipStream_t s) {
  hipLaunchKernelGGL(chunk_offsets_kernel, dim3(grid1(nbins, 256)), dim3(256), 0, s, chunk_count,
                     bin_start, nchunks, nbins, offsets);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_scatter(const int32_t* bin, const int32_t* rank, const int32_t* offsets,
                          const uint32_t* loc_u, const double* frac_u, int64_t N, int d,
                          int nbins, int32_t* perm, uint32_t* loc, R* frac, hipStream_t s) {
  hipLaunchKernelGGL(scatter_kernel<R>, dim3(grid1(N, 256)), dim3(256), 0, s, bin, rank, offsets,
                     loc_u, frac_u, N, d, nbins, perm, loc, frac);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_row_sort(const int32_t* bstart, int nbins, int T, int64_t N, int d,
                           const int32_t* perm, const uint32_t* loc, const R* frac, int32_t* perm2,
                           uint32_t* loc2, R* frac2, hipStream_t s) {
  if (T > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(row_sort_kernel<R>, dim3(nbins), dim3(256), 0, s, bstart, T, N, d, perm, loc,
                     frac, perm2, loc2, frac2);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_permute_weights(const double* w, const int32_t* perm, int64_t N,
                                  cplx<R>* w_sorted, hipStream_t s) {
  hipLaunchKernelGGL(permute_weights_kernel<R>, dim3(grid1(N, 256)), dim3(256), 0, s, w, perm, N,
                     w_sorted);
  return hipGetLastError();
}

// Zero the padded-tile slots of the tiles that hold no nodes (no work item
// writes them, and the first FFT pass reads them as zeros).
template <typename R>
__global__ __launch_bounds__(256) void zero_tiles_kernel(cplx<R>* tilep, int64_t tile_rs,
                                                         const int32_t* bins, int nbins, int Ptot) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)nbins * Ptot) return;
  const int b = bins[i / Ptot];
  const int c = (int)(i % Ptot);
  tilep[blockIdx.y * tile_rs + (int64_t)b * Ptot + c] = mkc<R>(0, 0);
}

template <typename R>
hipError_t launch_zero_tiles(cplx<R>* tilep, int64_t tile_rs, const int32_t* bins, int nbins,
                             int Ptot, int nrhs, hipStream_t s) {
  if (nbins == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_tiles_kernel<R>, dim3(grid1((int64_t)nbins * Ptot, 256), nrhs),
                     dim3(256), 0, s, tilep, tile_rs, bins, nbins, Ptot);
  return hipGetLastError();
}

template hipError_t launch_zero_tiles<float>(cplx<float>*, int64_t, const int32_t*, int, int, int,
                                             hipStream_t);
template hipError_t launch_zero_tiles<double>(cplx<double>*, int64_t, const int32_t*, int, int,
                                              int, hipStream_t);
template hipError_t launch_scatter<float>(const int32_t*, const int32_t*, const int32_t*,
                                          const uint32_t*, const double*, int64_t, int, int,
                                          int32_t*, uint32_t*, float*, hipStream_t);
template hipError_t launch_scatter<double>(const int32_t*, const int32_t*, const int32_t*,
                                           const uint32_t*, const double*, int64_t, int, int,
                                           int32_t*, uint32_t*, double*, hipStream_t);
template hipError_t launch_row_sort<float>(const int32_t*, int, int, int64_t, int, const int32_t*,
                                           const uint32_t*, const float*, int32_t*, uint32_t*,
                                           float*, hipStream_t);
template hipError_t launch_row_sort<double>(const int32_t*, int, int, int64_t, int, const int32_t*,
                                            const uint32_t*, const double*, int32_t*, uint32_t*,
                                            double*, hipStream_t);
template hipError_t launch_permute_weights<float>(const double*, const int32_t*, int64_t,
                                                  cplx<float>*, hipStream_t);
template hipError_t launch_permute_weights<double>(const double*, const int32_t*, int64_t,
                                                   cplx<double>*, hipStream_t);

}  // namespace nfft
