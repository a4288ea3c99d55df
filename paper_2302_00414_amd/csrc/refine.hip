// Norm reductions of the weighted iterative refinement: the squared 2-norms
// of f and of the residuals r = f - A fhat. The residual itself is formed
// where the forward transform writes its window sums, and the update
// fhat += A^* W r where the adjoint's last FFT pass stores. The iterates are
// the partial sums of the Neumann series of (A^* W A)^{-1} in the proof of
// Theorem 3.15 applied to A^* W f; the transforms themselves are the plan's
// forward (Algorithm 2.1) and weighted adjoint (Algorithm 2.4 with (3.7)).
// Norms are summed in float64 in a fixed order (block sums over a fixed
// grid, then one block), so they do not depend on timing.
#include "internal.hpp"

namespace nfft {

namespace {

constexpr int kThreads = 256;

// sum of sh[0..kThreads) into sh[0], pairwise in a fixed order
__device__ __forceinline__ void block_sum(double* sh) {
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w /= 2) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
}

// block sums of |a_i|^2
template <typename R>
__global__ __launch_bounds__(kThreads) void sumsq_kernel(const cplx<R>* __restrict__ a, int64_t n,
                                                         double* __restrict__ partial) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const cplx<R> v = a[i];
    acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
  }
  sh[threadIdx.x] = acc;
  block_sum(sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// *out = sum of partial[0..nb)
__global__ __launch_bounds__(kThreads) void sum_partials_kernel(const double* __restrict__ partial,
                                                                int nb, double* __restrict__ out) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kThreads) acc += partial[i];
  sh[threadIdx.x] = acc;
  block_sum(sh);
  if (threadIdx.x == 0) *out = sh[0];
}

unsigned blocks_for(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return (unsigned)(b < kRefineBlocks ? (b > 0 ? b : 1) : kRefineBlocks);
}

}  // namespace

template <typename R>
hipError_t launch_sumsq(const cplx<R>* a, int64_t n, double* partial, double* out, hipStream_t s) {
  const unsigned nb = blocks_for(n);
  hipLaunchKernelGGL(sumsq_kernel<R>, dim3(nb), dim3(kThreads), 0, s, a, n, partial);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kThreads), 0, s, partial, (int)nb, out);
  return hipGetLastError();
}

template hipError_t launch_sumsq<float>(const cplx<float>*, int64_t, double*, double*, hipStream_t);
template hipError_t launch_sumsq<double>(const cplx<double>*, int64_t, double*, double*, hipStream_t);

}  // namespace nfft
