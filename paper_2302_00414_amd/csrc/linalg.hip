// Float64 vector kernels for the conjugate-gradient solve of the weight
// conditions (Algorithm 3.6): fills, dot products and norms reduced in a fixed
// order (deterministic), fused vector updates and the residual maximum.
#include <algorithm>

#include "dirichlet.hpp"
#include "internal.hpp"

namespace nfft {

namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;  // partial sums of the first pass

__global__ void fill_kernel(cplx<double>* v, int64_t n, double re, double im) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) v[i] = mkc<double>(re, im);
}

__global__ void conj_kernel(cplx<double>* v, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) v[i].y = -v[i].y;
}

// block sums of Re(conj(a_i) b_i) (op 0) or of max |a_i - e_i| with e the
// unit vector at index e_idx (op 1), grid-stride in a fixed order
__global__ __launch_bounds__(kRedThreads) void reduce_pass1(const cplx<double>* a,
                                                            const cplx<double>* b, int64_t n,
                                                            int op, int64_t e_idx,
                                                            double* partial) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads) {
    if (op == 0) {
      acc += a[i].x * b[i].x + a[i].y * b[i].y;
    } else {
      // op 1: distance to the unit vector at e_idx; op 2: to the all-ones vector
      const double dx = a[i].x - ((op == 2 || i == e_idx) ? 1.0 : 0.0);
      acc = fmax(acc, sqrt(dx * dx + a[i].y * a[i].y));
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w /= 2) {
    if (threadIdx.x < w)
      sh[threadIdx.x] = op == 0 ? sh[threadIdx.x] + sh[threadIdx.x + w]
                                : fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kRedThreads) void reduce_pass2(const double* partial, int n, int op,
                                                            double* out) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kRedThreads)
    acc = op == 0 ? acc + partial[i] : fmax(acc, partial[i]);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w /= 2) {
    if (threadIdx.x < w)
      sh[threadIdx.x] = op == 0 ? sh[threadIdx.x] + sh[threadIdx.x + w]
                                : fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// x += alpha p, r -= alpha q
__global__ void cg_update_kernel(cplx<double>* x, cplx<double>* r, const cplx<double>* p,
                                 const cplx<double>* q, int64_t n, double alpha) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i].x += alpha * p[i].x;
  x[i].y += alpha * p[i].y;
  r[i].x -= alpha * q[i].x;
  r[i].y -= alpha * q[i].y;
}

// p = r + beta p
__global__ void cg_direction_kernel(cplx<double>* p, const cplx<double>* r, int64_t n, double beta) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  p[i].x = r[i].x + beta * p[i].x;
  p[i].y = r[i].y + beta * p[i].y;
}

// (3.62): w_j = |I_M| / sum_h |[A A^*]_{j,h}|^2 with
// [A A^*]_{j,h} = prod_t (D_{M/2-1} + e^{-M pi i .})(x_jt - x_ht); every
// thread sums over all h in a fixed order, the coordinates staged in LDS
__global__ __launch_bounds__(256) void pcf_kernel(const double* __restrict__ x, int64_t N, int d,
                                                  int M, cplx<double>* __restrict__ w) {
  __shared__ double xs[256 * 3];
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double xj[3] = {0, 0, 0};
  if (j < N)
    for (int t = 0; t < d; ++t) xj[t] = x[j * d + t];
  double sum = 0.0;
  for (int64_t h0 = 0; h0 < N; h0 += 256) {
    __syncthreads();
    const int64_t hh = h0 + threadIdx.x;
    if (hh < N)
      for (int t = 0; t < d; ++t) xs[threadIdx.x * 3 + t] = x[hh * d + t];
    __syncthreads();
    const int nh = (int)((N - h0) < 256 ? (N - h0) : 256);
    for (int q = 0; q < nh; ++q) {
      double pr = 1.0, pi = 0.0;
      for (int t = 0; t < d; ++t) {
        double re, im;
        dirichlet_term(M, xj[t] - xs[q * 3 + t], &re, &im);
        const double nr = pr * re - pi * im;
        pi = pr * im + pi * re;
        pr = nr;
      }
      sum += pr * pr + pi * pi;
    }
  }
  if (j < N) {
    double md = 1.0;
    for (int t = 0; t < d; ++t) md *= (double)M;
    w[j] = mkc<double>(md / sum, 0.0);
  }
}

unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

size_t reduce_scratch_doubles() { return kRedBlocks + 1; }

hipError_t launch_fill(cplx<double>* v, int64_t n, double re, double im, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(blocks(n)), dim3(256), 0, s, v, n, re, im);
  return hipGetLastError();
}

hipError_t launch_pcf(const double* x, int64_t N, int d, int M, cplx<double>* w, hipStream_t s) {
  hipLaunchKernelGGL(pcf_kernel, dim3(blocks(N)), dim3(256), 0, s, x, N, d, M, w);
  return hipGetLastError();
}

hipError_t launch_conj(cplx<double>* v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(conj_kernel, dim3(blocks(n)), dim3(256), 0, s, v, n);
  return hipGetLastError();
}

// op 0: Re <a, b>; op 1: max_i |a_i - delta_{i, e_idx}|; op 2: max_i |a_i - 1|. The result lands in
// scratch[kRedBlocks] (device); scratch holds reduce_scratch_doubles() values.
hipError_t launch_reduce(const cplx<double>* a, const cplx<double>* b, int64_t n, int op,
                         int64_t e_idx, double* scratch, hipStream_t s) {
  const int nb = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (n + kRedThreads - 1) / kRedThreads));
  hipLaunchKernelGGL(reduce_pass1, dim3(nb), dim3(kRedThreads), 0, s, a, b, n, op, e_idx, scratch);
  hipLaunchKernelGGL(reduce_pass2, dim3(1), dim3(kRedThreads), 0, s, scratch, nb, op,
                     scratch + kRedBlocks);
  return hipGetLastError();
}

hipError_t launch_cg_update(cplx<double>* x, cplx<double>* r, const cplx<double>* p,
                            const cplx<double>* q, int64_t n, double alpha, hipStream_t s) {
  hipLaunchKernelGGL(cg_update_kernel, dim3(blocks(n)), dim3(256), 0, s, x, r, p, q, n, alpha);
  return hipGetLastError();
}

hipError_t launch_cg_direction(cplx<double>* p, const cplx<double>* r, int64_t n, double beta,
                               hipStream_t s) {
  hipLaunchKernelGGL(cg_direction_kernel, dim3(blocks(n)), dim3(256), 0, s, p, r, n, beta);
  return hipGetLastError();
}

}  // namespace nfft
