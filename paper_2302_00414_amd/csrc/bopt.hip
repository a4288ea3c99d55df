// Optimized sparse matrix B_opt (Algorithm 4.3) and its adjoint spreading
// (Algorithm 4.4 step 1, B_opt^* f), float64 precompute.
//
// B_opt has the nonzero pattern of B: column l (a cell of the oversampled
// grid, numbered in C order of s_t = l_t + M_s/2) holds the nodes whose
// closed window support reaches l periodically. Per column the values
// minimise ||H_l b - |I_Ms|^{-1} D^{-1} f_l||_2 over real b, i.e. solve the
// real normal equations Re(H_l^* H_l) b = Re(v_l) with
//   [H_l^* H_l]_{hj} = prod_t (D_{M/2-1}(x_ht - x_jt) + e^{-M pi i (x_ht - x_jt)})   (4.13),
//   v_j = prod_t sum_{k=-M/2}^{M/2-1} w^(k) e^{2 pi i k (x_jt - l_t/M_s)}            (4.14),
// D_{M/2-1}(s) = sin((M-1) pi s)/sin(pi s). One work-group per column builds
// the packed lower triangle of the Gram matrix in LDS, factors it by Cholesky
// and solves by forward and back substitution. A column with more nodes than
// the polynomials of degree M tell apart inside one window support (or with
// duplicate nodes) has singular normal equations: a pivot falls below a
// relative threshold. Such a column is factorised again with a ridge of
// 1e-12 times the Gram diagonal (|I_M|), and its solution then reaches the
// least-squares objective (a Cholesky that only zeroes the small pivots loses
// the fit there by orders of magnitude); other columns are solved exactly. Columns whose triangle does not
// fit in LDS (dense node sets, sigma near 1) take the same steps with the
// triangle and the per-node arrays in a device-memory workspace, one per
// work-group, in batches.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dirichlet.hpp"
#include "internal.hpp"

namespace nfft {

namespace {

__device__ __forceinline__ double wrap_half(double x) {
  double y = x - floor(x + 0.5);
  return y >= 0.5 ? y - 1.0 : y;
}

// Each node visits the (2m+1)^d candidate cells of its closed support; op 0
// counts nodes per column, op 1 writes node ids at col_ptr[c] + fill[c]++.
__global__ void bopt_pattern_kernel(const double* __restrict__ nodes, int64_t N, int d, int Ms,
                                    int m, int op, int* __restrict__ count,
                                    const int64_t* __restrict__ col_ptr,
                                    int* __restrict__ fill, int32_t* __restrict__ col_node) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= N) return;
  double u[3];
  int lo[3];
  for (int t = 0; t < d; ++t) {
    u[t] = wrap_half(nodes[j * d + t]) * Ms + 0.5 * Ms;
    lo[t] = (int)ceil(u[t] - m);
  }
  const int K = 2 * m + 1;
  int total = 1;
  for (int t = 0; t < d; ++t) total *= K;
  for (int q = 0; q < total; ++q) {
    int rem = q;
    int64_t c = 0;
    bool ok = true;
    for (int t = 0; t < d; ++t) {
      const int o = rem % K;
      rem /= K;
      const int l = lo[t] + o;
      ok = ok && fabs(u[t] - (double)l) <= (double)m;
      c = c * Ms + (int64_t)(((l % Ms) + Ms) % Ms);
    }
    if (!ok) continue;
    if (op == 0) {
      atomicAdd(count + c, 1);
    } else {
      const int pos = atomicAdd(fill + c, 1);
      col_node[col_ptr[c] + pos] = (int32_t)j;
    }
  }
}

// sum_{k=-M/2}^{M/2-1} w^(k) e^{2 pi i k s} for an even table w^ (entry
// k + M/2): the cosine series by Clenshaw's recurrence plus the unpaired
// term k = -M/2
__device__ __forceinline__ void window_series(const double* __restrict__ wh, int M, double s,
                                              double* re, double* im) {
  const int H = M / 2;
  double c, sn;
  sincospi(2.0 * s, &sn, &c);
  double b1 = 0.0, b2 = 0.0;
  for (int k = H - 1; k >= 1; --k) {
    const double b0 = 2.0 * wh[H + k] + 2.0 * c * b1 - b2;
    b2 = b1;
    b1 = b0;
  }
  // sum_{k=1}^{H-1} 2 w^(k) cos(2 pi k s) = b1 cos - b2 (with a_0 = 0)
  double cm, sm;
  sincospi((double)M * s, &sm, &cm);
  *re = wh[H] + b1 * c - b2 + wh[0] * cm;
  *im = -wh[0] * sm;
}

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }  // i >= j

// Right-looking Cholesky of the packed lower triangle A (n x n), one
// column per step, for triangles in LDS. A pivot at or below tol gives a zero
// column of L (its node is dropped); with stop_at_drop the factorisation
// ends at the first such pivot. Returns whether a pivot was dropped.
__device__ bool chol_unblocked(double* A, int n, double tol, bool stop_at_drop) {
  const int tid = threadIdx.x, NT = blockDim.x;
  bool dropped = false;
  for (int k = 0; k < n; ++k) {
    const double akk = A[tri(k, k)];
    const bool keep = akk > tol;
    if (!keep && stop_at_drop) return true;  // uniform: every thread read akk
    dropped = dropped || !keep;
    const double lkk = keep ? sqrt(akk) : 0.0;
    __syncthreads();
    if (tid == 0) A[tri(k, k)] = lkk;
    for (int i = k + 1 + tid; i < n; i += NT) A[tri(i, k)] = keep ? A[tri(i, k)] / lkk : 0.0;
    __syncthreads();
    if (keep) {
      const int rest = n - k - 1;
      const int nup = rest * (rest + 1) / 2;
      for (int q = tid; q < nup; q += NT) {
        int i = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
        while (tri(i, 0) > q) --i;
        while (tri(i + 1, 0) <= q) ++i;
        const int j = q - tri(i, 0);
        const int ii = k + 1 + i, jj = k + 1 + j;
        A[tri(ii, jj)] -= A[tri(ii, k)] * A[tri(jj, k)];
      }
    }
    __syncthreads();
  }
  return dropped;
}

// The same factorisation for triangles in device memory, by panels of kPB
// columns: the panel's diagonal block is factorised in LDS (one column per
// step, as above), the rows below it solve against that block (one thread per
// row, the row's kPB values in registers), and the trailing triangle takes
// the panel's rank-kPB update in kTB x kTB tiles staged through LDS, each
// thread holding a 4 x 4 block of sums. Only the order of the roundings
// differs from the one-column-per-step form. 256 threads.
constexpr int kPB = 32;
constexpr int kTB = 64;

__device__ bool chol_blocked(double* A, int n, double tol, bool stop_at_drop) {
  __shared__ double Dg[kPB][kPB + 1];
  __shared__ double Li[kTB][kPB + 1];
  __shared__ double Lj[kTB][kPB + 1];
  const int tid = threadIdx.x;
  bool dropped = false;
  for (int k0 = 0; k0 < n; k0 += kPB) {
    const int kb = min(kPB, n - k0);
    // diagonal block
    for (int e = tid; e < kPB * kPB; e += 256) {
      const int i = e / kPB, j = e % kPB;
      if (i < kb && j <= i) Dg[i][j] = A[tri(k0 + i, k0 + j)];
    }
    __syncthreads();
    for (int k = 0; k < kb; ++k) {
      const double akk = Dg[k][k];
      const bool keep = akk > tol;
      if (!keep && stop_at_drop) return true;  // uniform: every thread read akk
      dropped = dropped || !keep;
      const double lkk = keep ? sqrt(akk) : 0.0;
      __syncthreads();
      if (tid == 0) Dg[k][k] = lkk;
      if (tid > k && tid < kb) Dg[tid][k] = keep ? Dg[tid][k] / lkk : 0.0;
      __syncthreads();
      if (keep)
        for (int e = tid; e < kPB * kPB; e += 256) {
          const int i = e / kPB, j = e % kPB;
          if (j > k && j <= i && i < kb) Dg[i][j] -= Dg[i][k] * Dg[j][k];
        }
      __syncthreads();
    }
    for (int e = tid; e < kPB * kPB; e += 256) {
      const int i = e / kPB, j = e % kPB;
      if (i < kb && j <= i) A[tri(k0 + i, k0 + j)] = Dg[i][j];
    }
    // rows below the block: l_ip = (a_ip - sum_{q<p} l_iq l_pq) / l_pp
    for (int i = k0 + kb + tid; i < n; i += 256) {
      double* row = A + tri(i, k0);
      double l[kPB];
#pragma unroll
      for (int p = 0; p < kPB; ++p) l[p] = p < kb ? row[p] : 0.0;
#pragma unroll
      for (int p = 0; p < kPB; ++p) {
        double sacc = l[p];
#pragma unroll
        for (int q = 0; q < p; ++q) sacc -= l[q] * Dg[p][q];
        const double dpp = p < kb ? Dg[p][p] : 0.0;
        l[p] = dpp > 0.0 ? sacc / dpp : 0.0;
      }
#pragma unroll
      for (int p = 0; p < kPB; ++p)
        if (p < kb) row[p] = l[p];
    }
    __syncthreads();
    // trailing update of rows and columns >= k0 + kb, lower tiles only
    const int r0 = k0 + kb;
    const int T = (n - r0 + kTB - 1) / kTB;
    const int tr = tid >> 4, tc = tid & 15;
    for (int t = 0; t < T * (T + 1) / 2; ++t) {
      int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
      while (ti * (ti + 1) / 2 > t) --ti;
      while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
      const int tj = t - ti * (ti + 1) / 2;
      const int i0 = r0 + ti * kTB, j0 = r0 + tj * kTB;
      for (int e = tid; e < kTB * kPB; e += 256) {
        const int r = e / kPB, q = e % kPB;
        const int i = i0 + r, j = j0 + r;
        Li[r][q] = (i < n && q < kb) ? A[tri(i, k0 + q)] : 0.0;
        Lj[r][q] = (j < n && q < kb) ? A[tri(j, k0 + q)] : 0.0;
      }
      __syncthreads();
      double acc[4][4] = {};
#pragma unroll 4
      for (int q = 0; q < kPB; ++q) {
        double li[4], lj[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) li[a] = Li[tr + 16 * a][q];
#pragma unroll
        for (int b = 0; b < 4; ++b) lj[b] = Lj[tc + 16 * b][q];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] += li[a] * lj[b];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int i = i0 + tr + 16 * a;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int j = j0 + tc + 16 * b;
          if (i < n && j <= i) A[tri(i, j)] -= acc[a][b];
        }
      }
      __syncthreads();
    }
  }
  return dropped;
}

// One work-group per column. cols: the columns to solve (blockIdx.x indexes
// it), or null for all. ws null: the triangle and the per-node arrays live in
// dynamic LDS, laid out for nmax nodes (columns of more than nmax nodes are
// left to the other launch); else at ws + ws_off[blockIdx.x] in device
// memory, laid out for the column's own n (bopt_workspace_doubles(n)
// doubles), and the factorisation goes by panels.
template <typename R, bool BLOCKED>
__global__ __launch_bounds__(256) void bopt_solve_kernel(
    const double* __restrict__ nodes, int d, int M, int Ms, const double* __restrict__ wh,
    const int64_t* __restrict__ col_ptr, int32_t* __restrict__ col_node, R* __restrict__ col_val,
    int nmax, double piv_rel, double ridge, int* __restrict__ dropped,
    const int64_t* __restrict__ cols, double* ws, const int64_t* __restrict__ ws_off) {
  extern __shared__ double sm[];
  const int64_t c = cols ? cols[blockIdx.x] : (int64_t)blockIdx.x;
  const int64_t start = col_ptr[c];
  const int n = (int)(col_ptr[c + 1] - start);
  if (n == 0 || n > nmax) return;
  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  const int nl = BLOCKED ? n : nmax;  // layout size
  // packed lower triangle, n(n+1)/2
  double* A = BLOCKED ? ws + ws_off[blockIdx.x] : sm;
  double* xs = A + (size_t)nl * (nl + 1) / 2;   // n x 3 coordinates
  double* v = xs + (size_t)nl * 3;              // right side, then solution
  int* ids = reinterpret_cast<int*>(v + nl);    // sorted node ids
  int* idr = ids + nl;                          // unsorted
  __shared__ int ridged;
  if (tid == 0) ridged = 0;
  for (int i = tid; i < n; i += NT) idr[i] = col_node[start + i];
  __syncthreads();
  // rank sort (ids are distinct): deterministic order by node id
  for (int i = tid; i < n; i += NT) {
    const int me = idr[i];
    int r = 0;
    for (int q = 0; q < n; ++q) r += idr[q] < me;
    ids[r] = me;
  }
  __syncthreads();
  // grid index of this column: l_t = s_t - M_s/2
  int64_t cc = c;
  double lt[3] = {0, 0, 0};
  for (int t = d - 1; t >= 0; --t) {
    lt[t] = (double)(cc % Ms) - 0.5 * Ms;
    cc /= Ms;
  }
  for (int i = tid; i < n; i += NT)
    for (int t = 0; t < d; ++t) xs[i * 3 + t] = wrap_half(nodes[(int64_t)ids[i] * d + t]);
  __syncthreads();
  // right side (4.14), real part
  for (int i = tid; i < n; i += NT) {
    double pr = 1.0, pi = 0.0;
    for (int t = 0; t < d; ++t) {
      double re, im;
      window_series(wh, M, xs[i * 3 + t] - lt[t] / Ms, &re, &im);
      const double nr = pr * re - pi * im;
      pi = pr * im + pi * re;
      pr = nr;
    }
    v[i] = pr;
  }
  // Gram matrix (4.13), real part, lower triangle, and its Cholesky factor.
  // A pivot below piv_rel * |I_M| (the diagonal of H^* H) marks a dependent
  // node: the normal equations are singular, the first factorisation stops
  // there and the Gram matrix is factorised again with the ridge on its
  // diagonal; a pivot still below the threshold then drops its node (its
  // column of L and its value are zero).
  double tol = piv_rel;
  for (int t = 0; t < d; ++t) tol *= (double)M;
  const int npairs = n * (n + 1) / 2;
  for (int pass = 0; pass < 2; ++pass) {
    const double rid = pass ? ridge : 0.0;
    for (int q = tid; q < npairs; q += NT) {
      int i = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
      while (tri(i, 0) > q) --i;
      while (tri(i + 1, 0) <= q) ++i;
      const int j = q - tri(i, 0);
      double pr = 1.0, pi = 0.0;
      for (int t = 0; t < d; ++t) {
        double re, im;
        dirichlet_term(M, xs[i * 3 + t] - xs[j * 3 + t], &re, &im);
        const double nr = pr * re - pi * im;
        pi = pr * im + pi * re;
        pr = nr;
      }
      A[q] = i == j ? pr + rid : pr;
    }
    __syncthreads();
    bool singular;
    if constexpr (BLOCKED)
      singular = chol_blocked(A, n, tol, pass == 0);
    else
      singular = chol_unblocked(A, n, tol, pass == 0);
    __syncthreads();  // every thread is done with A before it is refilled
    if (!singular || pass == 1) break;
    if (tid == 0) ridged = 1;
  }
  // forward substitution L y = v
  for (int k = 0; k < n; ++k) {
    const double lkk = A[tri(k, k)];
    __syncthreads();
    if (tid == 0) v[k] = lkk > 0.0 ? v[k] / lkk : 0.0;
    __syncthreads();
    const double yk = v[k];
    for (int i = k + 1 + tid; i < n; i += NT) v[i] -= A[tri(i, k)] * yk;
    __syncthreads();
  }
  // back substitution L^T b = y
  for (int k = n - 1; k >= 0; --k) {
    const double lkk = A[tri(k, k)];
    if (tid == 0) v[k] = lkk > 0.0 ? v[k] / lkk : 0.0;
    __syncthreads();
    const double bk = v[k];
    for (int i = tid; i < k; i += NT) v[i] -= A[tri(k, i)] * bk;
    __syncthreads();
  }
  for (int i = tid; i < n; i += NT) {
    col_node[start + i] = ids[i];
    col_val[start + i] = (R)v[i];
  }
  if (tid == 0 && ridged) atomicAdd(dropped, 1);
}

// g_c = scale * sum over the column's nodes of b_cj f_j, G lanes per column
// (G sized to the mean column length, so that short columns do not leave most
// of a wave idle); scale converts to the units of the library's normalised
// window, which the deconvolution table of the FFT passes expects
template <typename R, int G>
__global__ __launch_bounds__(256) void bopt_apply_kernel(const int64_t* __restrict__ col_ptr,
                                                         const int32_t* __restrict__ col_node,
                                                         const R* __restrict__ col_val,
                                                         const cplx<R>* __restrict__ f,
                                                         int64_t f_rs, cplx<R>* __restrict__ grid,
                                                         int64_t g_rs, int64_t ncols, double scale) {
  const int64_t c = blockIdx.x * (int64_t)(256 / G) + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (c >= ncols) return;  // whole lane groups leave together
  const cplx<R>* fr = f + blockIdx.y * f_rs;
  double sx = 0.0, sy = 0.0;
  const int64_t e1 = col_ptr[c + 1];
  int64_t e = col_ptr[c] + lane;
  // two entries per trip, so that two gathers of f are in flight
  for (; e + G < e1; e += 2 * G) {
    const int32_t j0 = col_node[e], j1 = col_node[e + G];
    const double b0 = (double)col_val[e], b1 = (double)col_val[e + G];
    const cplx<R> v0 = fr[j0], v1 = fr[j1];
    sx += b0 * (double)v0.x;
    sy += b0 * (double)v0.y;
    sx += b1 * (double)v1.x;
    sy += b1 * (double)v1.y;
  }
  if (e < e1) {
    const cplx<R> v = fr[col_node[e]];
    const double b = (double)col_val[e];
    sx += b * (double)v.x;
    sy += b * (double)v.y;
  }
  for (int w = G / 2; w > 0; w >>= 1) {
    sx += __shfl_xor(sx, w);
    sy += __shfl_xor(sy, w);
  }
  if (lane == 0) grid[blockIdx.y * g_rs + c] = mkc<R>((R)(sx * scale), (R)(sy * scale));
}

// First cell of every node's closed support, per dimension (caller order).
__global__ void bopt_lo_kernel(const double* __restrict__ nodes, int64_t N, int d, int Ms, int m,
                               int32_t* __restrict__ lo) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= N) return;
  for (int t = 0; t < d; ++t)
    lo[j * d + t] = (int32_t)ceil(wrap_half(nodes[j * d + t]) * Ms + 0.5 * Ms - m);
}

// B_opt by rows: the value of node j in its footprint cell q (offsets
// q_t = s_t - lo_t in [0, 2m], q = sum q_t (2m+1)^(d-1-t)); cells outside the
// support stay zero. One thread per column; every (node, cell) pair is
// written once.
template <typename R>
__global__ void bopt_rows_kernel(const int64_t* __restrict__ col_ptr,
                                 const int32_t* __restrict__ col_node,
                                 const R* __restrict__ col_val, int64_t ncols, int d, int Ms,
                                 int m, const int32_t* __restrict__ lo, R* __restrict__ rows) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  const int K = 2 * m + 1;
  int F = 1;
  for (int t = 0; t < d; ++t) F *= K;
  int s[3];
  int64_t cc = c;
  for (int t = d - 1; t >= 0; --t) {
    s[t] = (int)(cc % Ms);
    cc /= Ms;
  }
  for (int64_t e = col_ptr[c]; e < col_ptr[c + 1]; ++e) {
    const int j = col_node[e];
    int q = 0;
    for (int t = 0; t < d; ++t) q = q * K + (((s[t] - lo[(int64_t)j * d + t]) % Ms) + Ms) % Ms;
    rows[(int64_t)j * F + q] = col_val[e];
  }
}

// f_j = scale * sum over the node's support of b_jl g_l (Remark 4.6's
// f = B_opt F D h, with g = F D h from the forward FFT passes)
template <typename R>
__global__ void bopt_gather_kernel(const int32_t* __restrict__ lo, const R* __restrict__ rows,
                                   const cplx<R>* __restrict__ grid, int64_t g_rs, int64_t N,
                                   int d, int Ms, int m, cplx<R>* __restrict__ f, int64_t f_rs,
                                   double scale) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= N) return;
  const cplx<R>* g = grid + blockIdx.y * g_rs;
  const int K = 2 * m + 1;
  int F = 1;
  for (int t = 0; t < d; ++t) F *= K;
  int l[3] = {0, 0, 0};
  for (int t = 0; t < d; ++t) l[t] = lo[j * d + t];
  double sx = 0.0, sy = 0.0;
  for (int q = 0; q < F; ++q) {
    const R b = rows[j * F + q];
    if (b == (R)0) continue;
    int rem = q;
    int64_t cell = 0;
    int o[3];
    for (int t = d - 1; t >= 0; --t) {
      o[t] = rem % K;
      rem /= K;
    }
    for (int t = 0; t < d; ++t) cell = cell * Ms + (((l[t] + o[t]) % Ms) + Ms) % Ms;
    const cplx<R> v = g[cell];
    sx += (double)b * (double)v.x;
    sy += (double)b * (double)v.y;
  }
  f[blockIdx.y * f_rs + j] = mkc<R>((R)(sx * scale), (R)(sy * scale));
}

unsigned grid1(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_bopt_lo(const double* nodes, int64_t N, int d, int Ms, int m, int32_t* lo,
                          hipStream_t s) {
  hipLaunchKernelGGL(bopt_lo_kernel, dim3(grid1(N, 256)), dim3(256), 0, s, nodes, N, d, Ms, m, lo);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_bopt_rows(const int64_t* col_ptr, const int32_t* col_node, const R* col_val,
                            int64_t ncols, int d, int Ms, int m, const int32_t* lo, R* rows,
                            hipStream_t s) {
  hipLaunchKernelGGL(bopt_rows_kernel<R>, dim3(grid1(ncols, 256)), dim3(256), 0, s, col_ptr,
                     col_node, col_val, ncols, d, Ms, m, lo, rows);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_bopt_gather(const int32_t* lo, const R* rows, const cplx<R>* grid, int64_t g_rs,
                              int64_t N, int d, int Ms, int m, cplx<R>* f, int64_t f_rs, int nrhs,
                              double scale, hipStream_t s) {
  hipLaunchKernelGGL(bopt_gather_kernel<R>, dim3(grid1(N, 256), nrhs), dim3(256), 0, s, lo, rows,
                     grid, g_rs, N, d, Ms, m, f, f_rs, scale);
  return hipGetLastError();
}

template hipError_t launch_bopt_rows<float>(const int64_t*, const int32_t*, const float*, int64_t,
                                            int, int, int, const int32_t*, float*, hipStream_t);
template hipError_t launch_bopt_rows<double>(const int64_t*, const int32_t*, const double*, int64_t,
                                             int, int, int, const int32_t*, double*, hipStream_t);
template hipError_t launch_bopt_gather<float>(const int32_t*, const float*, const cplx<float>*,
                                              int64_t, int64_t, int, int, int, cplx<float>*,
                                              int64_t, int, double, hipStream_t);
template hipError_t launch_bopt_gather<double>(const int32_t*, const double*, const cplx<double>*,
                                               int64_t, int64_t, int, int, int, cplx<double>*,
                                               int64_t, int, double, hipStream_t);

hipError_t launch_bopt_pattern(const double* nodes, int64_t N, int d, int Ms, int m, int op,
                               int* count, const int64_t* col_ptr, int* fill, int32_t* col_node,
                               hipStream_t s) {
  hipLaunchKernelGGL(bopt_pattern_kernel, dim3(grid1(N, 256)), dim3(256), 0, s, nodes, N, d, Ms, m,
                     op, count, col_ptr, fill, col_node);
  return hipGetLastError();
}

// Doubles of one column's workspace: the packed triangle and the per-node
// arrays (coordinates, right side / solution, two id arrays).
int64_t bopt_workspace_doubles(int n) {
  return (int64_t)n * (n + 1) / 2 + (int64_t)n * 4 + n;
}

// dynamic LDS of the column solve with everything in LDS for columns of up
// to nmax nodes (plus 64 bytes of headroom for the kernel's static LDS)
size_t bopt_solve_lds(int nmax) {
  return (size_t)bopt_workspace_doubles(nmax) * sizeof(double) + 64;
}

template <typename R>
hipError_t launch_bopt_solve(const double* nodes, int d, int M, int Ms, const double* wh,
                             const int64_t* col_ptr, int32_t* col_node, R* col_val, int64_t ncols,
                             int nmax, double piv_rel, double ridge, int* dropped,
                             const int64_t* cols, double* ws, const int64_t* ws_off,
                             hipStream_t s) {
  if (ncols == 0) return hipSuccess;
  if (ws)
    hipLaunchKernelGGL((bopt_solve_kernel<R, true>), dim3((unsigned)ncols), dim3(256), 0, s,
                       nodes, d, M, Ms, wh, col_ptr, col_node, col_val, nmax, piv_rel, ridge,
                       dropped, cols, ws, ws_off);
  else
    hipLaunchKernelGGL((bopt_solve_kernel<R, false>), dim3((unsigned)ncols), dim3(256),
                       bopt_solve_lds(nmax), s, nodes, d, M, Ms, wh, col_ptr, col_node, col_val,
                       nmax, piv_rel, ridge, dropped, cols, ws, ws_off);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_bopt_apply(const int64_t* col_ptr, const int32_t* col_node, const R* col_val,
                             const cplx<R>* f, int64_t f_rs, cplx<R>* grid, int64_t g_rs,
                             int64_t ncols, int nrhs, double scale, int lanes, hipStream_t s) {
  const dim3 grid_of(grid1(ncols, 256 / lanes), nrhs);
#define NFFT_BOPT_APPLY(G)                                                                    \
  hipLaunchKernelGGL((bopt_apply_kernel<R, G>), grid_of, dim3(256), 0, s, col_ptr, col_node, \
                     col_val, f, f_rs, grid, g_rs, ncols, scale)
  switch (lanes) {
    case 4: NFFT_BOPT_APPLY(4); break;
    case 8: NFFT_BOPT_APPLY(8); break;
    case 16: NFFT_BOPT_APPLY(16); break;
    case 32: NFFT_BOPT_APPLY(32); break;
    case 64: NFFT_BOPT_APPLY(64); break;
    default: return hipErrorInvalidValue;
  }
#undef NFFT_BOPT_APPLY
  return hipGetLastError();
}

// lanes per column for columns of mean length avg: a power of two from 4 to
// 64, about an eighth of the mean (at 36 nonzeros per column, 8 lanes
// measured fastest, 4 and 16 slower by 22% and 12%, 64 three times slower)
int bopt_apply_lanes(double avg) {
  int g = 4;
  while (g < 64 && 8.0 * g < avg) g *= 2;
  return g;
}

template hipError_t launch_bopt_solve<float>(const double*, int, int, int, const double*,
                                             const int64_t*, int32_t*, float*, int64_t, int,
                                             double, double, int*, const int64_t*, double*,
                                             const int64_t*, hipStream_t);
template hipError_t launch_bopt_solve<double>(const double*, int, int, int, const double*,
                                              const int64_t*, int32_t*, double*, int64_t, int,
                                              double, double, int*, const int64_t*, double*,
                                              const int64_t*, hipStream_t);
template hipError_t launch_bopt_apply<float>(const int64_t*, const int32_t*, const float*,
                                             const cplx<float>*, int64_t, cplx<float>*, int64_t,
                                             int64_t, int, double, int, hipStream_t);
template hipError_t launch_bopt_apply<double>(const int64_t*, const int32_t*, const double*,
                                              const cplx<double>*, int64_t, cplx<double>*, int64_t,
                                              int64_t, int, double, int, hipStream_t);

}  // namespace nfft
