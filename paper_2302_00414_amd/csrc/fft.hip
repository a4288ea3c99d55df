// Batched 1-D FFT passes (step 2 of Algorithms 2.1 and 2.4), LDS-resident
// Stockham autosort with radix-8/4/2 butterflies.
//
// One launch transforms every line of one dimension of a d-dimensional
// array. A work-group holds `lpw` whole lines of length L in LDS (two
// ping-pong buffers). Each pass is fused with its neighbours' elementwise
// work:
//   loaders : kLoadMerge      -- the first adjoint pass sums the padded tile
//                                 partials of the spreading step into grid
//                                 cells (fixed order, no atomics);
//             kLoadStrided    -- plain strided read;
//             kLoadPadScaled  -- forward: read the M coefficients of a line,
//                                 multiply by the deconvolution factor and
//                                 zero-pad to L = M_sigma (D and the zero
//                                 padding of Algorithm 2.1 step 1);
//   storers : kStoreCropScaled -- adjoint: keep the M outputs k in I_M,
//                                 multiply by the deconvolution factor (D^*
//                                 and the crop of Algorithm 2.4 step 3);
//             kStoreFull       -- forward: write all M_sigma outputs.
// The deconvolution factor of a dimension also carries the sign (-1)^k that
// moves the grid origin from l = -M_sigma/2 to index 0.
#include "internal.hpp"

namespace nfft {

template <typename R, bool INV>
__device__ __forceinline__ cplx<R> rot_mi(cplx<R> a) {
  // multiply by -i (forward) or +i (inverse)
  return INV ? mkc<R>(-a.y, a.x) : mkc<R>(a.y, -a.x);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft2(cplx<R>* a) {
  cplx<R> t = a[1];
  a[1] = csub<R>(a[0], t);
  a[0] = cadd<R>(a[0], t);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft4(cplx<R>& a0, cplx<R>& a1, cplx<R>& a2, cplx<R>& a3) {
  cplx<R> t0 = cadd<R>(a0, a2), t1 = csub<R>(a0, a2);
  cplx<R> t2 = cadd<R>(a1, a3), t3 = rot_mi<R, INV>(csub<R>(a1, a3));
  a0 = cadd<R>(t0, t2);
  a2 = csub<R>(t0, t2);
  a1 = cadd<R>(t1, t3);
  a3 = csub<R>(t1, t3);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft8(cplx<R>* a) {
  // even / odd radix-4 halves, then combine with w8^k
  cplx<R> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  cplx<R> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<R, INV>(e0, e1, e2, e3);
  dft4<R, INV>(o0, o1, o2, o3);
  const R h = (R)0.70710678118654752440084436210484903928;
  // w8 = e^{-+ 2 pi i / 8}
  cplx<R> w1 = INV ? mkc<R>(h * (o1.x - o1.y), h * (o1.x + o1.y))
                   : mkc<R>(h * (o1.x + o1.y), h * (o1.y - o1.x));
  cplx<R> w2 = rot_mi<R, INV>(o2);
  cplx<R> w3 = INV ? mkc<R>(-h * (o3.x + o3.y), h * (o3.x - o3.y))
                   : mkc<R>(h * (o3.y - o3.x), -h * (o3.x + o3.y));
  a[0] = cadd<R>(e0, o0);
  a[4] = csub<R>(e0, o0);
  a[1] = cadd<R>(e1, w1);
  a[5] = csub<R>(e1, w1);
  a[2] = cadd<R>(e2, w2);
  a[6] = csub<R>(e2, w2);
  a[3] = cadd<R>(e3, w3);
  a[7] = csub<R>(e3, w3);
}

// One Stockham pass of radix RAD over `lpw` lines of length L.
template <typename R, int RAD, bool INV>
__device__ __forceinline__ void stockham_pass(const cplx<R>* src, cplx<R>* dst, int L, int lpw,
                                              int Ns, const cplx<R>* __restrict__ tw) {
  const int nbf = L / RAD;
  for (int q = threadIdx.x; q < lpw * nbf; q += blockDim.x) {
    const int line = q / nbf;
    const int j = q - line * nbf;
    const cplx<R>* s = src + line * L;
    cplx<R>* o = dst + line * L;
    cplx<R> a[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) a[r] = s[j + r * nbf];
    const int jm = j & (Ns - 1);
    if (Ns > 1) {
      const int step = jm * (L / (Ns * RAD));
#pragma unroll
      for (int r = 1; r < RAD; ++r) {
        cplx<R> w = tw[step * r];
        if (INV) w.y = -w.y;
        a[r] = cmul<R>(a[r], w);
      }
    }
    if constexpr (RAD == 8) {
      dft8<R, INV>(a);
    } else if constexpr (RAD == 4) {
      dft4<R, INV>(a[0], a[1], a[2], a[3]);
    } else {
      dft2<R, INV>(a);
    }
    const int idx = (j - jm) * RAD + jm;
#pragma unroll
    for (int r = 0; r < RAD; ++r) o[idx + r * Ns] = a[r];
  }
}

// Sum of the padded tile partials that cover grid cell c (per dimension:
// the own tile and, within m cells of its border, the neighbour tile whose
// padding reaches over; tiles wrap periodically).
template <typename R, int D>
__device__ __forceinline__ cplx<R> merge_cell(const cplx<R>* __restrict__ sub,
                                              const int32_t* __restrict__ item_first,
                                              const Geom& g, const int* c) {
  int bq[3][3], pq[3][3], nq[3];
#pragma unroll
  for (int t = 0; t < D; ++t) {
    const int r = c[t] % g.T;
    const int b0 = c[t] / g.T;
    int n = 0;
#pragma unroll
    for (int dl = -1; dl <= 1; ++dl) {
      const int p = r + g.m - dl * g.T;
      if (p >= 0 && p < g.P) {
        bq[t][n] = (b0 + dl + g.nb) % g.nb;
        pq[t][n] = p;
        ++n;
      }
    }
    nq[t] = n;
  }
  R sx = 0, sy = 0;
  const int n1 = D > 1 ? nq[1] : 1;
  const int n2 = D > 2 ? nq[2] : 1;
  for (int a0 = 0; a0 < nq[0]; ++a0)
    for (int a1 = 0; a1 < n1; ++a1)
      for (int a2 = 0; a2 < n2; ++a2) {
        int bin = bq[0][a0];
        int pl = pq[0][a0];
        if (D > 1) {
          bin = bin * g.nb + bq[1][a1];
          pl = pl * g.P + pq[1][a1];
        }
        if (D > 2) {
          bin = bin * g.nb + bq[2][a2];
          pl = pl * g.P + pq[2][a2];
        }
        const int s0 = item_first[bin], s1 = item_first[bin + 1];
        for (int s = s0; s < s1; ++s) {
          const cplx<R> v = sub[(int64_t)s * g.Ptot + pl];
          sx += v.x;
          sy += v.y;
        }
      }
  return mkc<R>(sx, sy);
}

template <typename R, int LD>
__device__ __forceinline__ cplx<R> load_elem(const FftArgs<R>& a, int b, int64_t o, int64_t i,
                                             int e, int L) {
  if constexpr (LD == kLoadStrided) {
    return a.in[b * a.in_bs + o * a.in_os + i * a.in_is + (int64_t)e * a.in_es];
  } else if constexpr (LD == kLoadPadScaled) {
    const int M = a.g.M;
    int kidx;
    if (e < M / 2)
      kidx = e + M / 2;
    else if (e >= L - M / 2)
      kidx = e - L + M / 2;
    else
      return mkc<R>(0, 0);
    const cplx<R> v = a.in[b * a.in_bs + o * a.in_os + i * a.in_is + (int64_t)kidx * a.in_es];
    return cscale<R>(v, a.fac[kidx]);
  } else {
    // merge: the line index o enumerates the leading d-1 grid coordinates
    int c[3] = {0, 0, 0};
    const int d = a.g.d;
    int64_t rem = o;
    for (int t = d - 2; t >= 0; --t) {
      c[t] = (int)(rem % a.g.Ms);
      rem /= a.g.Ms;
    }
    c[d - 1] = e;
    const cplx<R>* sub = a.sub + b * a.sub_bs;
    if (d == 1) return merge_cell<R, 1>(sub, a.item_first, a.g, c);
    if (d == 2) return merge_cell<R, 2>(sub, a.item_first, a.g, c);
    return merge_cell<R, 3>(sub, a.item_first, a.g, c);
  }
}

template <typename R, int ST>
__device__ __forceinline__ void store_elem(const FftArgs<R>& a, int b, int64_t o, int64_t i,
                                           int e, int L, cplx<R> v) {
  if constexpr (ST == kStoreFull) {
    a.out[b * a.out_bs + o * a.out_os + i * a.out_is + (int64_t)e * a.out_es] = v;
  } else {
    const int M = a.g.M;
    int kidx;
    if (e < M / 2)
      kidx = e + M / 2;
    else if (e >= L - M / 2)
      kidx = e - L + M / 2;
    else
      return;
    a.out[b * a.out_bs + o * a.out_os + i * a.out_is + (int64_t)kidx * a.out_es] =
        cscale<R>(v, a.fac[kidx]);
  }
}

template <typename R, int LOG2L, bool INV, int LD, int ST>
__global__ __launch_bounds__(256) void fft_pass_kernel(FftArgs<R> a) {
  constexpr int L = 1 << LOG2L;
  extern __shared__ unsigned char smem_raw[];
  const int lpw = a.lpw;
  cplx<R>* buf0 = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* buf1 = buf0 + lpw * L;
  const int64_t nlines = a.n_outer * a.n_inner;
  const int64_t q0 = (int64_t)blockIdx.x * lpw;
  const int b = blockIdx.y;

  for (int idx = threadIdx.x; idx < lpw * L; idx += blockDim.x) {
    int l, e;
    if (a.inner_major) {
      l = idx % lpw;
      e = idx / lpw;
    } else {
      l = idx / L;
      e = idx % L;
    }
    const int64_t q = q0 + l;
    cplx<R> v = mkc<R>(0, 0);
    if (q < nlines) {
      const int64_t o = q / a.n_inner, i = q % a.n_inner;
      v = load_elem<R, LD>(a, b, o, i, e, L);
    }
    buf0[l * L + e] = v;
  }
  __syncthreads();

  cplx<R>* src = buf0;
  cplx<R>* dst = buf1;
  int Ns = 1;
  constexpr int n8 = LOG2L / 3;
  constexpr int rem = LOG2L % 3;
#pragma unroll 1
  for (int p = 0; p < n8; ++p) {
    stockham_pass<R, 8, INV>(src, dst, L, lpw, Ns, a.tw);
    __syncthreads();
    cplx<R>* t = src;
    src = dst;
    dst = t;
    Ns *= 8;
  }
  if constexpr (rem == 2) {
    stockham_pass<R, 4, INV>(src, dst, L, lpw, Ns, a.tw);
    __syncthreads();
    cplx<R>* t = src;
    src = dst;
    dst = t;
  } else if constexpr (rem == 1) {
    stockham_pass<R, 2, INV>(src, dst, L, lpw, Ns, a.tw);
    __syncthreads();
    cplx<R>* t = src;
    src = dst;
    dst = t;
  }

  for (int idx = threadIdx.x; idx < lpw * L; idx += blockDim.x) {
    int l, e;
    if (a.inner_major) {
      l = idx % lpw;
      e = idx / lpw;
    } else {
      l = idx / L;
      e = idx % L;
    }
    const int64_t q = q0 + l;
    if (q < nlines) {
      const int64_t o = q / a.n_inner, i = q % a.n_inner;
      store_elem<R, ST>(a, b, o, i, e, L, src[l * L + e]);
    }
  }
}

template <typename R, int LOG2L, bool INV, int LD, int ST>
static hipError_t fft_launch(const FftArgs<R>& a, int nbatch, hipStream_t s) {
  constexpr int L = 1 << LOG2L;
  const int64_t nlines = a.n_outer * a.n_inner;
  const unsigned nblk = (unsigned)((nlines + a.lpw - 1) / a.lpw);
  const size_t lds = 2 * (size_t)a.lpw * L * sizeof(cplx<R>);
  hipLaunchKernelGGL((fft_pass_kernel<R, LOG2L, INV, LD, ST>), dim3(nblk, nbatch), dim3(256), lds,
                     s, a);
  return hipGetLastError();
}

template <typename R, int LOG2L>
static hipError_t fft_modes(const FftArgs<R>& a, bool inverse, LoadMode ld, StoreMode st,
                            int nbatch, hipStream_t s) {
  if (!inverse && ld == kLoadMerge && st == kStoreCropScaled)
    return fft_launch<R, LOG2L, false, kLoadMerge, kStoreCropScaled>(a, nbatch, s);
  if (!inverse && ld == kLoadStrided && st == kStoreCropScaled)
    return fft_launch<R, LOG2L, false, kLoadStrided, kStoreCropScaled>(a, nbatch, s);
  if (inverse && ld == kLoadPadScaled && st == kStoreFull)
    return fft_launch<R, LOG2L, true, kLoadPadScaled, kStoreFull>(a, nbatch, s);
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_fft_pass(const FftArgs<R>& a, int L, bool inverse, LoadMode ld, StoreMode st,
                           int nbatch, hipStream_t s) {
  switch (L) {
    case 8: return fft_modes<R, 3>(a, inverse, ld, st, nbatch, s);
    case 16: return fft_modes<R, 4>(a, inverse, ld, st, nbatch, s);
    case 32: return fft_modes<R, 5>(a, inverse, ld, st, nbatch, s);
    case 64: return fft_modes<R, 6>(a, inverse, ld, st, nbatch, s);
    case 128: return fft_modes<R, 7>(a, inverse, ld, st, nbatch, s);
    case 256: return fft_modes<R, 8>(a, inverse, ld, st, nbatch, s);
    case 512: return fft_modes<R, 9>(a, inverse, ld, st, nbatch, s);
    case 1024: return fft_modes<R, 10>(a, inverse, ld, st, nbatch, s);
    case 2048: return fft_modes<R, 11>(a, inverse, ld, st, nbatch, s);
    case 4096: return fft_modes<R, 12>(a, inverse, ld, st, nbatch, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_fft_pass<float>(const FftArgs<float>&, int, bool, LoadMode, StoreMode,
                                           int, hipStream_t);
template hipError_t launch_fft_pass<double>(const FftArgs<double>&, int, bool, LoadMode,
                                            StoreMode, int, hipStream_t);

}  // namespace nfft
