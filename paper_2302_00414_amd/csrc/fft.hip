// Batched 1-D FFT passes (step 2 of Algorithms 2.1 and 2.4), LDS-resident
// Stockham autosort with radix-8/4/2 butterflies.
//
// One launch transforms every line of one dimension of a d-dimensional
// array. A work-group holds `lpw` whole lines of length L in LDS: in two
// ping-pong buffers (passes of few work-groups), or in one buffer with each
// stage read into registers and written back in place, beside a copy of the
// pass's twiddle table (passes of many work-groups). Lines are read contiguously and the transformed axis
// is written as the new slowest axis, so after d passes the array is back in
// C order and every pass reads contiguous lines. Each pass is fused with its
// neighbours' elementwise work:
//   loaders : kLoadMerge      -- the first adjoint pass sums the tile
//                                 partials of the spreading step into grid
//                                 cells (fixed order, no atomics);
//             kLoadLine       -- plain contiguous read;
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

// LDS position of element i of a line: one pad slot per 8 elements breaks the
// power-of-two strides of the Stockham passes across the LDS banks.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 3); }

// One Stockham pass of radix RAD over `lpw` lines of length L, from buffer
// src to buffer dst (the latency layout: two buffers, no barrier inside).
template <typename R, int RAD, bool INV>
__device__ __forceinline__ void stockham_pass(const cplx<R>* src, cplx<R>* dst, int L, int LS,
                                              int lpw, int Ns, const cplx<R>* __restrict__ tw) {
  const int nbf = L / RAD;
  for (int q = threadIdx.x; q < lpw * nbf; q += blockDim.x) {
    const int line = q / nbf;
    const int j = q - line * nbf;
    const cplx<R>* s = src + line * LS;
    cplx<R>* o = dst + line * LS;
    cplx<R> a[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) a[r] = s[lpad(j + r * nbf)];
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
    for (int r = 0; r < RAD; ++r) o[lpad(idx + r * Ns)] = a[r];
  }
}


// The same pass in place (the throughput layout): every thread reads the
// butterflies it owns (NIT of them, RAD elements each) into registers, the
// work-group waits, then every thread writes its results; one buffer, so
// that the twiddle table fits beside the lines.
template <typename R, int RAD, int NIT, bool INV>
__device__ __forceinline__ void stockham_inplace(cplx<R>* buf, int L, int LS, int lpw, int Ns,
                                                 const cplx<R>* __restrict__ tw) {
  const int nbf = L / RAD;
  const int total = lpw * nbf;
  cplx<R> a[NIT][RAD];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int q = threadIdx.x + it * blockDim.x;
    if (q < total) {
      const int line = q / nbf;
      const int j = q - line * nbf;
      const cplx<R>* s = buf + line * LS;
#pragma unroll
      for (int r = 0; r < RAD; ++r) a[it][r] = s[lpad(j + r * nbf)];
      const int jm = j & (Ns - 1);
      if (Ns > 1) {
        const int step = jm * (L / (Ns * RAD));
#pragma unroll
        for (int r = 1; r < RAD; ++r) {
          cplx<R> w = tw[step * r];
          if (INV) w.y = -w.y;
          a[it][r] = cmul<R>(a[it][r], w);
        }
      }
      if constexpr (RAD == 8) dft8<R, INV>(a[it]);
      else if constexpr (RAD == 4) dft4<R, INV>(a[it][0], a[it][1], a[it][2], a[it][3]);
      else dft2<R, INV>(a[it]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int q = threadIdx.x + it * blockDim.x;
    if (q < total) {
      const int line = q / nbf;
      const int j = q - line * nbf;
      const int jm = j & (Ns - 1);
      cplx<R>* o = buf + line * LS;
      const int idx = (j - jm) * RAD + jm;
#pragma unroll
      for (int r = 0; r < RAD; ++r) o[lpad(idx + r * Ns)] = a[it][r];
    }
  }
}

// Sum of the tile partials that cover grid cell c: per dimension the own
// tile and, within m cells of its border, the neighbour tile whose padding
// reaches over (tiles wrap periodically). Tiles without nodes hold zeros.
template <typename R, int D>
__device__ __forceinline__ cplx<R> merge_cell(const cplx<R>* __restrict__ tilep, const Geom& g,
                                              const int* c) {
  // T and the tile count per dimension are powers of two: shifts and masks
  double sx = 0.0, sy = 0.0;
  const int tm = g.T - 1, nm = g.nb - 1, ts = g.tshift;
  int r[3], b0[3];
#pragma unroll
  for (int t = 0; t < D; ++t) {
    r[t] = c[t] & tm;
    b0[t] = c[t] >> ts;
  }
#pragma unroll
  for (int d0 = -1; d0 <= 1; ++d0) {
    const int p0 = r[0] + g.m - d0 * g.T;
    if (p0 < 0 || p0 >= g.P) continue;
    const int q0 = (b0[0] + d0) & nm;
#pragma unroll
    for (int d1 = (D > 1 ? -1 : 0); d1 <= (D > 1 ? 1 : 0); ++d1) {
      int p1 = 0, q1 = 0;
      if (D > 1) {
        p1 = r[1] + g.m - d1 * g.T;
        if (p1 < 0 || p1 >= g.P) continue;
        q1 = (b0[1] + d1) & nm;
      }
#pragma unroll
      for (int d2 = (D > 2 ? -1 : 0); d2 <= (D > 2 ? 1 : 0); ++d2) {
        int p2 = 0, q2 = 0;
        if (D > 2) {
          p2 = r[2] + g.m - d2 * g.T;
          if (p2 < 0 || p2 >= g.P) continue;
          q2 = (b0[2] + d2) & nm;
        }
        int bin = q0, pl = p0;
        if (D > 1) {
          bin = (bin << (g.Ms_shift - ts)) + q1;
          pl = pl * g.P + p1;
        }
        if (D > 2) {
          bin = (bin << (g.Ms_shift - ts)) + q2;
          pl = pl * g.P + p2;
        }
        const cplx<R> v = tilep[(int64_t)bin * g.Ptot + pl];
        sx += (double)v.x;
        sy += (double)v.y;
      }
    }
  }
  return mkc<R>((R)sx, (R)sy);
}

// Tiles at least 2m wide: a cell lies within m of at most one border per
// dimension, so at most two tiles cover it per dimension (its own and one
// neighbour). All 2^d candidate loads are issued without branches; a missing
// neighbour is replaced by the own tile with weight zero.
template <typename R, int D>
__device__ __forceinline__ cplx<R> merge_cell2(const cplx<R>* __restrict__ tilep, const Geom& g,
                                               const int* c) {
  const int tm = g.T - 1, nm = g.nb - 1, ts = g.tshift;
  int qb[3][2], pp[3][2];
  float wt[3];
#pragma unroll
  for (int t = 0; t < D; ++t) {
    const int r = c[t] & tm;
    const int b0 = c[t] >> ts;
    qb[t][0] = b0;
    pp[t][0] = r + g.m;
    const bool lo = r < g.m, hi = r >= g.T - g.m;
    qb[t][1] = lo ? ((b0 - 1) & nm) : (hi ? ((b0 + 1) & nm) : b0);
    pp[t][1] = lo ? r + g.m + g.T : (hi ? r + g.m - g.T : r + g.m);
    wt[t] = (lo || hi) ? 1.0f : 0.0f;
  }
  const int bs = g.Ms_shift - ts;
  cplx<R> v[1 << D];
  float w[1 << D];
#pragma unroll
  for (int s = 0; s < (1 << D); ++s) {
    int bin = 0, pl = 0;
    float ws = 1.0f;
#pragma unroll
    for (int t = 0; t < D; ++t) {
      const int o = (s >> (D - 1 - t)) & 1;
      bin = (bin << bs) + qb[t][o];
      pl = pl * g.P + pp[t][o];
      ws = o ? ws * wt[t] : ws;
    }
    v[s] = tilep[(int64_t)bin * g.Ptot + pl];
    w[s] = ws;
  }
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int s = 0; s < (1 << D); ++s) {
    sx += (double)w[s] * (double)v[s].x;
    sy += (double)w[s] * (double)v[s].y;
  }
  return mkc<R>((R)sx, (R)sy);
}

// The NV elements j + r TPL (r < NV, TPL = L / NV threads per line) of grid
// line q merged from the tile partials, d = 2 or 3, tiles at least 2m wide
// whose edge divides TPL: the line fixes the leading d - 1 coordinates, and
// the elements sit at the same offset within their tiles, so the candidate
// tiles, offsets and weights are worked out once for all of them. Same
// candidates, weights and summation order as merge_cell2, so the same values.
template <typename R, int D, int TPL, int NV>
__device__ __forceinline__ void merge_line(const FftArgs<R>& a, int b, int64_t q, int j,
                                           cplx<R> (&v)[NV]) {
  static_assert(D == 2 || D == 3, "lines of a 2-D or 3-D grid");
  constexpr int NH = 1 << (D - 1);  // candidates over the leading coordinates
  const Geom& g = a.g;
  const cplx<R>* __restrict__ tp = a.tilep + b * a.tile_bs;
  const int tm = g.T - 1, nm = g.nb - 1, ts = g.tshift, bs = g.Ms_shift - ts;
  int c[2];
  if constexpr (D == 2) {
    c[0] = (int)q;
  } else {
    c[0] = (int)(q >> g.Ms_shift);
    c[1] = (int)(q & (g.Ms - 1));
  }
  int qb[2][2], pp[2][2];
  float wt[2];
#pragma unroll
  for (int t = 0; t < D - 1; ++t) {
    const int r = c[t] & tm;
    const int b0 = c[t] >> ts;
    const bool lo = r < g.m, hi = r >= g.T - g.m;
    qb[t][0] = b0;
    qb[t][1] = lo ? ((b0 - 1) & nm) : (hi ? ((b0 + 1) & nm) : b0);
    pp[t][0] = r + g.m;
    pp[t][1] = lo ? r + g.m + g.T : (hi ? r + g.m - g.T : r + g.m);
    wt[t] = (lo || hi) ? 1.0f : 0.0f;
  }
  // leading part of candidate s = (o_0 .. o_{d-2}, o_last): tile row, cell
  // row offset and the running weight product
  int bh[NH], ph[NH];
  float wh[NH];
#pragma unroll
  for (int sh = 0; sh < NH; ++sh) {
    int bin = 0, pl = 0;
    float ws = 1.0f;
#pragma unroll
    for (int t = 0; t < D - 1; ++t) {
      const int o = (sh >> (D - 2 - t)) & 1;
      bin = (bin << bs) + qb[t][o];
      pl = pl * g.P + pp[t][o];
      ws = o ? ws * wt[t] : ws;
    }
    bh[sh] = bin << bs;
    ph[sh] = pl * g.P;
    wh[sh] = ws;
  }
  // last coordinate: offset within the tile shared by the eight elements
  const int r1 = j & tm;
  const bool lo1 = r1 < g.m, hi1 = r1 >= g.T - g.m;
  const int dq1 = lo1 ? -1 : (hi1 ? 1 : 0);
  const int pc = r1 + g.m;
  const int pd = lo1 ? r1 + g.m + g.T : (hi1 ? r1 + g.m - g.T : r1 + g.m);
  const float wt1 = (lo1 || hi1) ? 1.0f : 0.0f;
  double w[2 * NH];
#pragma unroll
  for (int sh = 0; sh < NH; ++sh) {
    w[2 * sh] = (double)wh[sh];
    w[2 * sh + 1] = (double)(wh[sh] * wt1);
  }
  const int Ptot = g.Ptot;
  const int tstep = TPL >> ts;  // tiles between consecutive elements
#pragma unroll
  for (int r = 0; r < NV; ++r) {
    const int t1 = (j >> ts) + r * tstep;  // element < M_sigma: no wrap
    const int t1n = (t1 + dq1) & nm;
    cplx<R> u[2 * NH];
#pragma unroll
    for (int sh = 0; sh < NH; ++sh) {
      u[2 * sh] = tp[(int64_t)(bh[sh] + t1) * Ptot + ph[sh] + pc];
      u[2 * sh + 1] = tp[(int64_t)(bh[sh] + t1n) * Ptot + ph[sh] + pd];
    }
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int s = 0; s < 2 * NH; ++s) {
      sx += w[s] * (double)u[s].x;
      sy += w[s] * (double)u[s].y;
    }
    v[r] = mkc<R>((R)sx, (R)sy);
  }
}

template <typename R, int LD>
__device__ __forceinline__ cplx<R> load_elem(const FftArgs<R>& a, int b, int64_t q, int e, int L) {
  if constexpr (LD == kLoadLine) {
    return a.in[b * a.in_bs + q * L + e];
  } else if constexpr (LD == kLoadPadScaled) {
    const int M = a.g.M;
    int kidx;
    if (e < M / 2)
      kidx = e + M / 2;
    else if (e >= L - M / 2)
      kidx = e - L + M / 2;
    else
      return mkc<R>(0, 0);
    const cplx<R> v = a.in[b * a.in_bs + q * M + kidx];
    const double f = a.fac[kidx];
    return mkc<R>((R)((double)v.x * f), (R)((double)v.y * f));
  } else {
    // merge: the line index enumerates the leading d-1 grid coordinates
    const cplx<R>* tp = a.tilep + b * a.tile_bs;
    const int d = a.g.d;
    const bool two = a.g.T >= 2 * a.g.m;
    if (d == 1) {
      const int c[1] = {e};
      return two ? merge_cell2<R, 1>(tp, a.g, c) : merge_cell<R, 1>(tp, a.g, c);
    }
    if (d == 2) {
      const int c[2] = {(int)q, e};
      return two ? merge_cell2<R, 2>(tp, a.g, c) : merge_cell<R, 2>(tp, a.g, c);
    }
    const int c[3] = {(int)(q >> a.g.Ms_shift), (int)(q & (a.g.Ms - 1)), e};
    return two ? merge_cell2<R, 3>(tp, a.g, c) : merge_cell<R, 3>(tp, a.g, c);
  }
}

template <typename R, int ST>
__device__ __forceinline__ void store_elem(const FftArgs<R>& a, int b, int64_t q, int e, int L,
                                           cplx<R> v) {
  if constexpr (ST == kStoreFull) {
    a.out[b * a.out_bs + (int64_t)e * a.nlines + q] = v;
  } else {
    const int M = a.g.M;
    int kidx;
    if (e < M / 2)
      kidx = e + M / 2;
    else if (e >= L - M / 2)
      kidx = e - L + M / 2;
    else
      return;
    cplx<R>* o = a.out + b * a.out_bs + (int64_t)kidx * a.nlines + q;
    // the factor is float64; the product is rounded once to the precision
    // of the data
    const double f = a.fac[kidx];
    const double ux = (double)v.x * f, uy = (double)v.y * f;
    if (a.accumulate) {
      const cplx<R> c = *o;
      *o = mkc<R>((R)((double)c.x + ux), (R)((double)c.y + uy));
    } else {
      *o = mkc<R>((R)ux, (R)uy);
    }
  }
}

// Lines of a pass are dealt to work-groups so that consecutive lines land on
// one XCD: work-groups are dispatched to the 8 XCDs in turn, so work-group
// i runs on XCD i mod 8, and line block (i mod 8) * (n / 8) + i / 8 gives
// each XCD a contiguous range of lines. The lines one XCD reads and the
// output elements it writes (the transformed axis becomes the slowest, so
// consecutive lines are consecutive outputs) then share that XCD's L2
// instead of being split into partial cache lines between XCDs.
// work-groups of a pass from which on its stages read the twiddles from an
// LDS copy of the table (a pass of fewer work-groups is latency bound and
// would wait on the copy; measured on 512-point passes)
constexpr int64_t kFftTwiddleLdsGroups = 2048;

__device__ __forceinline__ int64_t xcd_block(unsigned bx, unsigned nblk) {
  if (nblk < 16 || (nblk & 7) != 0) return bx;
  return (int64_t)(bx & 7) * (nblk >> 3) + (bx >> 3);
}

// First stage: radix R0 on elements loaded straight into registers (Ns = 1,
// no twiddles); thread j of a line takes elements j + r L/R0. R0 = 8 (L/8
// threads per line) is the default; 4 and 2 give a line more threads where a
// pass has few lines.
template <typename R, int LOG2L, bool INV, int LD, int ST, int R0, bool TWL>
__global__ __launch_bounds__(512) void fft_pass_kernel(FftArgs<R> a) {
  constexpr int L = 1 << LOG2L;
  constexpr int TPL = L / R0;  // threads per line (one radix-R0 butterfly each)
  constexpr int LS = L + L / 8 + 1;  // LDS line stride: padded line plus one slot
  extern __shared__ unsigned char smem_raw[];
  const int lpw = a.lpw;      // blockDim.x == lpw * TPL
  cplx<R>* buf0 = reinterpret_cast<cplx<R>*>(smem_raw);
  // TWL (passes with many work-groups, throughput bound): one line buffer
  // with the stages in place and the twiddle table copied to LDS behind it,
  // where every butterfly of the later stages reads it. Otherwise (latency
  // bound): two line buffers, no barrier inside a stage, twiddles read from
  // device memory.
  cplx<R>* buf1 = buf0 + lpw * LS;
  cplx<R>* twl = buf1;
  if constexpr (TWL)
    for (int i = threadIdx.x; i < L; i += blockDim.x) twl[i] = a.tw[i];
  const int64_t nlines = a.nlines;
  const int64_t q0 = xcd_block(blockIdx.x, gridDim.x) * lpw;
  const int b = blockIdx.y;

  {
    const int l = threadIdx.x / TPL;
    const int j = threadIdx.x - l * TPL;
    const int64_t q = q0 + l;
    cplx<R> v[R0];
    bool per_line = false;
    if constexpr (LD == kLoadMerge)
      per_line = a.g.d >= 2 && a.g.T >= 2 * a.g.m && (TPL & (a.g.T - 1)) == 0;
    if constexpr (LD == kLoadMerge) {
      if (q < nlines && per_line) {
        if (a.g.d == 2)
          merge_line<R, 2, TPL, R0>(a, b, q, j, v);
        else
          merge_line<R, 3, TPL, R0>(a, b, q, j, v);
      } else if (q < nlines) {
#pragma unroll
        for (int r = 0; r < R0; ++r) v[r] = load_elem<R, LD>(a, b, q, j + r * TPL, L);
      } else {
#pragma unroll
        for (int r = 0; r < R0; ++r) v[r] = mkc<R>(0, 0);
      }
    } else {
      if (q < nlines) {
#pragma unroll
        for (int r = 0; r < R0; ++r) v[r] = load_elem<R, LD>(a, b, q, j + r * TPL, L);
      } else {
#pragma unroll
        for (int r = 0; r < R0; ++r) v[r] = mkc<R>(0, 0);
      }
    }
    if constexpr (R0 == 8) {
      dft8<R, INV>(v);
    } else if constexpr (R0 == 4) {
      dft4<R, INV>(v[0], v[1], v[2], v[3]);
    } else {
      dft2<R, INV>(v);
    }
    cplx<R>* o = buf0 + l * LS;
#pragma unroll
    for (int r = 0; r < R0; ++r) o[lpad(j * R0 + r)] = v[r];
  }
  __syncthreads();

  cplx<R>* src = buf0;
  int Ns = R0;
  constexpr int LOG2R0 = R0 == 8 ? 3 : (R0 == 4 ? 2 : 1);
  constexpr int n8 = (LOG2L - LOG2R0) / 3;
  constexpr int rem = (LOG2L - LOG2R0) % 3;
  if constexpr (TWL) {
#pragma unroll 1
    for (int p = 0; p < n8; ++p) {
      stockham_inplace<R, 8, 1, INV>(src, L, LS, lpw, Ns, twl);
      __syncthreads();
      Ns *= 8;
    }
    if constexpr (rem == 2) {
      stockham_inplace<R, 4, (R0 / 4 > 1 ? R0 / 4 : 1), INV>(src, L, LS, lpw, Ns, twl);
      __syncthreads();
    } else if constexpr (rem == 1) {
      stockham_inplace<R, 2, R0 / 2, INV>(src, L, LS, lpw, Ns, twl);
      __syncthreads();
    }
  } else {
    cplx<R>* dst = buf1;
#pragma unroll 1
    for (int p = 0; p < n8; ++p) {
      stockham_pass<R, 8, INV>(src, dst, L, LS, lpw, Ns, a.tw);
      __syncthreads();
      cplx<R>* t = src;
      src = dst;
      dst = t;
      Ns *= 8;
    }
    if constexpr (rem == 2) {
      stockham_pass<R, 4, INV>(src, dst, L, LS, lpw, Ns, a.tw);
      __syncthreads();
      src = dst;
    } else if constexpr (rem == 1) {
      stockham_pass<R, 2, INV>(src, dst, L, LS, lpw, Ns, a.tw);
      __syncthreads();
      src = dst;
    }
  }

  // store: consecutive threads walk across lines (the output axis is rotated)
  for (int idx = threadIdx.x; idx < lpw * L; idx += blockDim.x) {
    const int l = idx % lpw;
    const int e = idx / lpw;
    const int64_t q = q0 + l;
    if (q < nlines) store_elem<R, ST>(a, b, q, e, L, src[l * LS + lpad(e)]);
  }
}

template <typename R, int LOG2L, bool INV, int LD, int ST, int R0>
static hipError_t fft_launch_r0(const FftArgs<R>& a, int nbatch, hipStream_t s) {
  constexpr int L = 1 << LOG2L;
  const unsigned nblk = (unsigned)((a.nlines + a.lpw - 1) / a.lpw);
  const int threads = a.lpw * (L / R0);
  if (threads > 512) return hipErrorInvalidConfiguration;
  // throughput layout (one line buffer and the twiddle table) for passes of
  // many work-groups, latency layout (two line buffers) for the others
  const size_t lines_lds = (size_t)a.lpw * (L + L / 8 + 1) * sizeof(cplx<R>);
  if ((int64_t)nblk * nbatch >= kFftTwiddleLdsGroups)
    hipLaunchKernelGGL((fft_pass_kernel<R, LOG2L, INV, LD, ST, R0, true>), dim3(nblk, nbatch),
                       dim3(threads), lines_lds + L * sizeof(cplx<R>), s, a);
  else
    hipLaunchKernelGGL((fft_pass_kernel<R, LOG2L, INV, LD, ST, R0, false>), dim3(nblk, nbatch),
                       dim3(threads), 2 * lines_lds, s, a);
  return hipGetLastError();
}

// A pass whose lines already go one per work-group and still give few
// work-groups gets two or four times the threads per line (a.r0: first stage
// radix 4 or 2; the merge loader then takes 4 or 2 elements a thread).
template <typename R, int LOG2L, bool INV, int LD, int ST>
static hipError_t fft_launch(const FftArgs<R>& a, int nbatch, hipStream_t s) {
  constexpr int L = 1 << LOG2L;
  // L / R0 threads per line, at most 512 (the launch bound)
  if constexpr (L >= 64 && L <= 1024) {
    if (a.r0 == 2) return fft_launch_r0<R, LOG2L, INV, LD, ST, 2>(a, nbatch, s);
  }
  if constexpr (L >= 64 && L <= 2048) {
    if (a.r0 == 4) return fft_launch_r0<R, LOG2L, INV, LD, ST, 4>(a, nbatch, s);
  }
  return fft_launch_r0<R, LOG2L, INV, LD, ST, 8>(a, nbatch, s);
}

template <typename R, int LOG2L>
static hipError_t fft_modes(const FftArgs<R>& a, bool inverse, LoadMode ld, StoreMode st,
                            int nbatch, hipStream_t s) {
  if (!inverse && ld == kLoadMerge && st == kStoreCropScaled)
    return fft_launch<R, LOG2L, false, kLoadMerge, kStoreCropScaled>(a, nbatch, s);
  if (!inverse && ld == kLoadLine && st == kStoreCropScaled)
    return fft_launch<R, LOG2L, false, kLoadLine, kStoreCropScaled>(a, nbatch, s);
  if (inverse && ld == kLoadPadScaled && st == kStoreFull)
    return fft_launch<R, LOG2L, true, kLoadPadScaled, kStoreFull>(a, nbatch, s);
  return hipErrorInvalidValue;
}

// Work-group shape of a pass over nlines lines of nbatch batches. Lines per
// work-group are bounded by 32 KiB of LDS per line buffer and by 256
// threads (L/8 butterflies per line; 512 measured slower) and lowered while
// that leaves fewer than min_wg work-groups. A pass whose lines go one per work-group
// and still give few work-groups gets two or four times the threads per line
// (first stage radix 4 or 2, also for the merge loader). The radix is decided
// from one batch's lines, so a batched call computes exactly what separate
// calls compute; only the lines per work-group count all batches (a batched
// radix-4 pass may take several lines per work-group, up to 512 threads).
template <typename R>
static int fft_lines_per_wg(int L, int64_t lines, int min_wg) {
  const int lds_cap = max(1, 32768 / ((L + L / 8 + 1) * (int)sizeof(cplx<R>)));
  int lpw = max(1, min(lds_cap, 2048 / L));
  while (lpw > 1 && lines / lpw < min_wg) lpw /= 2;
  return lpw;
}

template <typename R>
static void fft_shape(FftArgs<R>& a, int L, int nbatch) {
  const int lpw1 = fft_lines_per_wg<R>(L, a.nlines, a.min_wg);
  a.r0 = 8;
  if (lpw1 == 1 && 2 * a.nlines <= a.min_wg)
    a.r0 = 2;
  else if (lpw1 == 1 && a.nlines < 2 * (int64_t)a.min_wg)
    a.r0 = 4;
  while (a.r0 < 8 && L / a.r0 > 512) a.r0 *= 2;  // at most 512 threads per work-group
  // lines per work-group from all batches' lines, at most 512 threads
  a.lpw = min(fft_lines_per_wg<R>(L, a.nlines * (int64_t)nbatch, a.min_wg), 512 / (L / a.r0));
}

template <typename R>
hipError_t launch_fft_pass(const FftArgs<R>& args, int L, bool inverse, LoadMode ld, StoreMode st,
                           int nbatch, hipStream_t s) {
  FftArgs<R> a = args;
  fft_shape(a, L, nbatch);
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
