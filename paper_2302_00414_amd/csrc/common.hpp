// Shared device-side types and helpers of the MI355X NFFT library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nfft {

template <typename R> struct cplx_sel;
template <> struct cplx_sel<float> { using type = float2; };
template <> struct cplx_sel<double> { using type = double2; };
template <typename R> using cplx = typename cplx_sel<R>::type;

template <typename R>
__device__ __forceinline__ cplx<R> mkc(R re, R im) {
  cplx<R> c;
  c.x = re;
  c.y = im;
  return c;
}
template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return mkc<R>(a.x + b.x, a.y + b.y); }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return mkc<R>(a.x - b.x, a.y - b.y); }
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return mkc<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R>
__device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) { return mkc<R>(a.x * s, a.y * s); }

// Packed per-node cell record: bits 8t..8t+7 hold the node's floor cell
// relative to its tile origin in dimension t; bit 24+t flags a node that
// sits exactly on a grid line in dimension t (offset zero), for which the
// closed window support contains one more cell.
constexpr int kLocBits = 8;
constexpr uint32_t kLocMask = 0xffu;
constexpr int kEdgeShift = 24;

// Geometry of the tile decomposition of the oversampled grid, passed by value
// to kernels.
struct Geom {
  int d;        // dimension
  int Ms;       // oversampled grid edge
  int M;        // bandwidth
  int m;        // window truncation
  int T;        // tile edge in cells (divides Ms, >= m)
  int nb;       // tiles per dimension, Ms / T
  int P;        // padded tile edge, T + 2m
  int Ptot;     // P^d
  int nbins;    // nb^d
  int nsub;     // number of spreading work items (tile chunks)
  int tshift;   // log2(T)
  int Ms_shift; // log2(Ms)
  int64_t N;    // nodes
};

}  // namespace nfft
