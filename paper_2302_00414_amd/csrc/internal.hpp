// Internal launcher interface between the host plan code and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace nfft {

// ---------------------------------------------------------------- plan time
// Wrap nodes, split M_sigma x + M_sigma/2 into floor cell and offset, assign
// tiles. Outputs in caller order. err receives 1 if a node is not finite.
hipError_t launch_encode(const double* nodes, int64_t N, const Geom& g, int32_t* bin,
                         uint32_t* loc, double* frac, int* err, hipStream_t s);
hipError_t launch_count(const int32_t* bin, int64_t N, int32_t* counts, hipStream_t s);
// Stable within-tile ranks by chunks of kRankChunk nodes.
constexpr int kRankChunk = 1024;
hipError_t launch_rank(const int32_t* bin, int64_t N, int nbins, int32_t* rank,
                       int32_t* chunk_count, hipStream_t s);
hipError_t launch_chunk_offsets(const int32_t* chunk_count, const int32_t* bin_start,
                                int64_t nchunks, int nbins, int32_t* offsets, hipStream_t s);
template <typename R>
hipError_t launch_scatter(const int32_t* bin, const int32_t* rank, const int32_t* offsets,
                          const uint32_t* loc_u, const double* frac_u, int64_t N, int d,
                          int nbins, int32_t* perm, uint32_t* loc, R* frac, hipStream_t s);
template <typename R>
hipError_t launch_permute_weights(const double* w, const int32_t* perm, int64_t N,
                                  cplx<R>* w_sorted, hipStream_t s);

// ------------------------------------------------------- spreading / sums
template <typename R>
struct SpreadArgs {
  const uint32_t* loc;       // packed tile-local cells, tile order
  const R* frac;             // d planes of N offsets in [0, 1), tile order
  const cplx<R>* w;          // weights in tile order
  const int32_t* perm;       // tile order -> caller index
  const cplx<R>* f;          // samples, caller order, rhs stride f_rs
  cplx<R>* sub;              // padded tile sums [rhs][item][P^d]
  const int32_t* item_start; // first node of each work item
  const int32_t* item_count; // nodes of each work item
  int64_t f_rs;
  int64_t sub_rs;
  R b, mr, edge;
  Geom g;
};
template <typename R>
hipError_t launch_spread(const SpreadArgs<R>& a, int nrhs, hipStream_t s);

template <typename R>
struct InterpArgs {
  const uint32_t* loc;
  const R* frac;
  const int32_t* perm;
  const cplx<R>* grid;       // full oversampled grid, C order, rhs stride grid_rs
  cplx<R>* f;                // output samples, caller order, rhs stride f_rs
  const int32_t* item_start;
  const int32_t* item_count;
  const int32_t* item_bin;
  int64_t grid_rs;
  int64_t f_rs;
  R b, mr, edge;
  Geom g;
};
template <typename R>
hipError_t launch_interp(const InterpArgs<R>& a, int nrhs, hipStream_t s);

// ------------------------------------------------------------------- FFT
enum LoadMode { kLoadMerge = 0, kLoadStrided = 1, kLoadPadScaled = 2 };
enum StoreMode { kStoreCropScaled = 0, kStoreFull = 1 };

template <typename R>
struct FftArgs {
  // lines: q in [0, n_outer * n_inner), q = o * n_inner + i
  int64_t n_outer, n_inner;
  // input addressing (strided / padded loads)
  const cplx<R>* in;
  int64_t in_bs, in_os, in_is, in_es;
  // output addressing
  cplx<R>* out;
  int64_t out_bs, out_os, out_is, out_es;
  // merge loader: padded tile sums and tile -> first work item table
  const cplx<R>* sub;
  int64_t sub_bs;
  const int32_t* item_first;
  // twiddles e^{-2 pi i q / L}, q < L
  const cplx<R>* tw;
  // deconvolution factors over I_M (compressed index), length M
  const R* fac;
  int lpw;          // lines per work-group
  int inner_major;  // 1: consecutive threads walk lines (strided passes)
  Geom g;
};
template <typename R>
hipError_t launch_fft_pass(const FftArgs<R>& a, int L, bool inverse, LoadMode ld, StoreMode st,
                           int nbatch, hipStream_t s);

}  // namespace nfft
