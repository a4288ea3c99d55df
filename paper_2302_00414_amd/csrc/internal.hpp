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
// Stable in-tile sort of the tile-ordered node arrays by tile row (the
// tile-local cell of dimension 0); results in perm2 / loc2 / frac2.
template <typename R>
hipError_t launch_row_sort(const int32_t* bstart, int nbins, int T, int64_t N, int d,
                           const int32_t* perm, const uint32_t* loc, const R* frac, int32_t* perm2,
                           uint32_t* loc2, R* frac2, hipStream_t s);
template <typename R>
hipError_t launch_permute_weights(const double* w, const int32_t* perm, int64_t N,
                                  cplx<R>* w_sorted, hipStream_t s);

// Zero the tile slots of the nbins tiles listed in bins (tiles without nodes).
template <typename R>
hipError_t launch_zero_tiles(cplx<R>* tilep, int64_t tile_rs, const int32_t* bins, int nbins,
                             int Ptot, int nrhs, hipStream_t s);

// ------------------------------------------------------- spreading / sums
// Tile partials: every tile owns a padded-tile slot in `tilep` ([rhs][tile]
// [P^d], zero for tiles without nodes). A tile with a single work item is
// spread straight into its slot; the items of a tile split into several work
// items write to their own slots in `itemp` and tile_reduce sums them.
template <typename R>
struct SpreadArgs {
  const uint32_t* loc;       // packed tile-local cells, tile order
  const R* frac;             // d planes of N offsets in [0, 1), tile order
  const cplx<R>* w;          // weights in tile order
  const int32_t* perm;       // tile order -> caller index
  const cplx<R>* f;          // samples, caller order, rhs stride f_rs
  cplx<R>* tilep;            // tile partials [rhs][tile][P^d]
  cplx<R>* itemp;            // item partials of split tiles [rhs][slot][P^d]
  const int32_t* item_start; // first node of each work item
  const int32_t* item_count; // nodes of each work item
  const int32_t* item_bin;   // tile of each work item
  const int32_t* item_slot;  // slot in itemp, or -1 for the only item of a tile
  const R* coef;             // window polynomials [2m][deg + 1]
  int64_t f_rs, tile_rs, item_rs;
  R edge;                    // window value at the closed edge |t| = m
  Geom g;
  int nt;                    // threads per work-group, d <= 2 float32 single-rhs kernel
  int nr;                    // right-hand sides per work-group (1, 2, 4 or 8; d <= 2)
  int planes;                // 2: float32 real and imaginary planes in separate groups
  int mode;                  // d = 2 single rhs: 1 LDS tiles, 2 register row sweep,
                             // 3 LDS tiles with precomputed window factors,
                             // 4 LDS tiles with the window evaluated late,
                             // 5 padded tile in registers (float32),
                             // 6 grid tiles gathered for 32 rhs per work-group
                             //   (float32; see launch_spread_gather),
                             // 7 padded tile on the matrix cores (d = 2, 3;
                             //   float32 and float64)
  const R* psi;              // d = 2: window factors [N][2m][2] in tile order (mode 3)
};
template <typename R>
hipError_t launch_spread(const SpreadArgs<R>& a, int nrhs, hipStream_t s);
// Spreading by output tiles for 32 right-hand sides per work-group (d = 2,
// float32, tile edge 16, m <= 8) into the grid [rhs][Ms^2]. Per tile the plan
// lists the nodes whose window reaches it (gl_node: node in tile order,
// gl_hdr: footprint origin relative to the tile + 64 in bits 0-7 (rows) and
// 8-15 (columns), closed-edge flags in bits 16, 17); a unit (tile, first
// entry, end, slot) spreads a run of one tile's list into the grid (slot -1)
// or into a partial slot [rhs][slot][256] that the reduction sums.
struct GatherArgs {
  const int32_t* units;   // [nunits][4]: tile (-1: padding), begin, end, slot
  int nunits;
  const int32_t* gl_node;
  const int32_t* gl_hdr;
  const int32_t* split;   // [nsplit][4]: tile, first slot, slots, 0
  int nsplit;
  float2* grid;
  int64_t grid_rs;
  float2* part;
  int64_t part_rs;
  // node-major weighted samples c = w f, [ceil(nrhs/32)][N][16] float4, node j's
  // float4 q = (Re c_q, Re c_16+q, Im c_q, Im c_16+q) of its group's 32
  // right-hand sides (written first)
  float2* fT;
  const int32_t* iperm;   // caller index -> tile order (for the weights)
};
bool spread_gather_supported(int d, int T, bool f64, int m);
size_t spread_gather_lds_bytes(int m);
hipError_t launch_spread_gather(const SpreadArgs<float>& a, const GatherArgs& ga, int nrhs,
                                hipStream_t s);
hipError_t launch_gather_reduce(const GatherArgs& ga, int nb, int Ms, int nrhs, hipStream_t s);
// Register row sweep (d = 2, padded tile edge <= 32, nodes row-sorted in tiles).
bool spread_rows_supported(int d, int P);
template <typename R>
hipError_t launch_spread_rows(const SpreadArgs<R>& a, int nrhs, hipStream_t s);
// Group kernel reading the precomputed window factors (d = 2, a.psi set).
template <typename R>
hipError_t launch_spread_pre(const SpreadArgs<R>& a, int nrhs, hipStream_t s);
// Group kernel evaluating the window late from offsets in device memory (d = 2).
template <typename R>
hipError_t launch_spread_late(const SpreadArgs<R>& a, int nrhs, hipStream_t s);
// Window factors of every node (tile order), [N][2m][2], from the same
// per-cell polynomials the spreading kernels evaluate (d = 2).
template <typename R>
hipError_t launch_psi(const R* frac, int64_t N, int m, const R* coef, R* psi, hipStream_t s);
// Register-tile spreading (float32, d = 2, tile edge 16, nodes row-sorted
// within tiles).
bool spread_reg_supported(int d, int T, bool f64);
size_t spread_reg_lds_bytes(int m);
hipError_t launch_spread_reg(const SpreadArgs<float>& a, int nrhs, hipStream_t s);
// Padded tile on the matrix cores, one tile row of nodes at a time (float32
// or float64, d = 2, tile edge 16, 2m + 1 <= 16, nodes row-sorted within
// tiles).
bool spread_mma_supported(int d, int T, bool f64, int m);
size_t spread_mma_lds_bytes(int m, int nt, bool f64);
template <typename R>
hipError_t launch_spread_mma(const SpreadArgs<R>& a, int nrhs, hipStream_t s);
// The d = 3 form of mode 7: one wave holds the padded tile (tile edge 8,
// 2m <= 8, nodes sorted by their dimension-0 cell within tiles) in
// matrix-core accumulators, float32 or float64.
bool spread3_mma_supported(int d, int T, bool f64, int m);
size_t spread3_mma_lds_bytes(bool f64);
template <typename R>
hipError_t launch_spread3_mma(const SpreadArgs<R>& a, int nrhs, hipStream_t s);
// Several right-hand sides per work-group (d <= 2, nr > 1).
template <typename R>
hipError_t launch_spread_multi(const SpreadArgs<R>& a, int nrhs, hipStream_t s);
// LDS bytes one spreading work-group needs for these launch parameters, or 0
// if the combination is not built.
size_t spread_lds_bytes(int d, bool f64, int m, int T, int Ptot, int nt, int nr, int planes);

// Sum the item partials of every split tile into its tile slot, in item order
// (deterministic; compensated summation).
template <typename R>
struct ReduceArgs {
  cplx<R>* tilep;
  const cplx<R>* itemp;
  const int32_t* multi_bin;    // split tiles
  const int32_t* multi_first;  // first itemp slot of each split tile (nmulti + 1)
  int nmulti;
  int64_t tile_rs, item_rs;
  Geom g;
};
template <typename R>
hipError_t launch_tile_reduce(const ReduceArgs<R>& a, int nrhs, hipStream_t s);

template <typename R>
struct InterpArgs {
  const uint32_t* loc;
  const R* frac;
  const int32_t* perm;
  const cplx<R>* grid;       // full oversampled grid, C order, rhs stride grid_rs
  cplx<R>* f;                // output samples, caller order, rhs stride f_rs
  const cplx<R>* sub;        // if set: f = sub - (window sums), sub in caller order, stride f_rs
  const int32_t* item_start;
  const int32_t* item_count;
  const int32_t* item_bin;
  const R* coef;
  const R* psi;              // d = 2: window factor table [N][2m][2] in tile order, or null
  int64_t grid_rs;
  int64_t f_rs;
  R edge;
  Geom g;
};
template <typename R>
hipError_t launch_interp(const InterpArgs<R>& a, int nrhs, hipStream_t s);

// ------------------------------------------------------------------- FFT
enum LoadMode { kLoadMerge = 0, kLoadLine = 1, kLoadPadScaled = 2 };
enum StoreMode { kStoreCropScaled = 0, kStoreFull = 1 };

// Every pass reads whole lines that are contiguous in memory (line q at
// in + q * Lin) and writes its transformed axis as the new slowest axis
// (element k of line q at out + k * nlines + q). After d passes the axes are
// back in C order.
template <typename R>
struct FftArgs {
  int64_t nlines;
  const cplx<R>* in;   // strided / padded loads
  int64_t in_bs;       // batch stride (elements)
  int Lin;             // input line length (M_sigma, or M for padded loads)
  cplx<R>* out;
  int64_t out_bs;
  // merge loader: tile partials [rhs][tile][P^d]
  const cplx<R>* tilep;
  int64_t tile_bs;
  const cplx<R>* tw;   // twiddles e^{-2 pi i q / L}, q < L
  const double* fac;   // deconvolution factors over I_M (compressed index), float64
  int accumulate;      // kStoreCropScaled: add to the output instead of writing it
  int min_wg;          // the launch keeps at least this many work-groups where it can
  int lpw;             // lines per work-group (set by launch_fft_pass)
  int r0;              // radix of the first stage (8, 4 or 2: L/r0 threads per line;
                       // set by launch_fft_pass)
  Geom g;
};
template <typename R>
hipError_t launch_fft_pass(const FftArgs<R>& a, int L, bool inverse, LoadMode ld, StoreMode st,
                           int nbatch, hipStream_t s);

// ------------------------------------------------ optimized sparse matrix
// op 0: nodes per grid column; op 1: node ids into the column lists
hipError_t launch_bopt_pattern(const double* nodes, int64_t N, int d, int Ms, int m, int op,
                               int* count, const int64_t* col_ptr, int* fill, int32_t* col_node,
                               hipStream_t s);
// LDS of one column solve for up to nmax nodes with the Gram triangle and the
// per-node arrays in LDS
size_t bopt_solve_lds(int nmax);
// doubles of the device-memory workspace of a column of n nodes
int64_t bopt_workspace_doubles(int n);
// Column solves. ws null: columns 0..ncols-1 (or the ncols listed in cols)
// with everything in LDS, columns of more than nmax nodes skipped; ws set:
// the ncols columns listed in cols, the i-th with its workspace at
// ws + ws_off[i] (device memory), factorised by panels.
template <typename R>
hipError_t launch_bopt_solve(const double* nodes, int d, int M, int Ms, const double* wh,
                             const int64_t* col_ptr, int32_t* col_node, R* col_val, int64_t ncols,
                             int nmax, double piv_rel, double ridge, int* dropped,
                             const int64_t* cols, double* ws, const int64_t* ws_off,
                             hipStream_t s);
template <typename R>
hipError_t launch_bopt_apply(const int64_t* col_ptr, const int32_t* col_node, const R* col_val,
                             const cplx<R>* f, int64_t f_rs, cplx<R>* grid, int64_t g_rs,
                             int64_t ncols, int nrhs, double scale, int lanes, hipStream_t s);
// lanes per column of the apply (4..64) for columns of mean length avg
int bopt_apply_lanes(double avg);

hipError_t launch_bopt_lo(const double* nodes, int64_t N, int d, int Ms, int m, int32_t* lo,
                          hipStream_t s);
template <typename R>
hipError_t launch_bopt_rows(const int64_t* col_ptr, const int32_t* col_node, const R* col_val,
                            int64_t ncols, int d, int Ms, int m, const int32_t* lo, R* rows,
                            hipStream_t s);
template <typename R>
hipError_t launch_bopt_gather(const int32_t* lo, const R* rows, const cplx<R>* grid, int64_t g_rs,
                              int64_t N, int d, int Ms, int m, cplx<R>* f, int64_t f_rs, int nrhs,
                              double scale, hipStream_t s);

// ------------------------------------------------ float64 vector kernels
size_t reduce_scratch_doubles();
hipError_t launch_fill(cplx<double>* v, int64_t n, double re, double im, hipStream_t s);
hipError_t launch_conj(cplx<double>* v, int64_t n, hipStream_t s);
hipError_t launch_pcf(const double* x, int64_t N, int d, int M, cplx<double>* w, hipStream_t s);
hipError_t launch_reduce(const cplx<double>* a, const cplx<double>* b, int64_t n, int op,
                         int64_t e_idx, double* scratch, hipStream_t s);
hipError_t launch_cg_update(cplx<double>* x, cplx<double>* r, const cplx<double>* p,
                            const cplx<double>* q, int64_t n, double alpha, hipStream_t s);
hipError_t launch_cg_direction(cplx<double>* p, const cplx<double>* r, int64_t n, double beta,
                               hipStream_t s);

// ------------------------------------------------ weighted iterative refinement
// partial sums of the norm reductions: at most kRefineBlocks doubles
constexpr int kRefineBlocks = 512;
// *out = ||a||_2^2
template <typename R>
hipError_t launch_sumsq(const cplx<R>* a, int64_t n, double* partial, double* out, hipStream_t s);

}  // namespace nfft
