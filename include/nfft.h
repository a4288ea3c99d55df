/*
 * nfft.h -- C ABI of the MI355X (gfx950) weighted adjoint NFFT library.
 *
 * Operations (Kircheis & Potts, arXiv 2302.00414):
 *
 *   adjoint : fhat ~ D^* F^* B^* W f                (eq. (3.7), Algorithm 3.7 step 1,
 *                                                     evaluated by Algorithm 2.4)
 *   forward : f    ~ B F D fhat                     (Algorithm 2.1, A ~ B F D)
 *
 * with the nonequispaced Fourier matrix A of eq. (2.7), W = diag(w) the
 * density-compensation weights of eq. (3.6), D (2.13), F (2.14) and B (2.15).
 * The window is the Kaiser-Bessel pair with shape b = pi (2 - 1/sigma),
 * truncated to the closed cube |M_sigma x_t - l_t| <= m (index set (2.12)).
 *
 * Conventions shared by every entry point
 *   - d in {1, 2, 3}; M even; I_M = {-M/2, ..., M/2-1}^d; M_sigma =
 *     2 ceil(ceil(sigma M) / 2) as in the definition before (2.9).
 *   - Nodes: N x d float64, row-major (node j at nodes[j*d .. j*d+d-1]), any
 *     real coordinates; they are wrapped onto the torus [-1/2, 1/2)^d
 *     (A is 1-periodic).
 *   - Coefficient vectors fhat: M^d complex values in C order of k in I_M
 *     (k_1 slowest, each k_t running from -M/2 to M/2-1).
 *   - Sample vectors f: N complex values in the caller's node order.
 *   - Complex numbers are interleaved (re, im): complex128 for an NFFT_F64
 *     plan, complex64 for an NFFT_F32 plan. With nrhs right-hand sides the
 *     vectors are stacked, right-hand side r at offset r*N (resp. r*M^d).
 *   - Pointers passed to nfft_plan / nfft_set_weights may be host or device
 *     memory; they are copied before the call returns and the caller keeps
 *     ownership. Pointers passed to nfft_adjoint / nfft_forward must be
 *     device memory of the plan's device; the work is enqueued on `stream`
 *     (a hipStream_t, NULL = default stream) and the call returns without
 *     waiting. The buffers must stay valid until the stream reaches that
 *     point. Outputs are overwritten, never accumulated.
 *   - Every entry point returns a status code (nfft_status); nothing is thrown
 *     across the ABI. Arguments are validated before anything is enqueued; on
 *     a validation failure the outputs are left untouched and a detail string
 *     is available from nfft_last_error(plan) (or nfft_last_error(NULL) when
 *     no plan exists). A device failure after enqueueing is reported by the
 *     next call on the plan.
 *   - A plan owns device workspace that each transform reuses: transforms of
 *     one plan must not run concurrently on different streams.
 */
#ifndef NFFT_MI355X_H
#define NFFT_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nfft_plan_s *nfft_plan_t;

enum nfft_status {
  NFFT_OK = 0,
  NFFT_EINVAL = 1,       /* invalid argument (shape, range, non-finite node, null pointer) */
  NFFT_ENOMEM = 2,       /* device allocation failed */
  NFFT_EDEVICE = 3,      /* HIP runtime or kernel failure */
  NFFT_ESTATE = 4,       /* call not allowed in the plan's state (e.g. adjoint before weights) */
  NFFT_EUNSUPPORTED = 5  /* valid but not implemented (e.g. M_sigma not a power of two, m > 8) */
};

enum nfft_precision {
  NFFT_F64 = 0, /* float64 nodes offsets, float64 window, complex128 data */
  NFFT_F32 = 1  /* float32 node offsets (cell index kept as an integer), float32
                   window and accumulation, complex64 data; deconvolution factors
                   and plan-time geometry are computed in float64 */
};

/*
 * nfft_plan -- precomputation for one node set (done once, Algorithm 3.7 step 0
 * minus the weights). Wraps the nodes onto [-1/2, 1/2)^d, splits
 * M_sigma x_j into a grid cell and an offset, sorts the nodes into spatial
 * tiles of the oversampled grid (the column index sets (4.7) grouped by
 * tile), and tabulates the deconvolution factors 1/(|I_Msigma| hat w(k)) of D.
 *
 *   out      receives the plan handle (set to NULL on failure)
 *   d        dimension, 1..3
 *   M        bandwidth per dimension, even, >= 2
 *   sigma    oversampling factor, >= 1; M_sigma must be a power of two in
 *            [8, 4096] (else NFFT_EUNSUPPORTED)
 *   m        window truncation, 1..8, with M_sigma >= 2m + 2
 *   N        number of nodes, 1 .. 2^31 - 1
 *   nodes    N*d float64 (host or device), finite
 *   precision  NFFT_F64 or NFFT_F32
 *   max_rhs  largest nrhs later passed to adjoint/forward (workspace is sized for it), >= 1
 *   stream   hipStream_t used for the plan's kernels; the call synchronises it
 * Returns NFFT_OK, NFFT_EINVAL, NFFT_EUNSUPPORTED, NFFT_ENOMEM or NFFT_EDEVICE.
 */
int nfft_plan(nfft_plan_t *out, int d, int M, double sigma, int m, int64_t N,
              const double *nodes, int precision, int max_rhs, void *stream);

/*
 * Tuning. The spreading and FFT kernels take seven launch parameters that
 * change their speed, never their result beyond rounding order. An array
 * tuning[NFFT_TUNE_*] selects them; an entry of 0, or an entry past
 * ntuning, selects the library default:
 *   NFFT_TUNE_TILE_EDGE       tile edge in cells: a power of two in [8, 256],
 *                             >= m; clipped to M_sigma (default: d = 1: 256,
 *                             d = 2: 16, d = 3: 8). Fixed at plan time.
 *   NFFT_TUNE_ITEM_NODES      most nodes in one spreading work item,
 *                             16..65536 (default 256). Fixed at plan time.
 *   NFFT_TUNE_SPREAD_THREADS  threads of a spreading work-group for d <= 2,
 *                             float32, one right-hand side per work-group:
 *                             64, 128 or 256 (default 128); 512 for spread
 *                             modes 5 and 7 (resolved to 256 for the others).
 *                             Float64 plans use it in spread mode 7 only.
 *   NFFT_TUNE_RHS_PER_GROUP   right-hand sides that one spreading work-group
 *                             takes when nrhs > 1 and d <= 2: 1, 2, 4 or 8
 *                             (default 1). Above 1 the node data and window
 *                             factors are read and evaluated once for them all.
 *   NFFT_TUNE_FFT_MIN_WG      an FFT pass gives each work-group fewer lines
 *                             while it would launch fewer work-groups than
 *                             this, 1..65536 (default 256); a pass whose lines
 *                             (of one right-hand side) then still go one per
 *                             work-group and number less than twice this gets
 *                             two or four times the threads per line (first
 *                             stage radix 4 or 2).
 *   NFFT_TUNE_SPREAD_PLANES   layout of the private LDS tiles of that float32
 *                             kernel: 1 = one complex tile per lane group,
 *                             2 = two groups per node, one for the real and
 *                             one for the imaginary plane (default 1).
 *   NFFT_TUNE_SPREAD_MODE     single right-hand-side spreading for d = 2:
 *                             1 = accumulation in LDS tiles, 2 = register
 *                             row sweep (nodes of a tile taken row by row,
 *                             the rows a node reaches kept in registers;
 *                             needs T + 2m <= 32; resolved to 1 elsewhere).
 *                             3 = as 1, with the 2m window factors per
 *                             dimension of every node read from a table
 *                             computed once per node set (Algorithm 2.4
 *                             step 1 with the values of the window
 *                             precomputed, as the node set is fixed) instead
 *                             of evaluated on every call; the plan keeps
 *                             16 m (float32) or 32 m (float64) more bytes
 *                             per node; resolved to 1 for d != 2, and a
 *                             call with nrhs > 1 and NFFT_TUNE_RHS_PER_GROUP
 *                             > 1 spreads as mode 1 does.
 *                             4 = as 3 without the table: each lane
 *                             evaluates its two window polynomials when the
 *                             node is spread, from offsets loaded from device
 *                             memory two nodes ahead (no extra memory);
 *                             resolved to 1 for d != 2, and as mode 3 for
 *                             several right-hand sides per work-group.
 *                             5 = float32, d = 2, tile edge 16: every
 *                             wave keeps the whole padded tile of its work
 *                             item in registers (lane c of a 32-lane half
 *                             owns padded column c) and takes two nodes of
 *                             one tile row at a time; no LDS accumulation,
 *                             the waves' tiles are summed in a fixed order
 *                             at the end; the window is evaluated per call
 *                             as in mode 4. Resolved to 4 for float64 plans
 *                             and other tile edges; one right-hand side per
 *                             work-group.
 *                             6 = float32, d = 2, tile edge 16, m <= 8, for
 *                             many right-hand sides: a work-group owns one
 *                             16 x 16 tile of the grid and 32 right-hand
 *                             sides, visits the nodes of that tile and of
 *                             its eight neighbours whose window reaches it
 *                             (plan-time lists, cut into units of at most
 *                             NFFT_TUNE_ITEM_NODES entries), and forms the
 *                             sums on the matrix cores, every grid cell in
 *                             one float32 accumulator in a fixed node order;
 *                             tiles of one unit write the grid directly, the
 *                             units of a longer list write partials summed
 *                             in unit order; no halo merges. Ignores the
 *                             thread count, planes and right-hand sides per
 *                             group. Resolved to 5 (and so on) where not
 *                             supported.
 *                             7 = d = 2, tile edge 16, 2m + 1 <= 16, float32
 *                             or float64 (sums in float64 accumulators, in a
 *                             fixed order): the padded tile of a work item
 *                             on the matrix cores; the nodes of one tile row reach 16
 *                             padded rows, so four nodes at a time form a
 *                             16 x 32 block of products (rows held as
 *                             slots that shift with the tile row); the
 *                             waves' tiles are summed in a fixed order at
 *                             the end, and the output is the same padded
 *                             tile as modes 1 .. 5 write. Also float32,
 *                             d = 3, tile edge 8, 2m <= 8: one wave holds
 *                             the padded 3-D tile (one 16 x 16 block per
 *                             plane) and takes four nodes of one tile row
 *                             at a time. One right-hand side per
 *                             work-group. Resolved to 5 (and so on; mode 1
 *                             for d = 3) where not supported.
 *                             Default 1; the row sweep wins with many
 *                             right-hand sides per call, and in float32
 *                             takes two of them per wave when
 *                             NFFT_TUNE_RHS_PER_GROUP >= 2.
 * The environment variables NFFT_TILE_EDGE, NFFT_ITEM_NODES,
 * NFFT_SPREAD_THREADS, NFFT_RHS_PER_GROUP, NFFT_FFT_MIN_WG, NFFT_SPREAD_PLANES
 * and NFFT_SPREAD_MODE replace the defaults. A combination whose spreading
 * work-group does not fit in LDS is NFFT_EUNSUPPORTED.
 */
enum nfft_tune {
  NFFT_TUNE_TILE_EDGE = 0,
  NFFT_TUNE_ITEM_NODES = 1,
  NFFT_TUNE_SPREAD_THREADS = 2,
  NFFT_TUNE_RHS_PER_GROUP = 3,
  NFFT_TUNE_FFT_MIN_WG = 4,
  NFFT_TUNE_SPREAD_PLANES = 5,
  NFFT_TUNE_SPREAD_MODE = 6,
  NFFT_TUNE_COUNT = 7
};

/*
 * nfft_plan_tuned -- nfft_plan with explicit tuning (see above); tuning may
 * be NULL (ntuning ignored). Arguments and status codes as for nfft_plan.
 */
int nfft_plan_tuned(nfft_plan_t *out, int d, int M, double sigma, int m, int64_t N,
                    const double *nodes, int precision, int max_rhs, const int *tuning,
                    int ntuning, void *stream);

/* nfft_get_tuning -- the plan's resolved tuning into out[0..n-1], n <= NFFT_TUNE_COUNT. */
int nfft_get_tuning(nfft_plan_t plan, int *out, int n);

/*
 * nfft_set_tuning -- change a launch-time parameter of an existing plan
 * (NFFT_TUNE_SPREAD_THREADS, NFFT_TUNE_RHS_PER_GROUP, NFFT_TUNE_FFT_MIN_WG,
 * NFFT_TUNE_SPREAD_PLANES, NFFT_TUNE_SPREAD_MODE; value 0 restores the
 * default). Tile edge and item size are fixed at plan
 * time: NFFT_EINVAL for them. Takes effect for transforms enqueued later.
 * Switching a d = 2 plan to spread mode 3 the first time builds its window
 * factor table: it allocates device memory (NFFT_ENOMEM if there is none;
 * the tuning is then unchanged) and runs one kernel on the null stream,
 * which the call waits for.
 */
int nfft_set_tuning(nfft_plan_t plan, int knob, int value);

/*
 * nfft_plan_autotune -- plan a node set with the tuning that runs the
 * adjoint fastest on this device for nrhs right-hand sides. Candidate tile
 * edges and work-item sizes each get a plan (the node sort is redone per
 * candidate); on each, the launch-time parameters are swept; every candidate
 * is timed with HIP events over several adjoint calls on zero data (the run
 * time of the kernels does not depend on the values). The fastest plan is
 * returned; the others are freed. Its tuning is read with nfft_get_tuning.
 * Weights are not set: call nfft_set_weights before nfft_adjoint.
 *   nrhs        right-hand sides per call to tune for, 1..max_rhs
 *   best_ms     if not NULL, receives the winner's milliseconds per adjoint
 *   other arguments as for nfft_plan; the call synchronises `stream` and
 *   takes of the order of a second for a million nodes.
 */
int nfft_plan_autotune(nfft_plan_t *out, int d, int M, double sigma, int m, int64_t N,
                       const double *nodes, int precision, int max_rhs, int nrhs,
                       double *best_ms, void *stream);

/*
 * nfft_plan_clone -- a second handle on the same node set with its own
 * workspace for max_rhs right-hand sides. The clone shares the source plan's
 * sorted nodes, weights, tables and tuning (setting weights through either handle
 * changes both) but not its workspace, so transforms through different
 * handles may run concurrently on different streams. Each handle is
 * destroyed separately; the shared data is freed with the last one.
 *   out     receives the new handle (NULL on failure)
 *   stream  hipStream_t for initialising the workspace; the call synchronises it
 */
int nfft_plan_clone(nfft_plan_t src, int max_rhs, nfft_plan_t *out, void *stream);

/*
 * nfft_set_weights -- store W = diag(w) of eq. (3.6); the weights are complex in general.
 *   w  N complex128 values (host or device) in the caller's node order.
 * The plan keeps its own copy (permuted to its internal order, rounded to
 * complex64 for an NFFT_F32 plan); the call synchronises `stream`.
 */
int nfft_set_weights(nfft_plan_t plan, const double *w, void *stream);

/*
 * nfft_adjoint -- fhat = D^* F^* B^* W f for nrhs right-hand sides (eq. (3.7)):
 * scale by w_j and spread with the window (Algorithm 2.4 step 1), d-variate FFT
 * of the M_sigma^d grid (step 2), deconvolve by hat w and crop to I_M (step 3).
 *   f     device, nrhs*N complex (plan precision), caller's node order
 *   fhat  device, nrhs*M^d complex (plan precision), output
 *   nrhs  1 .. max_rhs
 * NFFT_ESTATE if nfft_set_weights has not been called.
 */
int nfft_adjoint(nfft_plan_t plan, const void *f, void *fhat, int nrhs, void *stream);

/*
 * nfft_adjoint_scratch -- nfft_adjoint for callers that cannot allocate
 * device memory or must not use the plan's workspace (code under HIP graph
 * capture, tight serving loops that run many requests on one resident plan,
 * harnesses that forbid allocation): the same kernels and the same result,
 * with the intermediate buffers (tile partials, item partials of split tiles,
 * FFT buffers) placed in a file-scope device array of the library, 32 MiB per
 * GPU, held from the library's first use on that GPU until the process ends.
 * The call allocates nothing and frees nothing; its first call on a device
 * looks the array's address up once (hipGetSymbolAddress).
 *   f, fhat, nrhs, stream  as for nfft_adjoint
 * The intermediate buffers of one call take about nrhs * 8 (float32) or 16
 * (float64) bytes times (tiles + split-tile items) * (tile edge + 2m)^d plus
 * M_sigma^(d-1) M (and M_sigma M^2 for d = 3); a call that needs more than
 * 32 MiB returns NFFT_EUNSUPPORTED before anything is enqueued (e.g. the
 * 512 x 512 polar set at M = 256 fits in both precisions, a 3-D jittered set
 * at M = 64 does not). Every call on one GPU uses the same array: calls that
 * overlap on that GPU (other streams, other plans, other threads) race and
 * give wrong results; the caller serialises them. Each call first clears the
 * part that must start at zero (the slots of tiles without nodes) with a
 * kernel, no memset. NFFT_ESTATE without weights.
 */
int nfft_adjoint_scratch(nfft_plan_t plan, const void *f, void *fhat, int nrhs, void *stream);

/*
 * nfft_forward -- f = B F D fhat for nrhs right-hand sides (Algorithm 2.1):
 * deconvolve and zero-pad (step 1), inverse FFT (step 2), window sums at the
 * nodes (step 3). No weights are involved.
 *   fhat  device, nrhs*M^d complex (plan precision)
 *   f     device, nrhs*N complex (plan precision), output in the caller's order
 */
int nfft_forward(nfft_plan_t plan, const void *fhat, void *f, int nrhs, void *stream);

/*
 * nfft_refine -- the reconstruction of nfft_adjoint improved iteratively with
 * the same weights: fhat_0 = A^* W f (eq. (3.7)), then
 *     fhat_{k+1} = fhat_k + A^* W (f - A fhat_k),   k = 0 .. iters-1,
 * with A and A^* the plan's nfft_forward and weighted nfft_adjoint. The
 * iterates are the partial sums of the Neumann series of (A^* W A)^{-1} in the
 * proof of Theorem 3.15 applied to A^* W f: with A^* W A = I + E and
 * ||E||_2 < 1 (e.g. |I_M| eps < 1, eps of (3.36)) they tend to the weighted
 * least-squares solution (A^* W A)^{-1} A^* W f, and for samples of a
 * trigonometric polynomial of degree M the error shrinks by ||E||_2 per
 * step (k = 0 is the bound (3.37)). The paper leaves the iteration open;
 * this is the plain one with the weights as approximate inverse.
 *   f      device, nrhs*N complex (plan precision), caller's node order
 *   fhat   device, nrhs*M^d complex (plan precision), output fhat_iters
 *   nrhs   1 .. max_rhs
 *   iters  0 .. 1000 correction steps (0: the same result as nfft_adjoint)
 *   res    NULL, or host memory for iters+1 doubles: the relative residuals
 *          ||f - A fhat_k||_2 / ||f||_2, k = 0..iters, over all right-hand
 *          sides (float64 sums in a fixed order; one more forward transform,
 *          and the call waits for `stream`)
 * Each step costs one forward and one adjoint; the residual is formed where
 * the forward writes its samples and the correction is added where the
 * adjoint writes its coefficients. The first call allocates max_rhs * N
 * complex values of workspace for the plan (NFFT_ENOMEM if there is none). NFFT_ESTATE without weights; NFFT_EINVAL for a bad
 * nrhs or iters, before anything is enqueued.
 */
int nfft_refine(nfft_plan_t plan, const void *f, void *fhat, int nrhs, int iters, double *res,
                void *stream);

/*
 * nfft_weights -- density-compensation weights of Algorithm 3.6 for a node
 * set, computed on the device in float64. The conditions (3.14),
 * A_2M^T w = e_0 on I_2M, are solved by conjugate gradients from zero: on
 * the normal equations of the second kind (3.15) when |I_2M| = (2M)^d <= N
 * (then w = conj(A_2M) v), otherwise on those of the first kind (3.16). The
 * products with A_2M^T and conj(A_2M) are this library's float64 NFFT at
 * bandwidth 2M with window parameter m and oversampling sigma (so
 * sigma * 2M must give a power-of-two M_sigma in [8, 4096]).
 *   nodes   N*d float64 (host or device), as for nfft_plan
 *   tol     stop once ||r|| <= tol ||b|| for the normal-equation residual r, > 0
 *   maxit   iteration limit, >= 1
 *   w       device, N complex128 in the caller's node order (output)
 *   info    host, 4 doubles, or NULL: iterations, final relative residual,
 *           branch (15 or 16 for (3.15) / (3.16)) and epsilon =
 *           max_k |[A_2M^T w]_k - delta_{0,k}| over I_2M (the quantity of
 *           (3.36)), evaluated with the same NFFT
 *   stream  hipStream_t; the call synchronises it (convergence is tested on
 *           the host after every iteration)
 * Returns the nfft_plan status codes; NFFT_EINVAL for a NULL w, tol <= 0,
 * maxit < 1 or an odd M (M is the bandwidth of the reconstruction).
 */
int nfft_weights(int d, int M, double sigma, int m, int64_t N, const double *nodes, double tol,
                 int maxit, void *w, double *info, void *stream);

/*
 * nfft_weights_ex -- nfft_weights with a choice of scheme:
 *   NFFT_WEIGHTS_ALG36    Algorithm 3.6 as above (info[2] = 15 or 16);
 *   NFFT_WEIGHTS_RELAXED  the summed conditions A A^* w = 1_N of (3.63),
 *                         float64 CG with the NFFT at bandwidth M; info[2] = 63
 *                         and info[3] = max_j |[A A^* w]_j - 1|;
 *   NFFT_WEIGHTS_PCF      (3.62), the minimiser of ||A A^* W - I_N||_F over
 *                         diagonal W: w_j = |I_M| / sum_h |[A A^*]_{j,h}|^2,
 *                         evaluated directly over all N^2 pairs in float64
 *                         with the Dirichlet-kernel form of the entries
 *                         (sigma, m, tol, maxit unused); info[2] = 62.
 */
enum nfft_weight_scheme { NFFT_WEIGHTS_ALG36 = 0, NFFT_WEIGHTS_RELAXED = 1, NFFT_WEIGHTS_PCF = 2 };
int nfft_weights_ex(int d, int M, double sigma, int m, int64_t N, const double *nodes, int scheme,
                    double tol, int maxit, void *w, double *info, void *stream);

/*
 * Optimized sparse matrix (Section 4): Algorithm 4.3 on the device in float64
 * and the reconstruction of Algorithm 4.4, h_opt = D^* F^* B_opt^* f
 * (eq. (4.12)), a modified adjoint NFFT that needs no weights.
 *
 * nfft_bopt_build -- compute B_opt for the plan's node set and keep it with
 * the plan (shared with its clones). B_opt is real and has the nonzero
 * pattern of B (2.15): grid column l holds the nodes whose closed window
 * support reaches l periodically. Its values minimise
 * ||H_l b - |I_Ms|^{-1} D^{-1} f_l||_2 over real b (H_l of (4.11)), i.e.
 * solve Re(H_l^* H_l) b = Re(v_l) with (4.13) and (4.14); the values are kept
 * in the plan's precision. A column whose Cholesky meets a pivot below 1e-13
 * |I_M| has singular normal equations (duplicate nodes, or more nodes than
 * the polynomials of degree M tell apart within one window support); it is
 * factorised again with 1e-12 |I_M| added to the diagonal, which reaches the
 * least-squares objective. Columns of up to about 190 nodes keep their Gram
 * triangle in LDS; larger ones, up to 16000 nodes, keep it and their
 * per-node arrays in a device-memory workspace of 8 (n^2/2 + 5.5 n) bytes
 * for n nodes, largest columns first, in batches of at most 4 GiB (or one
 * column), freed before the call returns; their Cholesky goes by panels of
 * 32 columns. A column of n nodes costs about n^3 / 3 float64 operations on
 * one work-group.
 *   nodes  the plan's nodes again, N*d float64 (host or device), same order
 *   info   host, 3 doubles, or NULL: largest column set, number of nonzeros,
 *          number of columns with singular normal equations
 * NFFT_EUNSUPPORTED if some column holds more than 16000 nodes (NFFT_ENOMEM
 * if the workspace cannot be had); NFFT_ESTATE if already built.
 * Synchronises `stream`.
 */
int nfft_bopt_build(nfft_plan_t plan, const double *nodes, double *info, void *stream);

/*
 * nfft_bopt_adjoint -- h_opt = D^* F^* B_opt^* f for nrhs right-hand sides
 * (Algorithm 4.4 step 1); f and fhat as for nfft_adjoint. NFFT_ESTATE before
 * nfft_bopt_build. The sparse product runs a group of lanes per grid column,
 * 4 to 64 lanes sized at build time to the mean column length (the
 * environment variable NFFT_BOPT_LANES, read by nfft_bopt_build, fixes it).
 */
int nfft_bopt_adjoint(nfft_plan_t plan, const void *f, void *fhat, int nrhs, void *stream);

/*
 * nfft_bopt_inverse_adjoint -- Remark 4.6: an approximate solution of
 * A^* f = h (the inverse adjoint NFFT) by f = B_opt F D h, i.e. Algorithm
 * 2.1 with B_opt in place of B, for nrhs right-hand sides.
 *   h  device, nrhs*M^d complex (plan precision), C order of I_M
 *   f  device, nrhs*N complex (plan precision), caller's node order (output)
 * NFFT_ESTATE before nfft_bopt_build.
 */
int nfft_bopt_inverse_adjoint(nfft_plan_t plan, const void *h, void *f, int nrhs, void *stream);

/*
 * nfft_bopt_get -- copy B_opt to host memory by grid columns (C order of
 * s_t = l_t + M_sigma/2): nnz receives the number of nonzeros; col_ptr
 * (M_sigma^d + 1 entries), nodes and vals (nnz entries each, vals as float64)
 * are filled where not NULL. Synchronous.
 */
int nfft_bopt_get(nfft_plan_t plan, int64_t *nnz, int64_t *col_ptr, int32_t *nodes, double *vals);

/* nfft_destroy -- wait for the plan's outstanding work and free it. NULL is a no-op. */
int nfft_destroy(nfft_plan_t plan);

/*
 * nfft_footprint -- upper bound of the device bytes a plan with these
 * parameters and the default tile edge and work-item size allocates, the
 * window factor table of spread mode 3 included (the exact figure depends on
 * how the nodes fill the tiles; nfft_plan_info reports it). Not included:
 * B_opt (nfft_bopt_build) and the workspace nfft_refine allocates on its
 * first call. -1 on invalid arguments.
 */
int64_t nfft_footprint(int d, int M, double sigma, int m, int64_t N, int precision, int max_rhs);

/* nfft_strerror -- static text for a status code. */
const char *nfft_strerror(int status);

/* nfft_last_error -- detail of the last failure on `plan` (or of the last
 * failure with no plan when plan is NULL); owned by the library. */
const char *nfft_last_error(nfft_plan_t plan);

/*
 * nfft_plan_info -- plan geometry, written to out[0..n-1] (n <= 13):
 *   0 d, 1 M, 2 M_sigma, 3 m, 4 N, 5 precision, 6 max_rhs,
 *   7 tile edge (cells), 8 number of tiles, 9 number of spreading work items,
 *   10 largest tile population, 11 device bytes this handle keeps alive
 *   (shared node data plus its workspace), 12 workspace bytes of this handle.
 */
int nfft_plan_info(nfft_plan_t plan, int64_t *out, int n);

/*
 * nfft_permutation -- the plan's internal node order: perm[i] is the caller
 * index of the i-th node in tile order (int32, host memory, N entries).
 */
int nfft_permutation(nfft_plan_t plan, int32_t *perm_host);

/*
 * Stage timing. With profiling on, nfft_adjoint, nfft_forward and
 * nfft_bopt_adjoint record HIP events on their stream around each kernel
 * stage; nfft_stage_times waits for them and returns, per stage, the
 * accumulated milliseconds and the number of calls since the last reset:
 *   out[2*s] = milliseconds, out[2*s+1] = calls, for s = 0..NFFT_STAGES-1
 * Stages: 0 spreading (adjoint step 1), 1 sum of tiles split into several
 * work items, 2 first FFT pass with the merge of tile partials into grid
 * cells, 3 remaining FFT passes with deconvolution and crop (adjoint steps 2
 * and 3), 4 forward deconvolution, zero padding and FFT passes (Algorithm 2.1
 * steps 1-2), 5 forward window sums (Algorithm 2.1 step 3), 6 the sparse
 * product B_opt^* f of nfft_bopt_adjoint (Algorithm 4.4 step 1), 7 its FFT
 * passes with deconvolution and crop.
 */
#define NFFT_STAGES 8
int nfft_set_profiling(nfft_plan_t plan, int enable);
int nfft_stage_times(nfft_plan_t plan, double *out, int n, int reset);

#ifdef __cplusplus
}
#endif

#endif /* NFFT_MI355X_H */
