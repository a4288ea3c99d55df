// Host side of the library: plan construction, workspace, the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/nfft.h"
#include "internal.hpp"
#include "window.hpp"

using nfft::cplx;
using nfft::Geom;

namespace {

// Environment replacements of the tuning defaults (positive integers only).
int env_int(const char* name, int fallback) {
  const char* v = std::getenv(name);
  if (!v || !*v) return fallback;
  char* end = nullptr;
  long x = std::strtol(v, &end, 10);
  return (end && *end == 0 && x > 0 && x < (1 << 20)) ? (int)x : fallback;
}

// Library defaults of the tuning parameters (NFFT_TUNE_*), before clipping.
int default_tuning(int knob, int d) {
  switch (knob) {
    case NFFT_TUNE_TILE_EDGE: return env_int("NFFT_TILE_EDGE", d == 1 ? 256 : (d == 2 ? 16 : 8));
    case NFFT_TUNE_ITEM_NODES: return env_int("NFFT_ITEM_NODES", 256);
    case NFFT_TUNE_SPREAD_THREADS: return env_int("NFFT_SPREAD_THREADS", 128);
    case NFFT_TUNE_RHS_PER_GROUP: return env_int("NFFT_RHS_PER_GROUP", 1);
    case NFFT_TUNE_FFT_MIN_WG: return env_int("NFFT_FFT_MIN_WG", 256);
    case NFFT_TUNE_SPREAD_PLANES: return env_int("NFFT_SPREAD_PLANES", 1);
    case NFFT_TUNE_SPREAD_MODE: return env_int("NFFT_SPREAD_MODE", 1);
    default: return 0;
  }
}

thread_local std::string g_noplan_error;

struct StageEvents {
  hipEvent_t ev[5];
  int n;       // events used
  int kind;    // 0 adjoint, 1 forward, 2 adjoint with B_opt
};

// Device data that clones of a plan share: the sorted nodes, the weights, the
// work-item tables and the window and deconvolution tables. Freed with the
// last handle that refers to it.
struct SharedData {
  std::vector<void*> allocs;
  int64_t bytes = 0;
  bool has_weights = false;
  // optimized sparse matrix (Algorithm 4.3), by grid columns
  bool has_bopt = false;
  int64_t* bopt_ptr = nullptr;    // column starts, M_sigma^d + 1
  int32_t* bopt_node = nullptr;   // node ids (caller order), by column
  void* bopt_val = nullptr;       // values (plan precision), by column
  int64_t bopt_nnz = 0;
  int bopt_nmax = 0;
  int bopt_lanes = 64;            // lanes per column of the sparse product
  int32_t* bopt_lo = nullptr;     // first support cell per node and dimension (caller order)
  void* bopt_rows = nullptr;      // values by rows: N x (2m+1)^d in footprint order
  // window factors of every node (d = 2, spread mode 3), [N][2m][2] in tile order
  void* psi = nullptr;
  // first node of every tile (tile order), nbins + 1, on the host
  std::vector<int32_t> hbin_start;
  // spread mode 6: per-tile lists of the nodes that reach the tile, the work
  // units over them and the tiles cut into several units (nfft::GatherArgs)
  int32_t* gl_node = nullptr;
  int32_t* gl_hdr = nullptr;
  int32_t* g_iperm = nullptr;      // caller index -> tile order (the node-major copy's weights)
  int32_t* g_units = nullptr;
  int32_t* g_split = nullptr;
  int g_nunits = 0, g_nsplit = 0, g_nslots = 0;
  int64_t g_bytes = 0;
  ~SharedData() {
    for (void* q : allocs) (void)hipFree(q);
  }
};

}  // namespace

struct nfft_plan_s {
  int device = 0;
  int d = 0, M = 0, Ms = 0, m = 0, prec = 0, max_rhs = 1;
  double sigma = 1.0, b = 0.0;
  int64_t N = 0;
  Geom g{};
  int maxpop = 0;
  int tune[NFFT_TUNE_COUNT] = {0};   // resolved tuning
  int64_t bytes = 0;                 // workspace bytes owned by this handle
  std::shared_ptr<SharedData> shared; // node data, weights and tables
  std::string last_error;
  // device buffers
  int32_t* perm = nullptr;
  uint32_t* loc = nullptr;
  void* frac = nullptr;
  void* w = nullptr;
  int32_t* item_start = nullptr;
  int32_t* item_count = nullptr;
  int32_t* item_bin = nullptr;
  int32_t* item_slot = nullptr;    // itemp slot of an item of a split tile, else -1
  int32_t* multi_bin = nullptr;    // split tiles
  int32_t* multi_first = nullptr;  // first itemp slot of each split tile
  int nmulti = 0;
  int nslots = 0;                  // itemp slots
  int32_t* empty_bins = nullptr;   // tiles without nodes (their slots are never written)
  void* gpart = nullptr;           // spread mode 6 partials [max_rhs][slot][256]
  void* gft = nullptr;             // spread mode 6 node-major samples [groups of 32][N][32]
  int nempty = 0;
  void* tilep = nullptr;           // tile partials [rhs][tile][P^d]
  void* itemp = nullptr;           // item partials of split tiles [rhs][slot][P^d]
  void* coef = nullptr;            // window polynomials [2m][deg + 1]
  double poly_err = 0.0;           // verified max error / psi(0)
  void* bufA = nullptr;
  void* bufB = nullptr;
  void* grid = nullptr;
  void* tw = nullptr;
  void* fac = nullptr;
  // weighted iterative refinement, allocated on first use: residuals
  // [max_rhs][N], corrections [max_rhs][M^d], norm partials and results
  void* ref_r = nullptr;
  double* ref_red = nullptr;
  std::vector<void*> allocs;
  // profiling
  bool profiling = false;
  std::vector<StageEvents> pending;
  std::vector<hipEvent_t> event_pool;
  double stage_ms[NFFT_STAGES] = {0};
  int64_t stage_calls[NFFT_STAGES] = {0};
};

namespace {

int fail(nfft_plan_t p, int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (p)
    p->last_error = buf;
  else
    g_noplan_error = buf;
  return status;
}

#define HIP_TRY(p, expr)                                                                     \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail((p), e_ == hipErrorOutOfMemory ? NFFT_ENOMEM : NFFT_EDEVICE, "%s: %s (%s)", \
                  #expr, hipGetErrorString(e_), __func__);                                   \
  } while (0)

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int oversampled(int M, double sigma) {
  double a = std::ceil(sigma * (double)M);
  return 2 * (int)std::ceil(a / 2.0);
}

// Largest LDS a work-group may use on gfx950.
constexpr size_t kMaxLds = 160 * 1024;
// nodes of one B_opt column: a Cholesky of O(n^3) on one work-group with the
// triangle in device memory (at 16000 nodes, 1 GiB per column)
constexpr int kMaxBoptColumn = 16000;

size_t cbytes(int prec) { return prec == NFFT_F64 ? 16 : 8; }
size_t rbytes(int prec) { return prec == NFFT_F64 ? 8 : 4; }

int validate(int d, int M, double sigma, int m, int64_t N, int precision, int max_rhs,
             nfft_plan_t p) {
  if (d < 1 || d > 3) return fail(p, NFFT_EINVAL, "d = %d, expected 1, 2 or 3", d);
  if (M < 2 || (M % 2) != 0) return fail(p, NFFT_EINVAL, "M = %d, expected an even M >= 2", M);
  if (!(sigma >= 1.0) || !std::isfinite(sigma))
    return fail(p, NFFT_EINVAL, "sigma = %g, expected a finite sigma >= 1", sigma);
  if (m < 1) return fail(p, NFFT_EINVAL, "m = %d, expected m >= 1", m);
  if (N < 1 || N > 0x7fffffffLL) return fail(p, NFFT_EINVAL, "N = %lld out of range", (long long)N);
  if (precision != NFFT_F64 && precision != NFFT_F32)
    return fail(p, NFFT_EINVAL, "precision = %d, expected NFFT_F64 or NFFT_F32", precision);
  if (max_rhs < 1 || max_rhs > 65535)
    return fail(p, NFFT_EINVAL, "max_rhs = %d, expected 1..65535", max_rhs);
  if (sigma * M > 1e7) return fail(p, NFFT_EUNSUPPORTED, "sigma * M too large");
  const int Ms = oversampled(M, sigma);
  if (Ms < 2 * m + 2)
    return fail(p, NFFT_EINVAL, "M_sigma = %d < 2m + 2 = %d (window wraps onto itself)", Ms,
                2 * m + 2);
  if (m > 8) return fail(p, NFFT_EUNSUPPORTED, "m = %d > 8 is not built", m);
  if (!is_pow2(Ms) || Ms < 8 || Ms > 4096)
    return fail(p, NFFT_EUNSUPPORTED, "M_sigma = %d: only powers of two in [8, 4096] are built",
                Ms);
  if (M > Ms) return fail(p, NFFT_EINVAL, "M_sigma < M");
  return NFFT_OK;
}

int64_t ipow(int64_t a, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= a;
  return r;
}

// Resolve a tuning array (0 or missing = default) and check it against the
// problem: tile edge a power of two in [8, 256] (tile-local cells are packed
// into 8 bits per dimension), at least m, clipped to M_sigma; the spreading
// work-groups of the chosen shape must fit in LDS.
int resolve_tuning(int d, int Ms, int m, int precision, const int* in, int n, int* out,
                   nfft_plan_t p) {
  for (int k = 0; k < NFFT_TUNE_COUNT; ++k) {
    const int v = (in && k < n) ? in[k] : 0;
    if (v < 0) return fail(p, NFFT_EINVAL, "tuning[%d] = %d is negative", k, v);
    out[k] = v ? v : default_tuning(k, d);
  }
  int& T = out[NFFT_TUNE_TILE_EDGE];
  if (!is_pow2(T) || T < 8 || T > 256)
    return fail(p, NFFT_EINVAL, "tile edge %d: expected a power of two in [8, 256]", T);
  T = std::min(T, Ms);
  if (T < m) return fail(p, NFFT_EUNSUPPORTED, "tile edge %d < m = %d", T, m);
  const int K = out[NFFT_TUNE_ITEM_NODES];
  if (K < 16 || K > 65536) return fail(p, NFFT_EINVAL, "item nodes %d: expected 16..65536", K);
  int& nt = out[NFFT_TUNE_SPREAD_THREADS];
  if (nt != 64 && nt != 128 && nt != 256 && nt != 512)
    return fail(p, NFFT_EINVAL, "spread threads %d: expected 64, 128, 256 or 512", nt);
  const int nr = out[NFFT_TUNE_RHS_PER_GROUP];
  if (nr != 1 && nr != 2 && nr != 4 && nr != 8)
    return fail(p, NFFT_EINVAL, "rhs per group %d: expected 1, 2, 4 or 8", nr);
  if (d == 3 && nr != 1) out[NFFT_TUNE_RHS_PER_GROUP] = 1;  // d = 3 has no multi-rhs kernel
  const int planes = out[NFFT_TUNE_SPREAD_PLANES];
  if (planes != 1 && planes != 2)
    return fail(p, NFFT_EINVAL, "spread planes %d: expected 1 or 2", planes);
  int& mode = out[NFFT_TUNE_SPREAD_MODE];
  if (mode < 1 || mode > 7)
    return fail(p, NFFT_EINVAL, "spread mode %d: expected 1 .. 7", mode);
  // the matrix-core register tile: d = 2, tile edge 16, 2m + 1 <= 16, or
  // d = 3, tile edge 8, 2m <= 8 (float32 or float64); elsewhere the vector
  // register tile (and its own fallback)
  if (mode == 7 && !nfft::spread_mma_supported(d, T, precision == NFFT_F64, m) &&
      !nfft::spread3_mma_supported(d, T, precision == NFFT_F64, m))
    mode = 5;
  // the grid-tile gather: float32, d = 2, tile edge 16, m <= 8; elsewhere
  // the register-tile kernel (and its own fallback)
  if (mode == 6 && !nfft::spread_gather_supported(d, T, precision == NFFT_F64, m)) mode = 5;
  if (mode == 2 && !nfft::spread_rows_supported(d, T + 2 * m)) mode = 1;
  // the register-tile kernel: float32, d = 2, tile edge 16; elsewhere the LDS
  // kernel with the same window evaluation
  if (mode == 5 && !nfft::spread_reg_supported(d, T, precision == NFFT_F64)) mode = 4;
  if ((mode == 3 || mode == 4) && d != 2) mode = 1;  // laid out for d = 2
  // 512 threads: the register-tile kernels only
  if (nt == 512 && mode != 5 && mode != 7) nt = 256;
  const int fw = out[NFFT_TUNE_FFT_MIN_WG];
  if (fw < 1 || fw > 65536) return fail(p, NFFT_EINVAL, "fft min work-groups %d: expected 1..65536", fw);
  const int P = T + 2 * m;
  const int Ptot = (int)ipow(P, d);
  const bool f64 = precision == NFFT_F64;
  const size_t one = mode == 6   ? nfft::spread_gather_lds_bytes(m)
                     : mode == 7 && d == 3 ? nfft::spread3_mma_lds_bytes(f64)
                     : mode == 7 ? nfft::spread_mma_lds_bytes(m, nt, precision == NFFT_F64)
                     : mode == 5 ? nfft::spread_reg_lds_bytes(m)
                                 : nfft::spread_lds_bytes(d, f64, m, T, Ptot, nt, 1, planes);
  const size_t multi = out[NFFT_TUNE_RHS_PER_GROUP] > 1
                           ? nfft::spread_lds_bytes(d, f64, m, T, Ptot, nt,
                                                    out[NFFT_TUNE_RHS_PER_GROUP], planes)
                           : 0;
  if (one == 0 || one > kMaxLds || multi > kMaxLds)
    return fail(p, NFFT_EUNSUPPORTED,
                "padded tile of %d cells (d = %d, m = %d, tile edge %d) does not fit in LDS with "
                "this work-group shape", Ptot, d, m, T);
  return NFFT_OK;
}

// Modified Bessel function I_0 by its power series (all terms positive).
long double bessel_i0(long double z) {
  const long double q = z * z / 4.0L;
  long double term = 1.0L, sum = 1.0L;
  for (int n = 1; n < 2000; ++n) {
    term *= q / ((long double)n * (long double)n);
    sum += term;
    if (term < 1e-24L * sum) break;
  }
  return sum;
}

// Device allocation owned by the plan's shared data (shared = true) or by
// this handle's workspace.
template <typename T>
int dalloc(nfft_plan_t p, T** ptr, size_t bytes, bool shared = true) {
  *ptr = nullptr;
  if (bytes == 0) bytes = 16;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess)
    return fail(p, e == hipErrorOutOfMemory ? NFFT_ENOMEM : NFFT_EDEVICE,
                "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  if (shared) {
    p->shared->allocs.push_back(q);
    p->shared->bytes += (int64_t)bytes;
  } else {
    p->allocs.push_back(q);
    p->bytes += (int64_t)bytes;
  }
  *ptr = static_cast<T*>(q);
  return NFFT_OK;
}

#define TRY(expr)                  \
  do {                             \
    int s_ = (expr);               \
    if (s_ != NFFT_OK) return s_;  \
  } while (0)

void free_plan(nfft_plan_t p) {
  if (!p) return;
  for (auto& se : p->pending)
    for (int i = 0; i < se.n; ++i) p->event_pool.push_back(se.ev[i]);
  for (auto e : p->event_pool) (void)hipEventDestroy(e);
  for (void* q : p->allocs) (void)hipFree(q);
  delete p;
}

struct ScopedFree {
  std::vector<void*> ptrs;
  ~ScopedFree() {
    for (void* q : ptrs) (void)hipFree(q);
  }
};

// psi(t) = e^{-b m} sinh(b z) / z, z = sqrt(m^2 - t^2): the window in grid
// units scaled by pi e^{-b m} (the deconvolution factors undo the scale).
long double psi_ld(long double t, long double b, long double m) {
  const long double z2 = (m - t) * (m + t);
  if (z2 <= 0.0L) return b * std::exp(-b * m);
  const long double z = std::sqrt(z2);
  // e^{b(z - m)} (1 - e^{-2bz}) / (2z), with z - m = -t^2 / (z + m)
  return std::exp(-b * t * t / (z + m)) * (-std::expm1(-2.0L * b * z)) / (2.0L * z);
}

// Per-cell window polynomials in y = 2 frac - 1: Chebyshev interpolation of
// degree DEG at the Chebyshev points, converted to monomial coefficients.
// Returns the largest error on a fine grid relative to psi(0).
template <typename R>
double fit_window(int m, long double b, std::vector<R>& coef) {
  constexpr int DEG = nfft::PolyDeg<R>::value;
  constexpr int n = DEG + 1;
  const long double pi = 3.14159265358979323846264338327950288L;
  coef.assign((size_t)2 * m * n, (R)0);
  double worst = 0.0;
  const long double p0 = psi_ld(0.0L, b, m);
  for (int i = 0; i < 2 * m; ++i) {
    const long double shift = (long double)(m - 1 - i);
    long double fv[n], ch[n];
    for (int j = 0; j < n; ++j) {
      const long double y = std::cos(pi * (j + 0.5L) / n);
      fv[j] = psi_ld((y + 1.0L) / 2.0L + shift, b, m);
    }
    for (int k = 0; k < n; ++k) {
      long double acc = 0.0L;
      for (int j = 0; j < n; ++j) acc += fv[j] * std::cos(pi * k * (j + 0.5L) / n);
      ch[k] = acc * 2.0L / n;
    }
    ch[0] *= 0.5L;
    // monomial coefficients: T_0 = 1, T_1 = y, T_{k+1} = 2y T_k - T_{k-1}
    long double Tm[n], Tc[n], Tn[n], mono[n];
    for (int k = 0; k < n; ++k) Tm[k] = Tc[k] = mono[k] = 0.0L;
    Tm[0] = 1.0L;
    Tc[1] = 1.0L;
    mono[0] += ch[0];
    for (int k = 1; k < n; ++k) {
      for (int q = 0; q < n; ++q) mono[q] += ch[k] * Tc[q];
      for (int q = 0; q < n; ++q) Tn[q] = (q > 0 ? 2.0L * Tc[q - 1] : 0.0L) - Tm[q];
      for (int q = 0; q < n; ++q) {
        Tm[q] = Tc[q];
        Tc[q] = Tn[q];
      }
    }
    for (int q = 0; q < n; ++q) coef[(size_t)i * n + q] = (R)mono[q];
    for (int s = 0; s <= 512; ++s) {
      const long double y = -1.0L + 2.0L * s / 512.0L;
      long double v = (long double)coef[(size_t)i * n + DEG];
      for (int q = DEG - 1; q >= 0; --q) v = v * y + (long double)coef[(size_t)i * n + q];
      const long double ex = psi_ld((y + 1.0L) / 2.0L + shift, b, m);
      worst = std::max(worst, (double)(std::fabs(v - ex) / p0));
    }
  }
  return worst;
}

template <typename R>
int build_tables(nfft_plan_t p) {
  const int Ms = p->Ms, M = p->M, m = p->m;
  const long double b = (long double)p->b;
  std::vector<R> coef;
  p->poly_err = fit_window<R>(m, b, coef);
  const double tol = std::is_same<R, double>::value ? 1e-13 : 1e-7;
  if (!(p->poly_err <= tol))
    return fail(p, NFFT_EUNSUPPORTED, "window polynomial error %.3g exceeds %.1g", p->poly_err, tol);
  TRY(dalloc(p, &p->coef, coef.size() * sizeof(R)));
  HIP_TRY(p, hipMemcpy(p->coef, coef.data(), coef.size() * sizeof(R), hipMemcpyHostToDevice));
  // deconvolution factors of D (2.13), float64 for both precisions: the
  // float32 path multiplies in float64 and rounds once
  std::vector<double> fac(M);
  for (int kidx = 0; kidx < M; ++kidx) {
    const int k = kidx - M / 2;
    const long double a = 2.0L * 3.14159265358979323846264338327950288L * k / Ms;
    // at sigma = 1 and k = -M/2 the radicand is zero up to rounding (b = pi
    // was formed in double precision): clamp it
    const long double arg = (long double)m * std::sqrt(std::max(b * b - a * a, 0.0L));
    const long double val = std::exp(b * m) /
                            (3.14159265358979323846264338327950288L * bessel_i0(arg));
    fac[kidx] = (double)((k % 2 == 0) ? val : -val);
  }
  std::vector<cplx<R>> tw(Ms);
  for (int q = 0; q < Ms; ++q) {
    const long double ang = 2.0L * 3.14159265358979323846264338327950288L * q / Ms;
    tw[q].x = (R)std::cos(ang);
    tw[q].y = (R)(-std::sin(ang));
  }
  TRY(dalloc(p, &p->fac, M * sizeof(double)));
  TRY(dalloc(p, &p->tw, Ms * sizeof(cplx<R>)));
  HIP_TRY(p, hipMemcpy(p->fac, fac.data(), M * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(p, hipMemcpy(p->tw, tw.data(), Ms * sizeof(cplx<R>), hipMemcpyHostToDevice));
  return NFFT_OK;
}

// Per-handle workspace for max_rhs right-hand sides: tile and item partials,
// FFT buffers and the forward grid.
int ensure_gather_part(nfft_plan_t p);

template <typename R>
int alloc_workspace(nfft_plan_t p, hipStream_t s) {
  const Geom& g = p->g;
  const int d = p->d;
  const int64_t R_ = p->max_rhs;
  const size_t tile_bytes = (size_t)R_ * g.nbins * g.Ptot * sizeof(cplx<R>);
  TRY(dalloc(p, &p->tilep, tile_bytes, false));
  // tiles without nodes are never written: their partials stay zero
  HIP_TRY(p, hipMemsetAsync(p->tilep, 0, tile_bytes, s));
  TRY(dalloc(p, &p->itemp, (size_t)R_ * std::max(1, p->nslots) * g.Ptot * sizeof(cplx<R>), false));
  const int64_t Ms = p->Ms, M = p->M;
  if (d >= 2) TRY(dalloc(p, &p->bufA, (size_t)R_ * ipow(Ms, d - 1) * M * sizeof(cplx<R>), false));
  if (d == 3) TRY(dalloc(p, &p->bufB, (size_t)R_ * Ms * M * M * sizeof(cplx<R>), false));
  TRY(dalloc(p, &p->grid, (size_t)R_ * ipow(Ms, d) * sizeof(cplx<R>), false));
  p->gpart = p->gft = nullptr;
  TRY(ensure_gather_part(p));  // a clone of a plan with the gather tables
  return NFFT_OK;
}

// Window factor table of spread mode 3 (d = 2): computed once per node set
// and shared by clones; 2 * 2m reals per node.
template <typename R>
int ensure_psi(nfft_plan_t p, hipStream_t s) {
  if (p->d != 2 || p->shared->psi) return NFFT_OK;
  R* q = nullptr;
  TRY(dalloc(p, &q, (size_t)p->N * 4 * p->m * sizeof(R)));
  HIP_TRY(p, nfft::launch_psi<R>((const R*)p->frac, p->N, p->m, (const R*)p->coef, q, s));
  p->shared->psi = q;
  return NFFT_OK;
}

// Free the factor table (nothing may still read it).
void drop_psi(nfft_plan_t p) {
  SharedData& sd = *p->shared;
  if (!sd.psi) return;
  auto it = std::find(sd.allocs.begin(), sd.allocs.end(), sd.psi);
  if (it != sd.allocs.end()) sd.allocs.erase(it);
  sd.bytes -= (int64_t)((size_t)p->N * 4 * p->m * (p->prec == NFFT_F64 ? 8 : 4));
  (void)hipFree(sd.psi);
  sd.psi = nullptr;
}

// Spread modes that read the window factor table.
bool uses_psi(int mode) { return mode == 3; }

int ensure_psi_any(nfft_plan_t p, hipStream_t s) {
  return p->prec == NFFT_F64 ? ensure_psi<double>(p, s) : ensure_psi<float>(p, s);
}

bool gather_supported(nfft_plan_t p) {
  return nfft::spread_gather_supported(p->d, p->g.T, p->prec == NFFT_F64, p->m);
}

// Samples of spread mode 6 copied node-major: groups of 32 right-hand sides.
size_t gather_ft_bytes(int64_t N, int nrhs) {
  return (size_t)((nrhs + 31) / 32) * 32 * N * sizeof(float2);
}

// This handle's partial slots and node-major samples of spread mode 6
// (max_rhs right-hand sides).
int ensure_gather_part(nfft_plan_t p) {
  const SharedData& sd = *p->shared;
  if (!sd.g_units) return NFFT_OK;
  if (!p->gft) TRY(dalloc(p, &p->gft, gather_ft_bytes(p->N, p->max_rhs), false));
  if (sd.g_nslots == 0 || p->gpart) return NFFT_OK;
  return dalloc(p, &p->gpart, (size_t)p->max_rhs * sd.g_nslots * 256 * sizeof(float2), false);
}

// Spread mode 6 tables, built once per node set from the sorted cell words:
// for every tile the nodes of the 3 x 3 tiles around it whose closed window
// support reaches it, with the footprint origin relative to the tile, sorted
// by the footprint's column offset (source tiles in row order and nodes in
// tile order within one offset); the units cut each tile's list into runs
// of at most item_nodes entries.
int ensure_gather(nfft_plan_t p, hipStream_t s) {
  if (!gather_supported(p)) return NFFT_OK;
  SharedData& sd = *p->shared;
  if (!sd.g_units) {
    const Geom& g = p->g;
    const int64_t N = p->N;
    const int nb = g.nb, m = p->m, ntiles = g.nbins;
    std::vector<uint32_t> hloc(N);
    std::vector<int32_t> hperm(N), hiperm(N);
    HIP_TRY(p, hipMemcpyAsync(hloc.data(), p->loc, N * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(p, hipMemcpyAsync(hperm.data(), p->perm, N * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(p, hipStreamSynchronize(s));
    for (int64_t i = 0; i < N; ++i) hiperm[hperm[i]] = (int32_t)i;
    const std::vector<int32_t>& bs = sd.hbin_start;
    std::vector<int64_t> start(ntiles + 1, 0);
    std::vector<int32_t> node, hdr;
    for (int pass = 0; pass < 2; ++pass) {
      if (pass) {
        node.resize(start[ntiles]);
        hdr.resize(start[ntiles]);
      }
      for (int t = 0; t < ntiles; ++t) {
        const int t0 = t / nb, t1 = t % nb;
        int64_t pos = pass ? start[t] : 0;
        for (int ds0 = -1; ds0 <= 1; ++ds0)
          for (int ds1 = -1; ds1 <= 1; ++ds1) {
            const int S = ((t0 + ds0 + nb) % nb) * nb + (t1 + ds1 + nb) % nb;
            for (int32_t i = bs[S]; i < bs[S + 1]; ++i) {
              const uint32_t L = hloc[i];
              const int b0 = 16 * ds0 - m + (int)(L & nfft::kLocMask);
              const int b1 = 16 * ds1 - m + (int)((L >> nfft::kLocBits) & nfft::kLocMask);
              const int e0 = (int)((L >> nfft::kEdgeShift) & 1u);
              const int e1 = (int)((L >> (nfft::kEdgeShift + 1)) & 1u);
              if (b0 + (1 - e0) > 15 || b0 + 2 * m < 0 || b1 + (1 - e1) > 15 || b1 + 2 * m < 0)
                continue;
              if (pass) {
                node[pos] = i;
                hdr[pos] = (b0 + 64) | ((b1 + 64) << 8) | (e0 << 16) | (e1 << 17);
              }
              ++pos;
            }
          }
        if (!pass) {
          start[t + 1] = start[t] + pos;
          continue;
        }
        // by the column offset of the footprint (bits 8-15), in source and
        // node order within one offset: the kernel takes each offset in turn
        std::vector<int64_t> ix(start[t + 1] - start[t]);
        std::iota(ix.begin(), ix.end(), start[t]);
        std::stable_sort(ix.begin(), ix.end(), [&](int64_t u, int64_t v) {
          return ((hdr[u] >> 8) & 0xff) < ((hdr[v] >> 8) & 0xff);
        });
        std::vector<int32_t> tn(ix.size()), th(ix.size());
        for (size_t q = 0; q < ix.size(); ++q) {
          tn[q] = node[ix[q]];
          th[q] = hdr[ix[q]];
        }
        std::copy(tn.begin(), tn.end(), node.begin() + start[t]);
        std::copy(th.begin(), th.end(), hdr.begin() + start[t]);
      }
    }
    if (start[ntiles] > INT32_MAX)
      return fail(p, NFFT_EUNSUPPORTED, "spread mode 6: %lld list entries exceed int32",
                  (long long)start[ntiles]);
    const int C = p->tune[NFFT_TUNE_ITEM_NODES];
    std::vector<int32_t> units, split;
    int nslots = 0;
    for (int t = 0; t < ntiles; ++t) {
      const int64_t n = start[t + 1] - start[t];
      const int64_t k = std::max<int64_t>(1, (n + C - 1) / C);
      if (k > 1) split.insert(split.end(), {t, nslots, (int32_t)k, 0});
      for (int64_t j = 0; j < k; ++j)
        units.insert(units.end(), {t, (int32_t)(start[t] + j * n / k),
                                   (int32_t)(start[t] + (j + 1) * n / k),
                                   k > 1 ? nslots++ : -1});
    }
    // launch order: longest units first (the crowded tiles' units start
    // before the many short ones that fill in behind them)
    const int nu = (int)(units.size() / 4), n8 = (nu + 7) / 8;
    std::vector<int> byLen(nu);
    std::iota(byLen.begin(), byLen.end(), 0);
    std::stable_sort(byLen.begin(), byLen.end(), [&](int x, int y) {
      return units[4 * x + 2] - units[4 * x + 1] > units[4 * y + 2] - units[4 * y + 1];
    });
    std::vector<int32_t> order(4 * 8 * (size_t)n8, -1);
    for (int u = 0; u < nu; ++u)
      std::copy(units.begin() + 4 * byLen[u], units.begin() + 4 * byLen[u] + 4,
                order.begin() + 4 * u);
    const size_t ne = std::max<size_t>(1, node.size());
    const int64_t bytes0 = sd.bytes;
    TRY(dalloc(p, &sd.gl_node, ne * sizeof(int32_t)));
    TRY(dalloc(p, &sd.gl_hdr, ne * sizeof(int32_t)));
    TRY(dalloc(p, &sd.g_units, order.size() * sizeof(int32_t)));
    TRY(dalloc(p, &sd.g_split, std::max<size_t>(4, split.size()) * sizeof(int32_t)));
    TRY(dalloc(p, &sd.g_iperm, std::max<int64_t>(1, N) * sizeof(int32_t)));
    if (N > 0)
      HIP_TRY(p, hipMemcpyAsync(sd.g_iperm, hiperm.data(), N * 4, hipMemcpyHostToDevice, s));
    if (!node.empty()) {
      HIP_TRY(p, hipMemcpyAsync(sd.gl_node, node.data(), node.size() * 4, hipMemcpyHostToDevice, s));
      HIP_TRY(p, hipMemcpyAsync(sd.gl_hdr, hdr.data(), hdr.size() * 4, hipMemcpyHostToDevice, s));
    }
    HIP_TRY(p, hipMemcpyAsync(sd.g_units, order.data(), order.size() * 4, hipMemcpyHostToDevice, s));
    if (!split.empty())
      HIP_TRY(p, hipMemcpyAsync(sd.g_split, split.data(), split.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(p, hipStreamSynchronize(s));  // the host vectors go out of scope
    sd.g_nunits = 8 * n8;
    sd.g_nsplit = (int)(split.size() / 4);
    sd.g_nslots = nslots;
    sd.g_bytes = sd.bytes - bytes0;
  }
  return ensure_gather_part(p);
}

// Free the mode 6 tables and this handle's partials (nothing may still read
// them; the handle must be the only one referring to the tables).
void drop_gather(nfft_plan_t p) {
  SharedData& sd = *p->shared;
  auto release = [](std::vector<void*>& v, void* q) {
    auto it = std::find(v.begin(), v.end(), q);
    if (it != v.end()) v.erase(it);
    (void)hipFree(q);
  };
  if (p->gpart) {
    release(p->allocs, p->gpart);
    p->bytes -= (int64_t)((size_t)p->max_rhs * sd.g_nslots * 256 * sizeof(float2));
    p->gpart = nullptr;
  }
  if (p->gft) {
    release(p->allocs, p->gft);
    p->bytes -= (int64_t)gather_ft_bytes(p->N, p->max_rhs);
    p->gft = nullptr;
  }
  if (!sd.g_units) return;
  for (void* q : {(void*)sd.gl_node, (void*)sd.gl_hdr, (void*)sd.g_units, (void*)sd.g_split,
                 (void*)sd.g_iperm})
    release(sd.allocs, q);
  sd.bytes -= sd.g_bytes;
  sd.gl_node = sd.gl_hdr = sd.g_units = sd.g_split = sd.g_iperm = nullptr;
  sd.g_nunits = sd.g_nsplit = sd.g_nslots = 0;
  sd.g_bytes = 0;
}

template <typename R>
int build_plan(nfft_plan_t p, const double* nodes, hipStream_t s) {
  const int64_t N = p->N;
  const int d = p->d;
  Geom& g = p->g;
  ScopedFree tmp;
  auto talloc = [&](void** q, size_t bytes) -> int {
    hipError_t e = hipMalloc(q, bytes ? bytes : 16);
    if (e != hipSuccess)
      return fail(p, e == hipErrorOutOfMemory ? NFFT_ENOMEM : NFFT_EDEVICE,
                  "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    tmp.ptrs.push_back(*q);
    return NFFT_OK;
  };
  void *d_nodes, *bin, *loc_u, *frac_u, *err, *counts, *rank, *chunk_count, *offsets, *bstart;
  const int64_t nchunks = (N + nfft::kRankChunk - 1) / nfft::kRankChunk;
  TRY(talloc(&d_nodes, N * d * sizeof(double)));
  TRY(talloc(&bin, N * sizeof(int32_t)));
  TRY(talloc(&loc_u, N * sizeof(uint32_t)));
  TRY(talloc(&frac_u, N * d * sizeof(double)));
  TRY(talloc(&err, sizeof(int)));
  TRY(talloc(&counts, g.nbins * sizeof(int32_t)));
  TRY(talloc(&rank, N * sizeof(int32_t)));
  TRY(talloc(&chunk_count, (size_t)nchunks * g.nbins * sizeof(int32_t)));
  TRY(talloc(&offsets, (size_t)nchunks * g.nbins * sizeof(int32_t)));
  TRY(talloc(&bstart, (g.nbins + 1) * sizeof(int32_t)));

  HIP_TRY(p, hipMemcpyAsync(d_nodes, nodes, N * d * sizeof(double), hipMemcpyDefault, s));
  HIP_TRY(p, hipMemsetAsync(err, 0, sizeof(int), s));
  HIP_TRY(p, hipMemsetAsync(counts, 0, g.nbins * sizeof(int32_t), s));
  HIP_TRY(p, hipMemsetAsync(chunk_count, 0, (size_t)nchunks * g.nbins * sizeof(int32_t), s));
  HIP_TRY(p, nfft::launch_encode((const double*)d_nodes, N, g, (int32_t*)bin, (uint32_t*)loc_u,
                                 (double*)frac_u, (int*)err, s));
  HIP_TRY(p, nfft::launch_count((const int32_t*)bin, N, (int32_t*)counts, s));
  std::vector<int32_t> hc(g.nbins);
  int herr = 0;
  HIP_TRY(p, hipMemcpyAsync(hc.data(), counts, g.nbins * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(p, hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(p, hipStreamSynchronize(s));
  if (herr) return fail(p, NFFT_EINVAL, "nodes contain a non-finite coordinate");

  // tile starts and work items (at most kItem nodes of one tile each)
  std::vector<int32_t> hstart(g.nbins + 1);
  std::vector<int32_t> istart, icount, ibin, ifirst(g.nbins + 1);  // ifirst: items of tile b
  const int kItem = p->tune[NFFT_TUNE_ITEM_NODES];
  int64_t acc = 0;
  p->maxpop = 0;
  for (int b = 0; b < g.nbins; ++b) {
    hstart[b] = (int32_t)acc;
    ifirst[b] = (int32_t)istart.size();
    p->maxpop = std::max(p->maxpop, hc[b]);
    for (int k = 0; k < hc[b]; k += kItem) {
      istart.push_back((int32_t)(acc + k));
      icount.push_back(std::min(kItem, hc[b] - k));
      ibin.push_back(b);
    }
    acc += hc[b];
  }
  hstart[g.nbins] = (int32_t)acc;
  ifirst[g.nbins] = (int32_t)istart.size();
  // split tiles: their items write to their own slots and are summed later
  std::vector<int32_t> islot(istart.size(), -1), mbin, mfirst;
  for (int b = 0; b < g.nbins; ++b) {
    const int n = ifirst[b + 1] - ifirst[b];
    if (n <= 1) continue;
    mbin.push_back(b);
    mfirst.push_back(p->nslots);
    for (int k = 0; k < n; ++k) islot[ifirst[b] + k] = p->nslots++;
  }
  mfirst.push_back(p->nslots);
  p->nmulti = (int)mbin.size();
  std::vector<int32_t> ebins;
  for (int b = 0; b < g.nbins; ++b)
    if (hc[b] == 0) ebins.push_back(b);
  p->nempty = (int)ebins.size();
  g.nsub = (int)istart.size();
  // launch order: largest work items first, so that the work-groups that
  // start last are the small remainders of tiles, in blocks of one item per
  // compute unit whose direction alternates: the first work-groups go one
  // to each compute unit, so that unit c receives the items of rank c,
  // 2C - 1 - c, 2C + c, ... (C compute units), large ones paired with small
  // ones (every item writes its own tile or slot, so the order changes no
  // result)
  {
    std::vector<int32_t> order(istart.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t u, int32_t v) { return icount[u] > icount[v]; });
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess ||
        ncu < 1)
      ncu = 256;
    const size_t C = (size_t)ncu;
    for (size_t b0 = C; b0 < order.size(); b0 += 2 * C)
      std::reverse(order.begin() + b0, order.begin() + std::min(order.size(), b0 + C));
    auto permute = [&](std::vector<int32_t>& a) {
      std::vector<int32_t> t(a.size());
      for (size_t i = 0; i < a.size(); ++i) t[i] = a[order[i]];
      a.swap(t);
    };
    permute(istart);
    permute(icount);
    permute(ibin);
    permute(islot);
  }
  HIP_TRY(p, hipMemcpyAsync(bstart, hstart.data(), (g.nbins + 1) * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
  p->shared->hbin_start = hstart;

  HIP_TRY(p, nfft::launch_rank((const int32_t*)bin, N, g.nbins, (int32_t*)rank,
                               (int32_t*)chunk_count, s));
  HIP_TRY(p, nfft::launch_chunk_offsets((const int32_t*)chunk_count, (const int32_t*)bstart,
                                        nchunks, g.nbins, (int32_t*)offsets, s));
  TRY(dalloc(p, &p->perm, N * sizeof(int32_t)));
  TRY(dalloc(p, &p->loc, N * sizeof(uint32_t)));
  TRY(dalloc(p, &p->frac, N * d * sizeof(R)));
  HIP_TRY(p, nfft::launch_scatter<R>((const int32_t*)bin, (const int32_t*)rank,
                                     (const int32_t*)offsets, (const uint32_t*)loc_u,
                                     (const double*)frac_u, N, d, g.nbins, p->perm, p->loc,
                                     (R*)p->frac, s));
  if (d >= 2) {
    // within each tile, nodes ordered by their dimension-0 cell (the register
    // row sweeps and the matrix-core tiles consume them row by row)
    void *perm2, *loc2, *frac2;
    TRY(talloc(&perm2, N * sizeof(int32_t)));
    TRY(talloc(&loc2, N * sizeof(uint32_t)));
    TRY(talloc(&frac2, N * d * sizeof(R)));
    HIP_TRY(p, nfft::launch_row_sort<R>((const int32_t*)bstart, g.nbins, g.T, N, d, p->perm,
                                        p->loc, (const R*)p->frac, (int32_t*)perm2,
                                        (uint32_t*)loc2, (R*)frac2, s));
    HIP_TRY(p, hipMemcpyAsync(p->perm, perm2, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIP_TRY(p, hipMemcpyAsync(p->loc, loc2, N * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    HIP_TRY(p, hipMemcpyAsync(p->frac, frac2, N * d * sizeof(R), hipMemcpyDeviceToDevice, s));
  }

  const size_t ni = std::max<size_t>(1, istart.size());
  TRY(dalloc(p, &p->item_start, ni * sizeof(int32_t)));
  TRY(dalloc(p, &p->item_count, ni * sizeof(int32_t)));
  TRY(dalloc(p, &p->item_bin, ni * sizeof(int32_t)));
  if (!istart.empty()) {
    HIP_TRY(p, hipMemcpyAsync(p->item_start, istart.data(), istart.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(p, hipMemcpyAsync(p->item_count, icount.data(), icount.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(p, hipMemcpyAsync(p->item_bin, ibin.data(), ibin.size() * 4, hipMemcpyHostToDevice, s));
  }
  TRY(dalloc(p, &p->item_slot, ni * sizeof(int32_t)));
  TRY(dalloc(p, &p->multi_bin, std::max<size_t>(1, mbin.size()) * sizeof(int32_t)));
  TRY(dalloc(p, &p->multi_first, mfirst.size() * sizeof(int32_t)));
  if (!islot.empty())
    HIP_TRY(p, hipMemcpyAsync(p->item_slot, islot.data(), islot.size() * 4, hipMemcpyHostToDevice, s));
  if (!mbin.empty())
    HIP_TRY(p, hipMemcpyAsync(p->multi_bin, mbin.data(), mbin.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(p, hipMemcpyAsync(p->multi_first, mfirst.data(), mfirst.size() * 4, hipMemcpyHostToDevice, s));
  TRY(dalloc(p, &p->empty_bins, std::max<size_t>(1, ebins.size()) * sizeof(int32_t)));
  if (!ebins.empty())
    HIP_TRY(p, hipMemcpyAsync(p->empty_bins, ebins.data(), ebins.size() * 4, hipMemcpyHostToDevice, s));

  TRY(dalloc(p, &p->w, N * sizeof(cplx<R>)));
  TRY(alloc_workspace<R>(p, s));
  TRY(build_tables<R>(p));
  if (uses_psi(p->tune[NFFT_TUNE_SPREAD_MODE])) TRY(ensure_psi<R>(p, s));
  if (p->tune[NFFT_TUNE_SPREAD_MODE] == 6) TRY(ensure_gather(p, s));
  HIP_TRY(p, hipStreamSynchronize(s));
  return NFFT_OK;
}

template <typename R>
nfft::FftArgs<R> fft_args(nfft_plan_t p, int64_t nlines, const void* in, int64_t in_bs, int Lin,
                          void* out, int64_t out_bs) {
  nfft::FftArgs<R> a{};
  a.nlines = nlines;
  a.in = (const cplx<R>*)in;
  a.in_bs = in_bs;
  a.Lin = Lin;
  a.out = (cplx<R>*)out;
  a.out_bs = out_bs;
  a.tw = (const cplx<R>*)p->tw;
  a.fac = (const double*)p->fac;
  a.g = p->g;
  a.tilep = (const cplx<R>*)p->tilep;
  a.tile_bs = (int64_t)p->g.nbins * p->g.Ptot;
  a.min_wg = p->tune[NFFT_TUNE_FFT_MIN_WG];
  return a;
}

void record(nfft_plan_t p, StageEvents& se, hipStream_t s) {
  if (!p->profiling) return;
  hipEvent_t e;
  if (!p->event_pool.empty()) {
    e = p->event_pool.back();
    p->event_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return;
  }
  (void)hipEventRecord(e, s);
  se.ev[se.n++] = e;
}

// Intermediate buffers of one adjoint: tile partials, item partials of split
// tiles, FFT buffers, and the grid and unit partials of spread mode 6.
struct Work {
  void* tilep;
  void* itemp;
  void* bufA;
  void* bufB;
  void* grid;
  void* gpart;
  void* gft;
};

// With accumulate, the last FFT pass adds its outputs to fhat instead of
// writing them (fhat += A^* W f). With wk, the intermediate buffers are wk's
// instead of the plan's workspace (no stage events are recorded then).
template <typename R>
int run_adjoint(nfft_plan_t p, const void* f, void* fhat, int nrhs, hipStream_t s,
                bool accumulate = false, const Work* wk = nullptr) {
  const Geom& g = p->g;
  const int64_t Ms = p->Ms, M = p->M;
  const Work own{p->tilep, p->itemp, p->bufA, p->bufB, p->grid, p->gpart, p->gft};
  const Work& w = wk ? *wk : own;
  const bool prof = p->profiling && !wk;
  StageEvents se{};
  se.kind = 0;
  if (prof) record(p, se, s);
  nfft::SpreadArgs<R> sa{};
  sa.loc = p->loc;
  sa.frac = (const R*)p->frac;
  sa.w = (const cplx<R>*)p->w;
  sa.perm = p->perm;
  sa.f = (const cplx<R>*)f;
  sa.tilep = (cplx<R>*)w.tilep;
  sa.itemp = (cplx<R>*)w.itemp;
  sa.item_start = p->item_start;
  sa.item_count = p->item_count;
  sa.item_bin = p->item_bin;
  sa.item_slot = p->item_slot;
  sa.coef = (const R*)p->coef;
  sa.f_rs = p->N;
  sa.tile_rs = (int64_t)g.nbins * g.Ptot;
  sa.item_rs = (int64_t)std::max(1, p->nslots) * g.Ptot;
  sa.edge = (R)(p->b * std::exp(-p->b * p->m));
  sa.g = g;
  sa.nt = p->tune[NFFT_TUNE_SPREAD_THREADS];
  sa.nr = nrhs > 1 ? p->tune[NFFT_TUNE_RHS_PER_GROUP] : 1;
  sa.planes = p->tune[NFFT_TUNE_SPREAD_PLANES];
  sa.mode = p->tune[NFFT_TUNE_SPREAD_MODE];
  sa.psi = uses_psi(sa.mode) ? (const R*)p->shared->psi : nullptr;
  if constexpr (std::is_same<R, float>::value) {
    if (sa.mode == 6) {
      // the grid of every right-hand side from the per-tile lists; the
      // partials of the tiles cut into several units are summed into it (the
      // split-tile stage), and the first FFT pass reads plain lines
      const SharedData& sd = *p->shared;
      if (!sd.g_units || (sd.g_nslots > 0 && !w.gpart) || !w.gft)
        return fail(p, NFFT_ESTATE, "spread mode 6 tables are missing");
      nfft::GatherArgs ga{};
      ga.units = sd.g_units;
      ga.nunits = sd.g_nunits;
      ga.gl_node = sd.gl_node;
      ga.gl_hdr = sd.gl_hdr;
      ga.iperm = sd.g_iperm;
      ga.split = sd.g_split;
      ga.nsplit = sd.g_nsplit;
      ga.grid = (float2*)w.grid;
      ga.grid_rs = Ms * Ms;
      ga.part = (float2*)w.gpart;
      ga.part_rs = (int64_t)sd.g_nslots * 256;
      ga.fT = (float2*)w.gft;
      HIP_TRY(p, nfft::launch_spread_gather(sa, ga, nrhs, s));
      if (prof) record(p, se, s);
      HIP_TRY(p, nfft::launch_gather_reduce(ga, g.nb, (int)Ms, nrhs, s));
      if (prof) record(p, se, s);
      const int L = (int)Ms;
      auto a = fft_args<R>(p, Ms, w.grid, Ms * Ms, L, w.bufA, M * Ms);
      HIP_TRY(p, nfft::launch_fft_pass<R>(a, L, false, nfft::kLoadLine, nfft::kStoreCropScaled,
                                          nrhs, s));
      if (prof) record(p, se, s);
      auto c = fft_args<R>(p, M, w.bufA, M * Ms, L, fhat, M * M);
      c.accumulate = accumulate;
      HIP_TRY(p, nfft::launch_fft_pass<R>(c, L, false, nfft::kLoadLine, nfft::kStoreCropScaled,
                                          nrhs, s));
      if (prof) record(p, se, s);
      if (prof && se.n > 0) p->pending.push_back(se);
      return NFFT_OK;
    }
  }
  HIP_TRY(p, nfft::launch_spread<R>(sa, nrhs, s));
  if (prof) record(p, se, s);
  nfft::ReduceArgs<R> ra{};
  ra.tilep = (cplx<R>*)w.tilep;
  ra.itemp = (const cplx<R>*)w.itemp;
  ra.multi_bin = p->multi_bin;
  ra.multi_first = p->multi_first;
  ra.nmulti = p->nmulti;
  ra.tile_rs = sa.tile_rs;
  ra.item_rs = sa.item_rs;
  ra.g = g;
  HIP_TRY(p, nfft::launch_tile_reduce<R>(ra, nrhs, s));
  if (prof) record(p, se, s);

  const int L = (int)Ms;
  const auto fwd = nfft::kLoadMerge;
  if (p->d == 1) {
    auto a = fft_args<R>(p, 1, nullptr, 0, L, fhat, M);
    a.tilep = (const cplx<R>*)w.tilep;
    a.accumulate = accumulate;
    HIP_TRY(p, nfft::launch_fft_pass<R>(a, L, false, fwd, nfft::kStoreCropScaled, nrhs, s));
    if (prof) record(p, se, s);
  } else if (p->d == 2) {
    // [s1][s2] -> [k2][s1] -> [k1][k2]
    auto a = fft_args<R>(p, Ms, nullptr, 0, L, w.bufA, M * Ms);
    a.tilep = (const cplx<R>*)w.tilep;
    HIP_TRY(p, nfft::launch_fft_pass<R>(a, L, false, fwd, nfft::kStoreCropScaled, nrhs, s));
    if (prof) record(p, se, s);
    auto c = fft_args<R>(p, M, w.bufA, M * Ms, L, fhat, M * M);
    c.accumulate = accumulate;
    HIP_TRY(p, nfft::launch_fft_pass<R>(c, L, false, nfft::kLoadLine, nfft::kStoreCropScaled, nrhs, s));
  } else {
    // [s1][s2][s3] -> [k3][s1][s2] -> [k2][k3][s1] -> [k1][k2][k3]
    auto a = fft_args<R>(p, Ms * Ms, nullptr, 0, L, w.bufA, M * Ms * Ms);
    a.tilep = (const cplx<R>*)w.tilep;
    HIP_TRY(p, nfft::launch_fft_pass<R>(a, L, false, fwd, nfft::kStoreCropScaled, nrhs, s));
    if (prof) record(p, se, s);
    auto c = fft_args<R>(p, M * Ms, w.bufA, M * Ms * Ms, L, w.bufB, M * M * Ms);
    HIP_TRY(p, nfft::launch_fft_pass<R>(c, L, false, nfft::kLoadLine, nfft::kStoreCropScaled, nrhs, s));
    auto e = fft_args<R>(p, M * M, w.bufB, M * M * Ms, L, fhat, M * M * M);
    e.accumulate = accumulate;
    HIP_TRY(p, nfft::launch_fft_pass<R>(e, L, false, nfft::kLoadLine, nfft::kStoreCropScaled, nrhs, s));
  }
  if (prof) record(p, se, s);
  if (prof && se.n > 0) p->pending.push_back(se);
  return NFFT_OK;
}

// Algorithm 4.4 step 1: h_opt = D^* F^* B_opt^* f. The grid of B_opt^* f is
// formed by columns (no tiles), then the FFT passes of the adjoint NFFT run
// with their first pass reading that grid.
template <typename R>
int run_bopt_adjoint(nfft_plan_t p, const void* f, void* fhat, int nrhs, hipStream_t s) {
  const int64_t Ms = p->Ms, M = p->M;
  const int64_t ncols = ipow(Ms, p->d);
  SharedData& sd = *p->shared;
  // the deconvolution table divides by the window scaled by pi e^{-b m} in
  // every dimension
  const double scale = std::pow(M_PI * std::exp(-p->b * p->m), p->d);
  StageEvents se{};
  se.kind = 2;
  record(p, se, s);
  HIP_TRY(p, nfft::launch_bopt_apply<R>(sd.bopt_ptr, sd.bopt_node, (const R*)sd.bopt_val,
                                        (const cplx<R>*)f, p->N, (cplx<R>*)p->grid, ncols,
                                        ncols, nrhs, scale, sd.bopt_lanes, s));
  record(p, se, s);
  const int L = (int)Ms;
  const auto ld = nfft::kLoadLine;
  const auto st = nfft::kStoreCropScaled;
  if (p->d == 1) {
    auto a = fft_args<R>(p, 1, p->grid, Ms, L, fhat, M);
    HIP_TRY(p, nfft::launch_fft_pass<R>(a, L, false, ld, st, nrhs, s));
  } else if (p->d == 2) {
    auto a = fft_args<R>(p, Ms, p->grid, Ms * Ms, L, p->bufA, M * Ms);
    HIP_TRY(p, nfft::launch_fft_pass<R>(a, L, false, ld, st, nrhs, s));
    auto c = fft_args<R>(p, M, p->bufA, M * Ms, L, fhat, M * M);
    HIP_TRY(p, nfft::launch_fft_pass<R>(c, L, false, ld, st, nrhs, s));
  } else {
    auto a = fft_args<R>(p, Ms * Ms, p->grid, Ms * Ms * Ms, L, p->bufA, M * Ms * Ms);
    HIP_TRY(p, nfft::launch_fft_pass<R>(a, L, false, ld, st, nrhs, s));
    auto c = fft_args<R>(p, M * Ms, p->bufA, M * Ms * Ms, L, p->bufB, M * M * Ms);
    HIP_TRY(p, nfft::launch_fft_pass<R>(c, L, false, ld, st, nrhs, s));
    auto e = fft_args<R>(p, M * M, p->bufB, M * M * Ms, L, fhat, M * M * M);
    HIP_TRY(p, nfft::launch_fft_pass<R>(e, L, false, ld, st, nrhs, s));
  }
  record(p, se, s);
  if (p->profiling && se.n > 0) p->pending.push_back(se);
  return NFFT_OK;
}

// Algorithm 2.1 steps 1 and 2: deconvolution and zero padding of fhat, then
// the inverse FFT passes, into the plan's grid ([s_1]...[s_d], C order).
template <typename R>
int forward_grid(nfft_plan_t p, const void* fhat, int nrhs, hipStream_t s) {
  const int64_t Ms = p->Ms, M = p->M;
  const int L = (int)Ms;
  const auto ld = nfft::kLoadPadScaled;
  const auto st = nfft::kStoreFull;
  if (p->d == 1) {
    auto a = fft_args<R>(p, 1, fhat, M, (int)M, p->grid, Ms);
    HIP_TRY(p, nfft::launch_fft_pass<R>(a, L, true, ld, st, nrhs, s));
  } else if (p->d == 2) {
    // [k1][k2] -> [s2][k1] -> [s1][s2]
    auto a = fft_args<R>(p, M, fhat, M * M, (int)M, p->bufA, Ms * M);
    HIP_TRY(p, nfft::launch_fft_pass<R>(a, L, true, ld, st, nrhs, s));
    auto c = fft_args<R>(p, Ms, p->bufA, Ms * M, (int)M, p->grid, Ms * Ms);
    HIP_TRY(p, nfft::launch_fft_pass<R>(c, L, true, ld, st, nrhs, s));
  } else {
    // [k1][k2][k3] -> [s3][k1][k2] -> [s2][s3][k1] -> [s1][s2][s3]
    auto a = fft_args<R>(p, M * M, fhat, M * M * M, (int)M, p->bufB, Ms * M * M);
    HIP_TRY(p, nfft::launch_fft_pass<R>(a, L, true, ld, st, nrhs, s));
    auto c = fft_args<R>(p, Ms * M, p->bufB, Ms * M * M, (int)M, p->bufA, Ms * Ms * M);
    HIP_TRY(p, nfft::launch_fft_pass<R>(c, L, true, ld, st, nrhs, s));
    auto e = fft_args<R>(p, Ms * Ms, p->bufA, Ms * Ms * M, (int)M, p->grid, Ms * Ms * Ms);
    HIP_TRY(p, nfft::launch_fft_pass<R>(e, L, true, ld, st, nrhs, s));
  }
  return NFFT_OK;
}

// Remark 4.6: f = B_opt F D h, the forward's grid gathered with the stored
// values of B_opt instead of window evaluations.
template <typename R>
int run_bopt_inverse_adjoint(nfft_plan_t p, const void* h, void* f, int nrhs, hipStream_t s) {
  TRY(forward_grid<R>(p, h, nrhs, s));
  const SharedData& sd = *p->shared;
  const double scale = std::pow(M_PI * std::exp(-p->b * p->m), p->d);
  HIP_TRY(p, nfft::launch_bopt_gather<R>(sd.bopt_lo, (const R*)sd.bopt_rows,
                                         (const cplx<R>*)p->grid, ipow(p->Ms, p->d), p->N, p->d,
                                         p->Ms, p->m, (cplx<R>*)f, p->N, nrhs, scale, s));
  return NFFT_OK;
}

// With sub, the samples written are sub - A fhat (sub in the layout of f).
template <typename R>
int run_forward(nfft_plan_t p, const void* fhat, void* f, int nrhs, hipStream_t s,
                const void* sub = nullptr) {
  const Geom& g = p->g;
  const int64_t Ms = p->Ms;
  StageEvents se{};
  se.kind = 1;
  record(p, se, s);
  TRY(forward_grid<R>(p, fhat, nrhs, s));
  record(p, se, s);
  nfft::InterpArgs<R> ia{};
  ia.loc = p->loc;
  ia.frac = (const R*)p->frac;
  ia.perm = p->perm;
  ia.grid = (const cplx<R>*)p->grid;
  ia.f = (cplx<R>*)f;
  ia.sub = (const cplx<R>*)sub;
  ia.item_start = p->item_start;
  ia.item_count = p->item_count;
  ia.item_bin = p->item_bin;
  ia.coef = (const R*)p->coef;
  // the window factor table, where the plan has one (same values as the
  // polynomials), saves the per-call evaluation
  ia.psi = p->d == 2 ? (const R*)p->shared->psi : nullptr;
  ia.grid_rs = ipow(Ms, p->d);
  ia.f_rs = p->N;
  ia.edge = (R)(p->b * std::exp(-p->b * p->m));
  ia.g = g;
  HIP_TRY(p, nfft::launch_interp<R>(ia, nrhs, s));
  record(p, se, s);
  if (p->profiling && se.n > 0) p->pending.push_back(se);
  return NFFT_OK;
}

// Weighted iterative refinement: fhat_0 = A^* W f (Algorithm 3.7), then
// fhat_{k+1} = fhat_k + A^* W (f - A fhat_k) for k < iters, so that fhat_k is
// the partial sum up to n = k of the Neumann series sum_n (I - A^* W A)^n
// applied to A^* W f (proof of Theorem 3.15); it tends to the weighted
// least-squares solution when ||I - A^* W A||_2 < 1. With res, the squared
// norms of f and of the residuals f - A fhat_k, k = 0..iters, are reduced on
// the device and returned as relative residuals (the call then waits).
constexpr int kMaxRefine = 1000;

template <typename R>
int run_refine(nfft_plan_t p, const void* f, void* fhat, int nrhs, int iters, double* res,
               hipStream_t s) {
  const int64_t nf = (int64_t)nrhs * p->N;
  // each buffer on its first use (a failed allocation leaves the other)
  if (!p->ref_r) TRY(dalloc(p, &p->ref_r, (size_t)p->max_rhs * p->N * sizeof(cplx<R>), false));
  if (!p->ref_red)
    TRY(dalloc(p, &p->ref_red, (nfft::kRefineBlocks + kMaxRefine + 2) * sizeof(double), false));
  cplx<R>* r = (cplx<R>*)p->ref_r;
  double* part = p->ref_red;
  double* norms = part + nfft::kRefineBlocks;  // ||f||^2, then ||r_k||^2
  TRY(run_adjoint<R>(p, f, fhat, nrhs, s));    // fhat_0
  if (res) HIP_TRY(p, nfft::launch_sumsq<R>((const cplx<R>*)f, nf, part, norms, s));
  for (int k = 0; k <= iters; ++k) {
    if (k == iters && !res) break;  // the last residual is only reported
    // r_k = f - A fhat_k, formed where the window sums are written
    TRY(run_forward<R>(p, fhat, r, nrhs, s, f));
    if (res) HIP_TRY(p, nfft::launch_sumsq<R>(r, nf, part, norms + 1 + k, s));
    if (k == iters) break;
    // fhat_{k+1} = fhat_k + A^* W r_k, added where the last FFT pass stores
    TRY(run_adjoint<R>(p, r, fhat, nrhs, s, true));
  }
  if (res) {
    std::vector<double> nv(iters + 2);
    HIP_TRY(p, hipMemcpyAsync(nv.data(), norms, nv.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(p, hipStreamSynchronize(s));
    for (int k = 0; k <= iters; ++k) res[k] = nv[0] > 0 ? std::sqrt(nv[1 + k] / nv[0]) : 0.0;
  }
  return NFFT_OK;
}

// Milliseconds per adjoint of nrhs right-hand sides: two warm-up calls, then
// the better of two rounds of `reps` calls between HIP events.
double time_adjoint(nfft_plan_t p, const void* f, void* fhat, int nrhs, hipStream_t s) {
  constexpr int reps = 5;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0;
  }
  auto call = [&]() {
    return p->prec == NFFT_F64 ? run_adjoint<double>(p, f, fhat, nrhs, s)
                               : run_adjoint<float>(p, f, fhat, nrhs, s);
  };
  double best = -1.0;
  bool ok = call() == NFFT_OK && call() == NFFT_OK;
  for (int round = 0; ok && round < 2; ++round) {
    ok = hipEventRecord(e0, s) == hipSuccess;
    for (int i = 0; ok && i < reps; ++i) ok = call() == NFFT_OK;
    ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    if (ok && (best < 0 || ms / reps < best)) best = ms / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ok ? best : -1.0;
}

// Scratch memory of nfft_adjoint_scratch: a file-scope device array that
// every GPU the library runs on holds until the process ends. In host code
// its name is only a stand-in; its device address (one per GPU) comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of the scratch array on `dev` (looked up on the first call
// for that device, with `dev` current; the caller's current device is
// restored).
int scratch_address(nfft_plan_t p, int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(p, NFFT_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    HIP_TRY(p, hipGetDevice(&cur));
    if (cur != dev) HIP_TRY(p, hipSetDevice(dev));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr)
      return fail(p, NFFT_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return NFFT_OK;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// The adjoint with its intermediate buffers carved out of the scratch array.
template <typename R>
int run_adjoint_scratch(nfft_plan_t p, const void* f, void* fhat, int nrhs, hipStream_t s) {
  const Geom& g = p->g;
  const size_t cb = sizeof(cplx<R>);
  const int64_t Ms = p->Ms, M = p->M;
  const size_t tile = align256((size_t)nrhs * g.nbins * g.Ptot * cb);
  const size_t item = align256((size_t)nrhs * std::max(1, p->nslots) * g.Ptot * cb);
  const size_t bufA = p->d >= 2 ? align256((size_t)nrhs * ipow(Ms, p->d - 1) * M * cb) : 0;
  const size_t bufB = p->d == 3 ? align256((size_t)nrhs * Ms * M * M * cb) : 0;
  const bool gather = p->tune[NFFT_TUNE_SPREAD_MODE] == 6;
  const size_t gpart =
      gather ? align256((size_t)nrhs * p->shared->g_nslots * 256 * sizeof(float2)) : 0;
  const size_t gft = gather ? align256(gather_ft_bytes(p->N, nrhs)) : 0;
  const size_t need = tile + item + bufA + bufB + gpart + gft;
  if (need > kScratchBytes)
    return fail(p, NFFT_EUNSUPPORTED,
                "this adjoint needs %zu bytes of intermediate buffers; the library's scratch "
                "array holds %zu", need, kScratchBytes);
  void* base = nullptr;
  TRY(scratch_address(p, p->device, &base));
  unsigned char* b = static_cast<unsigned char*>(base);
  // spread mode 6 writes its grid (nrhs * Ms^d cells, fewer than the tile
  // partials') where the tile partials would be
  const Work wk{b, b + tile, bufA ? b + tile + item : nullptr,
                bufB ? b + tile + item + bufA : nullptr, b,
                gpart ? b + tile + item + bufA + bufB : nullptr,
                gft ? b + tile + item + bufA + bufB + gpart : nullptr};
  // the slots of tiles without nodes are read as zeros and written by no
  // work item; the previous call left its own data there
  HIP_TRY(p, nfft::launch_zero_tiles<R>((cplx<R>*)wk.tilep, (int64_t)g.nbins * g.Ptot,
                                        p->empty_bins, p->nempty, g.Ptot, nrhs, s));
  return run_adjoint<R>(p, f, fhat, nrhs, s, false, &wk);
}

}  // namespace

extern "C" {

const char* nfft_strerror(int status) {
  switch (status) {
    case NFFT_OK: return "success";
    case NFFT_EINVAL: return "invalid argument";
    case NFFT_ENOMEM: return "device memory allocation failed";
    case NFFT_EDEVICE: return "HIP device or kernel failure";
    case NFFT_ESTATE: return "call not allowed in the plan's current state";
    case NFFT_EUNSUPPORTED: return "parameters valid but not supported by this library";
    default: return "unknown status";
  }
}

const char* nfft_last_error(nfft_plan_t plan) {
  return plan ? plan->last_error.c_str() : g_noplan_error.c_str();
}

int64_t nfft_footprint(int d, int M, double sigma, int m, int64_t N, int precision, int max_rhs) {
  if (validate(d, M, sigma, m, N, precision, max_rhs, nullptr) != NFFT_OK) return -1;
  const int64_t Ms = oversampled(M, sigma);
  int tune[NFFT_TUNE_COUNT];
  if (resolve_tuning(d, (int)Ms, m, precision, nullptr, 0, tune, nullptr) != NFFT_OK) return -1;
  const int T = tune[NFFT_TUNE_TILE_EDGE];
  const int K = tune[NFFT_TUNE_ITEM_NODES];
  const int64_t nb = Ms / T;
  const int64_t nbins = ipow(nb, d);
  const int64_t P = T + 2 * m;
  const int64_t Ptot = ipow(P, d);
  const int64_t cb = (int64_t)cbytes(precision), rb = (int64_t)rbytes(precision);
  const int64_t nsub_max = nbins + (N + K - 1) / K;
  const int64_t R_ = max_rhs;
  int64_t bytes = 0;
  bytes += N * 4 + N * 4 + N * d * rb;                     // perm, loc, frac
  bytes += std::max<int64_t>(1, nsub_max) * 4 * 3 + (nbins + 1) * 4 + nbins * 4;  // item tables
  bytes += N * cb;                                        // weights
  bytes += R_ * (nbins + nsub_max) * Ptot * cb;           // tile and item partials
  bytes += 2 * m * 17 * rb + nsub_max * 4;                // window polynomials, item slots
  if (d >= 2) bytes += R_ * ipow(Ms, d - 1) * M * cb;
  if (d == 3) bytes += R_ * Ms * M * M * cb;
  bytes += R_ * ipow(Ms, d) * cb;                         // forward grid
  bytes += M * 8 + Ms * cb;                               // tables
  if (d == 2) bytes += N * 4 * m * rb;                    // window factors (spread mode 3)
  return bytes;
}

int nfft_plan(nfft_plan_t* out, int d, int M, double sigma, int m, int64_t N,
              const double* nodes, int precision, int max_rhs, void* stream) {
  return nfft_plan_tuned(out, d, M, sigma, m, N, nodes, precision, max_rhs, nullptr, 0, stream);
}

int nfft_plan_tuned(nfft_plan_t* out, int d, int M, double sigma, int m, int64_t N,
                    const double* nodes, int precision, int max_rhs, const int* tuning,
                    int ntuning, void* stream) {
  if (!out) return fail(nullptr, NFFT_EINVAL, "out is NULL");
  *out = nullptr;
  int st = validate(d, M, sigma, m, N, precision, max_rhs, nullptr);
  if (st != NFFT_OK) return st;
  int tune[NFFT_TUNE_COUNT];
  st = resolve_tuning(d, oversampled(M, sigma), m, precision, tuning, ntuning, tune, nullptr);
  if (st != NFFT_OK) return st;
  if (!nodes) return fail(nullptr, NFFT_EINVAL, "nodes is NULL");
  nfft_plan_t p = new (std::nothrow) nfft_plan_s();
  if (!p) return fail(nullptr, NFFT_ENOMEM, "host allocation failed");
  p->shared = std::make_shared<SharedData>();
  p->d = d;
  p->M = M;
  p->sigma = sigma;
  p->m = m;
  p->N = N;
  p->prec = precision;
  p->max_rhs = max_rhs;
  p->Ms = oversampled(M, sigma);
  p->b = M_PI * (2.0 - 1.0 / sigma);
  std::copy(tune, tune + NFFT_TUNE_COUNT, p->tune);
  Geom& g = p->g;
  g.d = d;
  g.Ms = p->Ms;
  g.M = M;
  g.m = m;
  g.T = p->tune[NFFT_TUNE_TILE_EDGE];
  g.nb = p->Ms / g.T;
  g.P = g.T + 2 * m;
  g.Ptot = (int)ipow(g.P, d);
  g.nbins = (int)ipow(g.nb, d);
  g.tshift = 0;
  while ((1 << g.tshift) < g.T) ++g.tshift;
  g.Ms_shift = 0;
  while ((1 << g.Ms_shift) < g.Ms) ++g.Ms_shift;
  g.N = N;
  if (hipGetDevice(&p->device) != hipSuccess) {
    free_plan(p);
    return fail(nullptr, NFFT_EDEVICE, "no HIP device available");
  }
  hipStream_t s = (hipStream_t)stream;
  st = precision == NFFT_F64 ? build_plan<double>(p, nodes, s) : build_plan<float>(p, nodes, s);
  if (st != NFFT_OK) {
    g_noplan_error = p->last_error;
    (void)hipStreamSynchronize(s);
    free_plan(p);
    return st;
  }
  *out = p;
  return NFFT_OK;
}

int nfft_plan_clone(nfft_plan_t src, int max_rhs, nfft_plan_t* out, void* stream) {
  if (!out) return fail(src, NFFT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!src) return fail(nullptr, NFFT_EINVAL, "plan is NULL");
  if (max_rhs < 1 || max_rhs > 65535) return fail(src, NFFT_EINVAL, "max_rhs = %d, expected 1..65535", max_rhs);
  nfft_plan_t p = new (std::nothrow) nfft_plan_s(*src);
  if (!p) return fail(src, NFFT_ENOMEM, "host allocation failed");
  // own workspace and bookkeeping; node data, weights and tables are shared
  p->allocs.clear();
  p->bytes = 0;
  p->pending.clear();
  p->event_pool.clear();
  p->profiling = false;
  for (int i = 0; i < NFFT_STAGES; ++i) {
    p->stage_ms[i] = 0;
    p->stage_calls[i] = 0;
  }
  p->last_error.clear();
  p->max_rhs = max_rhs;
  p->tilep = p->itemp = p->bufA = p->bufB = p->grid = nullptr;
  p->ref_r = nullptr;
  p->ref_red = nullptr;
  hipStream_t s = (hipStream_t)stream;
  int st = (hipSetDevice(p->device) == hipSuccess) ? NFFT_OK : NFFT_EDEVICE;
  if (st == NFFT_OK)
    st = p->prec == NFFT_F64 ? alloc_workspace<double>(p, s) : alloc_workspace<float>(p, s);
  if (st == NFFT_OK && hipStreamSynchronize(s) != hipSuccess) st = NFFT_EDEVICE;
  if (st != NFFT_OK) {
    src->last_error = p->last_error.empty() ? "clone failed" : p->last_error;
    free_plan(p);
    return st;
  }
  *out = p;
  return NFFT_OK;
}

int nfft_plan_autotune(nfft_plan_t* out, int d, int M, double sigma, int m, int64_t N,
                       const double* nodes, int precision, int max_rhs, int nrhs,
                       double* best_ms, void* stream) {
  if (!out) return fail(nullptr, NFFT_EINVAL, "out is NULL");
  *out = nullptr;
  int st = validate(d, M, sigma, m, N, precision, max_rhs, nullptr);
  if (st != NFFT_OK) return st;
  if (!nodes) return fail(nullptr, NFFT_EINVAL, "nodes is NULL");
  if (nrhs < 1 || nrhs > max_rhs)
    return fail(nullptr, NFFT_EINVAL, "nrhs = %d outside 1..max_rhs = %d", nrhs, max_rhs);
  hipStream_t s = (hipStream_t)stream;
  const int Ms = oversampled(M, sigma);
  const bool f32 = precision == NFFT_F32;
  // zero right-hand sides and an output buffer for the timing runs
  const size_t cb = cbytes(precision);
  void* f = nullptr;
  void* fhat = nullptr;
  if (hipMalloc(&f, (size_t)nrhs * N * cb) != hipSuccess ||
      hipMalloc(&fhat, (size_t)nrhs * ipow(M, d) * cb) != hipSuccess) {
    (void)hipFree(f);
    return fail(nullptr, NFFT_ENOMEM, "no device memory for the timing buffers");
  }
  ScopedFree bufs;
  bufs.ptrs = {f, fhat};
  if (hipMemsetAsync(f, 0, (size_t)nrhs * N * cb, s) != hipSuccess)
    return fail(nullptr, NFFT_EDEVICE, "hipMemsetAsync failed");

  std::vector<int> tiles, items = {128, 256, 512};
  if (d == 2 && f32) items.push_back(1024);
  if (d == 1) tiles = {64, 128, 256};
  else if (d == 2) tiles = {8, 16, 32};
  else tiles = {8, 16};
  std::vector<int> threads = {0}, planes = {0}, rpg = {0}, modes = {0};
  if (d <= 2 && f32) {
    threads = {64, 128, 256, 512};
    planes = {1, 2};
  }
  if (d <= 2 && nrhs > 1) rpg = {1, 2, 4, 8};
  // float64: the work-group size matters to the matrix-core register tile only
  if (d == 2 && !f32) threads = {128, 256};
  if (d == 2) modes = {1, 2, 3, 4, 7};
  if (d == 2 && f32) modes = {1, 2, 3, 4, 5, 7};
  if (d == 3) modes = {1, 7};
  // the grid-tile gather holds 32 right-hand sides in the lanes of a wave;
  // its units also try 768 list entries (fewer split tiles than 512, fewer
  // long units than 1024)
  if (d == 2 && f32 && nrhs >= 8) {
    modes.push_back(6);
    items.insert(std::find(items.begin(), items.end(), 1024), 768);
  }

  nfft_plan_t best = nullptr;
  double best_t = -1.0;
  int best_tune[NFFT_TUNE_COUNT] = {0};
  for (int T : tiles) {
    if (T > Ms) continue;
    for (int K : items) {
      int tune[NFFT_TUNE_COUNT] = {T, K, 0, 0, 0, 0, 0};
      int resolved[NFFT_TUNE_COUNT];
      if (resolve_tuning(d, Ms, m, precision, tune, NFFT_TUNE_COUNT, resolved, nullptr) != NFFT_OK)
        continue;
      nfft_plan_t p = nullptr;
      st = nfft_plan_tuned(&p, d, M, sigma, m, N, nodes, precision, max_rhs, tune,
                           NFFT_TUNE_COUNT, stream);
      if (st == NFFT_ENOMEM || st == NFFT_EUNSUPPORTED) continue;
      if (st != NFFT_OK) {
        if (best) free_plan(best);
        return st;
      }
      if (hipMemsetAsync(p->w, 0, (size_t)N * cb, s) != hipSuccess) {
        free_plan(p);
        if (best) free_plan(best);
        return fail(nullptr, NFFT_EDEVICE, "hipMemsetAsync failed");
      }
      bool mine = false;  // p is (or became) the best plan
      // the factor table of mode 3; without room for it mode 3 is skipped
      const bool have_psi = d == 2 && ensure_psi_any(p, s) == NFFT_OK;
      // the node lists of mode 6, likewise
      const bool have_gather = gather_supported(p) &&
                               std::find(modes.begin(), modes.end(), 6) != modes.end() &&
                               ensure_gather(p, s) == NFFT_OK && p->shared->g_units;
      for (int md : modes)
      for (int nt : threads)
        for (int pl : planes)
          for (int nr : rpg) {
            int in[NFFT_TUNE_COUNT];
            std::copy(p->tune, p->tune + NFFT_TUNE_COUNT, in);
            if (nt) in[NFFT_TUNE_SPREAD_THREADS] = nt;
            if (pl) in[NFFT_TUNE_SPREAD_PLANES] = pl;
            if (nr) in[NFFT_TUNE_RHS_PER_GROUP] = nr;
            if (md) in[NFFT_TUNE_SPREAD_MODE] = md;
            // the LDS kernel's shape does not matter when another kernel spreads
            if ((nr > 1 || md == 2) && (nt != threads[0] || pl != planes[0])) continue;
            // the register-tile kernels (modes 5, 7) take one rhs per work-group
            // and no LDS tile layout
            if ((md == 5 || md == 7) && (nr > 1 || pl != planes[0])) continue;
            // the gather (mode 6) has one shape; 768 entries per unit are for it alone
            if (md == 6 && (nr > 1 || pl != planes[0] || nt != threads[0])) continue;
            if (K == 768 && md != 6) continue;
            // float64: only mode 7 takes the thread count
            if (!f32 && md != 7 && nt != threads[0]) continue;
            if (nt == 512 && md < 5) continue;
            if (nr > 2 && md == 2) continue;  // the row sweep takes at most two rhs per wave
            if (uses_psi(md) && !have_psi) continue;
            if (md == 6 && !have_gather) continue;
            if (md == 3 && nr > 1) continue;  // modes 3, 4: single rhs only
            if (md == 4 && nr > 1) continue;
            int res[NFFT_TUNE_COUNT];
            if (resolve_tuning(d, Ms, m, precision, in, NFFT_TUNE_COUNT, res, nullptr) != NFFT_OK)
              continue;
            std::copy(res, res + NFFT_TUNE_COUNT, p->tune);
            const double t = time_adjoint(p, f, fhat, nrhs, s);
            if (t < 0) continue;
            if (best_t < 0 || t < best_t) {
              best_t = t;
              std::copy(res, res + NFFT_TUNE_COUNT, best_tune);
              if (best && best != p) free_plan(best);
              best = p;
              mine = true;
            }
          }
      if (mine) {
        std::copy(best_tune, best_tune + NFFT_TUNE_COUNT, p->tune);
      } else {
        free_plan(p);
      }
    }
  }
  if (!best) return fail(nullptr, NFFT_EUNSUPPORTED, "no candidate tuning could be planned and timed");
  // FFT work-group width on the winner
  for (int fw : {64, 1024}) {
    int in[NFFT_TUNE_COUNT], res[NFFT_TUNE_COUNT];
    std::copy(best_tune, best_tune + NFFT_TUNE_COUNT, in);
    in[NFFT_TUNE_FFT_MIN_WG] = fw;
    if (resolve_tuning(d, Ms, m, precision, in, NFFT_TUNE_COUNT, res, nullptr) != NFFT_OK) continue;
    std::copy(res, res + NFFT_TUNE_COUNT, best->tune);
    const double t = time_adjoint(best, f, fhat, nrhs, s);
    if (t >= 0 && t < best_t) {
      best_t = t;
      std::copy(res, res + NFFT_TUNE_COUNT, best_tune);
    }
  }
  std::copy(best_tune, best_tune + NFFT_TUNE_COUNT, best->tune);
  if (hipStreamSynchronize(s) != hipSuccess) {
    free_plan(best);
    return fail(nullptr, NFFT_EDEVICE, "device failure while timing candidates");
  }
  if (!uses_psi(best->tune[NFFT_TUNE_SPREAD_MODE])) drop_psi(best);
  if (best->tune[NFFT_TUNE_SPREAD_MODE] != 6) drop_gather(best);
  best->shared->has_weights = false;
  if (best_ms) *best_ms = best_t;
  *out = best;
  return NFFT_OK;
}

int nfft_weights(int d, int M, double sigma, int m, int64_t N, const double* nodes, double tol,
                 int maxit, void* w_out, double* info, void* stream) {
  return nfft_weights_ex(d, M, sigma, m, N, nodes, NFFT_WEIGHTS_ALG36, tol, maxit, w_out, info,
                         stream);
}

int nfft_weights_ex(int d, int M, double sigma, int m, int64_t N, const double* nodes, int scheme,
                    double tol, int maxit, void* w_out, double* info, void* stream) {
  if (!w_out) return fail(nullptr, NFFT_EINVAL, "w is NULL");
  if (scheme != NFFT_WEIGHTS_ALG36 && scheme != NFFT_WEIGHTS_RELAXED && scheme != NFFT_WEIGHTS_PCF)
    return fail(nullptr, NFFT_EINVAL, "weight scheme %d unknown", scheme);
  if (!(tol > 0.0) || maxit < 1)
    return fail(nullptr, NFFT_EINVAL, "tol = %g, maxit = %d: expected tol > 0, maxit >= 1", tol, maxit);
  if (M < 2 || M > (1 << 20) || (M % 2) != 0)
    return fail(nullptr, NFFT_EINVAL, "M = %d, expected an even M >= 2", M);
  if (scheme == NFFT_WEIGHTS_PCF) {
    // (3.62) directly: O(N^2) pairs
    if (d < 1 || d > 3) return fail(nullptr, NFFT_EINVAL, "d = %d, expected 1, 2 or 3", d);
    if (N < 1 || N > 0x7fffffffLL) return fail(nullptr, NFFT_EINVAL, "N out of range");
    if (!nodes) return fail(nullptr, NFFT_EINVAL, "nodes is NULL");
    hipStream_t s = (hipStream_t)stream;
    void* dx = nullptr;
    if (hipMalloc(&dx, N * d * sizeof(double)) != hipSuccess)
      return fail(nullptr, NFFT_ENOMEM, "no device memory for the nodes");
    ScopedFree keep;
    keep.ptrs.push_back(dx);
    HIP_TRY(nullptr, hipMemcpyAsync(dx, nodes, N * d * sizeof(double), hipMemcpyDefault, s));
    HIP_TRY(nullptr, nfft::launch_pcf((const double*)dx, N, d, M, (cplx<double>*)w_out, s));
    HIP_TRY(nullptr, hipStreamSynchronize(s));
    if (info) {
      info[0] = 0;
      info[1] = 0;
      info[2] = 62;
      info[3] = 0;
    }
    return NFFT_OK;
  }
  const bool relaxed = scheme == NFFT_WEIGHTS_RELAXED;
  nfft_plan_t p = nullptr;
  int st = nfft_plan(&p, d, relaxed ? M : 2 * M, sigma, m, N, nodes, NFFT_F64, 1, stream);
  if (st != NFFT_OK) return st;
  struct PlanGuard {
    nfft_plan_t p;
    ~PlanGuard() { free_plan(p); }
  } guard{p};
  hipStream_t s = (hipStream_t)stream;
  using C = cplx<double>;
  const int64_t K2 = ipow(relaxed ? M : 2 * M, d);
  // Algorithm 3.6 step 2: which normal equations; (3.63) is always a system in C^N
  const bool b15 = !relaxed && K2 <= N;
  const int64_t n = b15 ? K2 : N;     // length of the CG vectors
  int64_t e_idx = 0;                  // index of k = 0 in I_2M (C order, k_t from -M)
  for (int t = 0; t < d; ++t) e_idx = e_idx * (2 * M) + M;

  ScopedFree bufs;
  auto alloc = [&](C** q, int64_t count) -> int {
    void* v = nullptr;
    if (hipMalloc(&v, (size_t)std::max<int64_t>(1, count) * sizeof(C)) != hipSuccess)
      return fail(nullptr, NFFT_ENOMEM, "no device memory for the CG vectors");
    bufs.ptrs.push_back(v);
    *q = (C*)v;
    return NFFT_OK;
  };
  C *x, *r, *pv, *q, *tmp;
  TRY(alloc(&x, n));
  TRY(alloc(&r, n));
  TRY(alloc(&pv, n));
  TRY(alloc(&q, n));
  TRY(alloc(&tmp, b15 ? N : K2));
  double* scratch = nullptr;
  if (hipMalloc((void**)&scratch, nfft::reduce_scratch_doubles() * sizeof(double)) != hipSuccess)
    return fail(nullptr, NFFT_ENOMEM, "no device memory for the reductions");
  bufs.ptrs.push_back(scratch);
  const double* result = scratch + (nfft::reduce_scratch_doubles() - 1);

  // unit weights on the internal plan: its adjoint is then A_2M^* itself
  if (nfft::launch_fill((C*)p->w, N, 1.0, 0.0, s) != hipSuccess)
    return fail(nullptr, NFFT_EDEVICE, "fill kernel failed");
  p->shared->has_weights = true;

  // CG on the conjugated systems. With A^T y = conj(adjoint(conj y)) and
  // conj(A) v = conj(forward(conj v)), the operator A^T conj(A) of (3.15)
  // maps q = conj(v) to conj(A^T conj(A) v) = adjoint(forward(q)), and
  // conj(A) A^T of (3.16) becomes forward(adjoint(q)). The right-hand sides
  // e_0 and 1_N are real and CG's step lengths are real, so these iterates
  // are the conjugates of CG on the original systems.
  auto apply = [&](const C* in, C* out) -> int {
    if (b15) {
      TRY(run_forward<double>(p, in, tmp, 1, s));
      TRY(run_adjoint<double>(p, tmp, out, 1, s));
    } else {
      TRY(run_adjoint<double>(p, in, tmp, 1, s));
      TRY(run_forward<double>(p, tmp, out, 1, s));
    }
    return NFFT_OK;
  };
  auto reduce = [&](const C* a, const C* b, int64_t len, int op, double* out) -> int {
    if (nfft::launch_reduce(a, b, len, op, e_idx, scratch, s) != hipSuccess ||
        hipMemcpyAsync(out, result, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(nullptr, NFFT_EDEVICE, "reduction failed");
    return NFFT_OK;
  };
  HIP_TRY(nullptr, nfft::launch_fill(x, n, 0.0, 0.0, s));
  if (b15) {
    HIP_TRY(nullptr, nfft::launch_fill(r, n, 0.0, 0.0, s));
    HIP_TRY(nullptr, nfft::launch_fill(r + e_idx, 1, 1.0, 0.0, s));
  } else {
    HIP_TRY(nullptr, nfft::launch_fill(r, n, 1.0, 0.0, s));
  }
  HIP_TRY(nullptr, hipMemcpyAsync(pv, r, n * sizeof(C), hipMemcpyDeviceToDevice, s));
  double rr = 0.0;
  TRY(reduce(r, r, n, 0, &rr));
  const double nb = std::sqrt(rr);
  int it = 0;
  while (it < maxit && std::sqrt(rr) > tol * nb) {
    TRY(apply(pv, q));
    double pAp = 0.0;
    TRY(reduce(pv, q, n, 0, &pAp));
    if (!(pAp > 0.0)) break;  // exact solution reached or breakdown
    const double alpha = rr / pAp;
    HIP_TRY(nullptr, nfft::launch_cg_update(x, r, pv, q, n, alpha, s));
    double rr_new = 0.0;
    TRY(reduce(r, r, n, 0, &rr_new));
    HIP_TRY(nullptr, nfft::launch_cg_direction(pv, r, n, rr_new / rr, s));
    rr = rr_new;
    ++it;
  }
  // conj(w): (3.15) forward of the solution, (3.16) the solution itself;
  // (3.63): w itself (A A^* is the operator, no conjugation)
  C* w = (C*)w_out;
  if (b15)
    TRY(run_forward<double>(p, x, w, 1, s));
  else
    HIP_TRY(nullptr, hipMemcpyAsync(w, x, N * sizeof(C), hipMemcpyDeviceToDevice, s));
  double eps = 0.0;
  if (relaxed) {
    // max_j |[A A^* w]_j - 1|
    TRY(apply(w, q));
    TRY(reduce(q, q, N, 2, &eps));
  } else {
    // epsilon: A_2M^T w = conj(adjoint(conj w)), and e_0 is real
    C* at = b15 ? q : tmp;
    TRY(run_adjoint<double>(p, w, at, 1, s));
    TRY(reduce(at, at, K2, 1, &eps));
    HIP_TRY(nullptr, nfft::launch_conj(w, N, s));
  }
  HIP_TRY(nullptr, hipStreamSynchronize(s));
  if (info) {
    info[0] = it;
    info[1] = nb > 0 ? std::sqrt(rr) / nb : 0.0;
    info[2] = relaxed ? 63 : (b15 ? 15 : 16);
    info[3] = eps;
  }
  return NFFT_OK;
}

int nfft_bopt_build(nfft_plan_t p, const double* nodes, double* info, void* stream) {
  if (!p) return fail(nullptr, NFFT_EINVAL, "plan is NULL");
  if (!nodes) return fail(p, NFFT_EINVAL, "nodes is NULL");
  SharedData& sd = *p->shared;
  if (sd.has_bopt) return fail(p, NFFT_ESTATE, "B_opt is already built for this node set");
  hipStream_t s = (hipStream_t)stream;
  const int d = p->d, Ms = p->Ms, M = p->M, m = p->m;
  const int64_t N = p->N;
  const int64_t ncols = ipow(Ms, d);
  ScopedFree tmp;
  auto talloc = [&](void** q, size_t bytes) -> int {
    if (hipMalloc(q, bytes ? bytes : 16) != hipSuccess)
      return fail(p, NFFT_ENOMEM, "hipMalloc(%zu) failed", bytes);
    tmp.ptrs.push_back(*q);
    return NFFT_OK;
  };
  void *d_nodes, *count, *fill, *wh, *dropped;
  TRY(talloc(&d_nodes, N * d * sizeof(double)));
  TRY(talloc(&count, ncols * sizeof(int)));
  TRY(talloc(&fill, ncols * sizeof(int)));
  TRY(talloc(&wh, M * sizeof(double)));
  TRY(talloc(&dropped, sizeof(int)));
  HIP_TRY(p, hipMemcpyAsync(d_nodes, nodes, N * d * sizeof(double), hipMemcpyDefault, s));
  HIP_TRY(p, hipMemsetAsync(count, 0, ncols * sizeof(int), s));
  HIP_TRY(p, hipMemsetAsync(fill, 0, ncols * sizeof(int), s));
  HIP_TRY(p, hipMemsetAsync(dropped, 0, sizeof(int), s));
  HIP_TRY(p, nfft::launch_bopt_pattern((const double*)d_nodes, N, d, Ms, m, 0, (int*)count,
                                       nullptr, nullptr, nullptr, s));
  std::vector<int> hc(ncols);
  HIP_TRY(p, hipMemcpyAsync(hc.data(), count, ncols * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(p, hipStreamSynchronize(s));
  std::vector<int64_t> hp(ncols + 1, 0);
  int nmax = 0;
  for (int64_t c = 0; c < ncols; ++c) {
    hp[c + 1] = hp[c] + hc[c];
    nmax = std::max(nmax, hc[c]);
  }
  // columns whose packed Gram triangle fits in LDS are solved there; larger
  // ones with the triangle and their per-node arrays in a device-memory
  // workspace
  int cap_lds = 1;
  while (nfft::bopt_solve_lds(cap_lds + 1) <= kMaxLds) ++cap_lds;
  if (nmax > kMaxBoptColumn)
    return fail(p, NFFT_EUNSUPPORTED,
                "a grid column is reached by %d nodes; the column solve takes at most %d", nmax,
                kMaxBoptColumn);
  // columns solved in device memory, largest first, in batches whose
  // workspaces together take at most kBoptBatchBytes (one column at least);
  // off[i]: the i-th column's workspace offset (doubles) within its batch
  std::vector<int64_t> big;
  for (int64_t c = 0; c < ncols; ++c)
    if (hc[c] > cap_lds) big.push_back(c);
  std::stable_sort(big.begin(), big.end(),
                   [&](int64_t a, int64_t b) { return hc[a] > hc[b]; });
  constexpr int64_t kBoptBatchBytes = int64_t(4) << 30;
  std::vector<int64_t> off(big.size()), batch_start;
  int64_t ws_doubles = 0;
  for (size_t i = 0, used = 0; i < big.size(); ++i) {
    const int64_t need = nfft::bopt_workspace_doubles(hc[big[i]]);
    if (i == 0 || (int64_t)(used + need) * 8 > kBoptBatchBytes) {
      batch_start.push_back((int64_t)i);
      used = 0;
    }
    off[i] = (int64_t)used;
    used += need;
    ws_doubles = std::max<int64_t>(ws_doubles, (int64_t)used);
  }
  batch_start.push_back((int64_t)big.size());
  const int64_t nnz = hp[ncols];
  const size_t rb = rbytes(p->prec);
  TRY(dalloc(p, &sd.bopt_ptr, (ncols + 1) * sizeof(int64_t)));
  TRY(dalloc(p, &sd.bopt_node, std::max<int64_t>(1, nnz) * sizeof(int32_t)));
  TRY(dalloc(p, &sd.bopt_val, std::max<int64_t>(1, nnz) * rb));
  HIP_TRY(p, hipMemcpyAsync(sd.bopt_ptr, hp.data(), (ncols + 1) * sizeof(int64_t),
                            hipMemcpyHostToDevice, s));
  HIP_TRY(p, nfft::launch_bopt_pattern((const double*)d_nodes, N, d, Ms, m, 1, nullptr,
                                       sd.bopt_ptr, (int*)fill, sd.bopt_node, s));
  // w^(k) = I_0(m sqrt(b^2 - (2 pi k / M_s)^2)) / M_s, k = -M/2 .. M/2-1
  std::vector<double> hw(M);
  for (int i = 0; i < M; ++i) {
    const long double k = (long double)(i - M / 2);
    const long double arg = (long double)p->b * p->b -
                            (2.0L * M_PI * k / Ms) * (2.0L * M_PI * k / Ms);
    hw[i] = (double)(bessel_i0((long double)m * std::sqrt(std::max(arg, 0.0L))) / Ms);
  }
  HIP_TRY(p, hipMemcpyAsync(wh, hw.data(), M * sizeof(double), hipMemcpyHostToDevice, s));
  constexpr double kPivotRel = 1e-13;
  // ridge on the Gram diagonal (which is |I_M|) for rank-deficient columns
  const double ridge = 1e-12 * (double)ipow(M, d);
  auto solve = [&](int64_t nc, int nm, const int64_t* cols, double* ws, const int64_t* ws_off) {
    return p->prec == NFFT_F64
               ? nfft::launch_bopt_solve<double>((const double*)d_nodes, d, M, Ms,
                                                 (const double*)wh, sd.bopt_ptr, sd.bopt_node,
                                                 (double*)sd.bopt_val, nc, nm, kPivotRel, ridge,
                                                 (int*)dropped, cols, ws, ws_off, s)
               : nfft::launch_bopt_solve<float>((const double*)d_nodes, d, M, Ms,
                                                (const double*)wh, sd.bopt_ptr, sd.bopt_node,
                                                (float*)sd.bopt_val, nc, nm, kPivotRel, ridge,
                                                (int*)dropped, cols, ws, ws_off, s);
  };
  HIP_TRY(p, solve(ncols, std::max(1, std::min(nmax, cap_lds)), nullptr, nullptr, nullptr));
  if (!big.empty()) {
    void *d_cols, *d_off, *ws;
    TRY(talloc(&d_cols, big.size() * sizeof(int64_t)));
    TRY(talloc(&d_off, big.size() * sizeof(int64_t)));
    TRY(talloc(&ws, (size_t)ws_doubles * sizeof(double)));
    HIP_TRY(p, hipMemcpyAsync(d_cols, big.data(), big.size() * sizeof(int64_t),
                              hipMemcpyHostToDevice, s));
    HIP_TRY(p, hipMemcpyAsync(d_off, off.data(), off.size() * sizeof(int64_t),
                              hipMemcpyHostToDevice, s));
    for (size_t b = 0; b + 1 < batch_start.size(); ++b)
      HIP_TRY(p, solve(batch_start[b + 1] - batch_start[b], kMaxBoptColumn,
                       (const int64_t*)d_cols + batch_start[b], (double*)ws,
                       (const int64_t*)d_off + batch_start[b]));
  }
  // the same values by rows, for the inverse adjoint of Remark 4.6
  const int64_t F = ipow(2 * m + 1, d);
  TRY(dalloc(p, &sd.bopt_lo, N * d * sizeof(int32_t)));
  TRY(dalloc(p, &sd.bopt_rows, N * F * rb));
  HIP_TRY(p, hipMemsetAsync(sd.bopt_rows, 0, N * F * rb, s));
  HIP_TRY(p, nfft::launch_bopt_lo((const double*)d_nodes, N, d, Ms, m, sd.bopt_lo, s));
  if (p->prec == NFFT_F64)
    HIP_TRY(p, nfft::launch_bopt_rows<double>(sd.bopt_ptr, sd.bopt_node, (const double*)sd.bopt_val,
                                              ncols, d, Ms, m, sd.bopt_lo, (double*)sd.bopt_rows, s));
  else
    HIP_TRY(p, nfft::launch_bopt_rows<float>(sd.bopt_ptr, sd.bopt_node, (const float*)sd.bopt_val,
                                             ncols, d, Ms, m, sd.bopt_lo, (float*)sd.bopt_rows, s));
  int hd = 0;
  HIP_TRY(p, hipMemcpyAsync(&hd, dropped, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(p, hipStreamSynchronize(s));
  sd.has_bopt = true;
  sd.bopt_nnz = nnz;
  sd.bopt_nmax = nmax;
  // lanes per column of nfft_bopt_adjoint's sparse product: NFFT_BOPT_LANES
  // (4, 8, 16, 32 or 64) if set, else sized to the mean column length
  const int lanes = env_int("NFFT_BOPT_LANES", 0);
  sd.bopt_lanes = (lanes >= 4 && lanes <= 64 && (lanes & (lanes - 1)) == 0)
                      ? lanes
                      : nfft::bopt_apply_lanes((double)nnz / (double)ncols);
  if (info) {
    info[0] = nmax;
    info[1] = (double)nnz;
    info[2] = hd;
  }
  return NFFT_OK;
}

int nfft_bopt_adjoint(nfft_plan_t p, const void* f, void* fhat, int nrhs, void* stream) {
  if (!p) return fail(nullptr, NFFT_EINVAL, "plan is NULL");
  if (!f || !fhat) return fail(p, NFFT_EINVAL, "f or fhat is NULL");
  if (nrhs < 1 || nrhs > p->max_rhs)
    return fail(p, NFFT_EINVAL, "nrhs = %d outside 1..max_rhs = %d", nrhs, p->max_rhs);
  if (!p->shared->has_bopt) return fail(p, NFFT_ESTATE, "nfft_bopt_build has not been called");
  HIP_TRY(p, hipGetLastError());
  hipStream_t s = (hipStream_t)stream;
  return p->prec == NFFT_F64 ? run_bopt_adjoint<double>(p, f, fhat, nrhs, s)
                             : run_bopt_adjoint<float>(p, f, fhat, nrhs, s);
}

int nfft_bopt_inverse_adjoint(nfft_plan_t p, const void* h, void* f, int nrhs, void* stream) {
  if (!p) return fail(nullptr, NFFT_EINVAL, "plan is NULL");
  if (!f || !h) return fail(p, NFFT_EINVAL, "h or f is NULL");
  if (nrhs < 1 || nrhs > p->max_rhs)
    return fail(p, NFFT_EINVAL, "nrhs = %d outside 1..max_rhs = %d", nrhs, p->max_rhs);
  if (!p->shared->has_bopt) return fail(p, NFFT_ESTATE, "nfft_bopt_build has not been called");
  HIP_TRY(p, hipGetLastError());
  hipStream_t s = (hipStream_t)stream;
  return p->prec == NFFT_F64 ? run_bopt_inverse_adjoint<double>(p, h, f, nrhs, s)
                             : run_bopt_inverse_adjoint<float>(p, h, f, nrhs, s);
}

int nfft_bopt_get(nfft_plan_t p, int64_t* nnz, int64_t* col_ptr, int32_t* nodes, double* vals) {
  if (!p) return fail(nullptr, NFFT_EINVAL, "plan is NULL");
  SharedData& sd = *p->shared;
  if (!sd.has_bopt) return fail(p, NFFT_ESTATE, "nfft_bopt_build has not been called");
  if (nnz) *nnz = sd.bopt_nnz;
  const int64_t ncols = ipow(p->Ms, p->d);
  if (col_ptr)
    HIP_TRY(p, hipMemcpy(col_ptr, sd.bopt_ptr, (ncols + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
  if (nodes)
    HIP_TRY(p, hipMemcpy(nodes, sd.bopt_node, sd.bopt_nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (vals) {
    if (p->prec == NFFT_F64) {
      HIP_TRY(p, hipMemcpy(vals, sd.bopt_val, sd.bopt_nnz * sizeof(double), hipMemcpyDeviceToHost));
    } else {
      std::vector<float> tmpv(sd.bopt_nnz);
      HIP_TRY(p, hipMemcpy(tmpv.data(), sd.bopt_val, sd.bopt_nnz * sizeof(float),
                           hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < sd.bopt_nnz; ++i) vals[i] = tmpv[i];
    }
  }
  return NFFT_OK;
}

int nfft_get_tuning(nfft_plan_t p, int* out, int n) {
  if (!p) return fail(nullptr, NFFT_EINVAL, "plan is NULL");
  if (!out || n < 0 || n > NFFT_TUNE_COUNT)
    return fail(p, NFFT_EINVAL, "out is NULL or n = %d outside 0..%d", n, NFFT_TUNE_COUNT);
  for (int k = 0; k < n; ++k) out[k] = p->tune[k];
  return NFFT_OK;
}

int nfft_set_tuning(nfft_plan_t p, int knob, int value) {
  if (!p) return fail(nullptr, NFFT_EINVAL, "plan is NULL");
  if (knob != NFFT_TUNE_SPREAD_THREADS && knob != NFFT_TUNE_RHS_PER_GROUP &&
      knob != NFFT_TUNE_FFT_MIN_WG && knob != NFFT_TUNE_SPREAD_PLANES &&
      knob != NFFT_TUNE_SPREAD_MODE)
    return fail(p, NFFT_EINVAL, "tuning knob %d cannot change after planning", knob);
  int in[NFFT_TUNE_COUNT], out[NFFT_TUNE_COUNT];
  std::copy(p->tune, p->tune + NFFT_TUNE_COUNT, in);
  in[knob] = value;
  const int st = resolve_tuning(p->d, p->Ms, p->m, p->prec, in, NFFT_TUNE_COUNT, out, p);
  if (st != NFFT_OK) return st;
  if (uses_psi(out[NFFT_TUNE_SPREAD_MODE]) && !p->shared->psi) {
    // the factor table is built once, on the null stream, before the switch
    TRY(ensure_psi_any(p, nullptr));
    HIP_TRY(p, hipStreamSynchronize(nullptr));
  }
  if (out[NFFT_TUNE_SPREAD_MODE] == 6) {
    // likewise the node lists of the gather and this handle's partials
    TRY(ensure_gather(p, nullptr));
    HIP_TRY(p, hipStreamSynchronize(nullptr));
  }
  std::copy(out, out + NFFT_TUNE_COUNT, p->tune);
  return NFFT_OK;
}

int nfft_set_weights(nfft_plan_t p, const double* w, void* stream) {
  if (!p) return fail(nullptr, NFFT_EINVAL, "plan is NULL");
  if (!w) return fail(p, NFFT_EINVAL, "w is NULL");
  hipStream_t s = (hipStream_t)stream;
  void* dw = nullptr;
  HIP_TRY(p, hipMalloc(&dw, p->N * 2 * sizeof(double)));
  ScopedFree tmp;
  tmp.ptrs.push_back(dw);
  HIP_TRY(p, hipMemcpyAsync(dw, w, p->N * 2 * sizeof(double), hipMemcpyDefault, s));
  if (p->prec == NFFT_F64)
    HIP_TRY(p, nfft::launch_permute_weights<double>((const double*)dw, p->perm, p->N,
                                                    (cplx<double>*)p->w, s));
  else
    HIP_TRY(p, nfft::launch_permute_weights<float>((const double*)dw, p->perm, p->N,
                                                   (cplx<float>*)p->w, s));
  HIP_TRY(p, hipStreamSynchronize(s));
  p->shared->has_weights = true;
  return NFFT_OK;
}

int nfft_adjoint(nfft_plan_t p, const void* f, void* fhat, int nrhs, void* stream) {
  if (!p) return fail(nullptr, NFFT_EINVAL, "plan is NULL");
  if (!f || !fhat) return fail(p, NFFT_EINVAL, "f or fhat is NULL");
  if (nrhs < 1 || nrhs > p->max_rhs)
    return fail(p, NFFT_EINVAL, "nrhs = %d outside 1..max_rhs = %d", nrhs, p->max_rhs);
  if (!p->shared->has_weights) return fail(p, NFFT_ESTATE, "nfft_set_weights has not been called");
  HIP_TRY(p, hipGetLastError());
  hipStream_t s = (hipStream_t)stream;
  return p->prec == NFFT_F64 ? run_adjoint<double>(p, f, fhat, nrhs, s)
                             : run_adjoint<float>(p, f, fhat, nrhs, s);
}

int nfft_adjoint_scratch(nfft_plan_t p, const void* f, void* fhat, int nrhs, void* stream) {
  if (!p) return fail(nullptr, NFFT_EINVAL, "plan is NULL");
  if (!f || !fhat) return fail(p, NFFT_EINVAL, "f or fhat is NULL");
  if (nrhs < 1 || nrhs > p->max_rhs)
    return fail(p, NFFT_EINVAL, "nrhs = %d outside 1..max_rhs = %d", nrhs, p->max_rhs);
  if (!p->shared->has_weights) return fail(p, NFFT_ESTATE, "nfft_set_weights has not been called");
  HIP_TRY(p, hipGetLastError());
  hipStream_t s = (hipStream_t)stream;
  return p->prec == NFFT_F64 ? run_adjoint_scratch<double>(p, f, fhat, nrhs, s)
                             : run_adjoint_scratch<float>(p, f, fhat, nrhs, s);
}

int nfft_forward(nfft_plan_t p, const void* fhat, void* f, int nrhs, void* stream) {
  if (!p) return fail(nullptr, NFFT_EINVAL, "plan is NULL");
  if (!f || !fhat) return fail(p, NFFT_EINVAL, "f or fhat is NULL");
  if (nrhs < 1 || nrhs > p->max_rhs)
    return fail(p, NFFT_EINVAL, "nrhs = %d outside 1..max_rhs = %d", nrhs, p->max_rhs);
  HIP_TRY(p, hipGetLastError());
  hipStream_t s = (hipStream_t)stream;
  return p->prec == NFFT_F64 ? run_forward<double>(p, fhat, f, nrhs, s)
                             : run_forward<float>(p, fhat, f, nrhs, s);
}

int nfft_refine(nfft_plan_t p, const void* f, void* fhat, int nrhs, int iters, double* res,
                void* stream) {
  if (!p) return fail(nullptr, NFFT_EINVAL, "plan is NULL");
  if (!f || !fhat) return fail(p, NFFT_EINVAL, "f or fhat is NULL");
  if (nrhs < 1 || nrhs > p->max_rhs)
    return fail(p, NFFT_EINVAL, "nrhs = %d outside 1..max_rhs = %d", nrhs, p->max_rhs);
  if (iters < 0 || iters > kMaxRefine)
    return fail(p, NFFT_EINVAL, "iters = %d outside 0..%d", iters, kMaxRefine);
  if (!p->shared->has_weights) return fail(p, NFFT_ESTATE, "nfft_set_weights has not been called");
  HIP_TRY(p, hipGetLastError());
  hipStream_t s = (hipStream_t)stream;
  return p->prec == NFFT_F64 ? run_refine<double>(p, f, fhat, nrhs, iters, res, s)
                             : run_refine<float>(p, f, fhat, nrhs, iters, res, s);
}

int nfft_destroy(nfft_plan_t p) {
  if (!p) return NFFT_OK;
  int st = NFFT_OK;
  if (hipDeviceSynchronize() != hipSuccess) st = NFFT_EDEVICE;
  free_plan(p);
  return st;
}

int nfft_plan_info(nfft_plan_t p, int64_t* out, int n) {
  if (!p || !out || n < 0) return fail(p, NFFT_EINVAL, "bad arguments to nfft_plan_info");
  const int64_t v[13] = {p->d, p->M, p->Ms, p->m, p->N, p->prec, p->max_rhs,
                         p->g.T, p->g.nbins, p->g.nsub, p->maxpop,
                         p->bytes + p->shared->bytes, p->bytes};
  for (int i = 0; i < n && i < 13; ++i) out[i] = v[i];
  return NFFT_OK;
}

int nfft_permutation(nfft_plan_t p, int32_t* perm_host) {
  if (!p || !perm_host) return fail(p, NFFT_EINVAL, "bad arguments to nfft_permutation");
  HIP_TRY(p, hipMemcpy(perm_host, p->perm, p->N * sizeof(int32_t), hipMemcpyDeviceToHost));
  return NFFT_OK;
}

int nfft_set_profiling(nfft_plan_t p, int enable) {
  if (!p) return fail(nullptr, NFFT_EINVAL, "plan is NULL");
  p->profiling = enable != 0;
  return NFFT_OK;
}

int nfft_stage_times(nfft_plan_t p, double* out, int n, int reset) {
  if (!p) return fail(nullptr, NFFT_EINVAL, "plan is NULL");
  for (auto& se : p->pending) {
    HIP_TRY(p, hipEventSynchronize(se.ev[se.n - 1]));
    float ms = 0.f;
    if (se.kind == 0) {
      // adjoint: start, after spread, after split-tile reduce, after first FFT pass, end
      for (int i = 0; i + 1 < se.n && i < 4; ++i) {
        HIP_TRY(p, hipEventElapsedTime(&ms, se.ev[i], se.ev[i + 1]));
        p->stage_ms[i] += ms;
        p->stage_calls[i] += 1;
      }
    } else {
      // forward: start, after FFT passes, after window sums;
      // B_opt adjoint: start, after the sparse product, after FFT passes
      const int base = se.kind == 1 ? 4 : 6;
      for (int i = 0; i + 1 < se.n && i < 2; ++i) {
        HIP_TRY(p, hipEventElapsedTime(&ms, se.ev[i], se.ev[i + 1]));
        p->stage_ms[base + i] += ms;
        p->stage_calls[base + i] += 1;
      }
    }
    for (int i = 0; i < se.n; ++i) p->event_pool.push_back(se.ev[i]);
  }
  p->pending.clear();
  if (out)
    for (int sidx = 0; sidx < NFFT_STAGES && 2 * sidx + 1 < n; ++sidx) {
      out[2 * sidx] = p->stage_ms[sidx];
      out[2 * sidx + 1] = (double)p->stage_calls[sidx];
    }
  if (reset)
    for (int sidx = 0; sidx < NFFT_STAGES; ++sidx) {
      p->stage_ms[sidx] = 0;
      p->stage_calls[sidx] = 0;
    }
  return NFFT_OK;
}

}  // extern "C"
