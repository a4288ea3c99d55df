// Spreading for d = 3 on the matrix cores, float32 and float64 (Algorithm
// 2.4 step 1 with the weights of (3.7)), tile edge 8 and 2m <= 8, so that
// the padded tile of a work item (P = 8 + 2m <= 16 cells per dimension) fits
// in the accumulators of one wave: plane i0 of the padded tile is one
// 16 x 16 block (rows i1, columns i2) of v_mfma_f32_16x16x4f32 (float64:
// v_mfma_f64_16x16x4f64) accumulators, real and imaginary part, 2P blocks in
// all.
//
// A node at tile-local cell (l0, l1, l2) reaches the padded cells
// (l0 + 1 + p0, l1 + 1 + p1, l2 + 1 + p2), p_t < 2m, with the window factors
// a(p0) b(p1) e(p2), and on a grid plane of dimension t also the closed-edge
// cell l_t of that dimension. For one plane i0 = l0 + 1 + p0 the update is
//     G[i0][i1][i2] += sum_n (a_n(p0) b_n[i1] c_n) e_n[i2],
// a product whose inner dimension runs over the nodes: four nodes of the
// same tile row l0 = r at a time, lane (k, i) supplies A_k[i] = b_k[i] c_k
// (real or imaginary part) and B_k[i] = a_k(p0) e_k[i], two operations per
// plane. The planes a tile row reaches are compile-time constants (the
// nodes of a tile are sorted by l0 at plan time and the node loop runs
// inside an unrolled loop over the 8 tile rows and the 2m planes). Lane
// (k, p) of a node's 16-lane row evaluates window polynomial p at the
// node's dimension-0 and dimension-1 offsets, lane (k, 8 + p) at its
// dimension-2 offset; a_k(p0) reaches the lanes of node k by a DPP row
// broadcast, b_k and e_k by ds_bpermute.
// The padded tile is written out like the other kernels' (the split-tile
// sums and the first FFT pass merge the tiles).
#include "spread_common.hpp"

namespace nfft {

namespace {

// Per precision: the accumulator block (four elements a lane, column l & 15;
// row 4 (l >> 4) + v for element v of lane l in float32, 4 v + (l >> 4) in
// float64), the operation, a lane read and the staged node.
template <typename R> struct Mma3T;
template <> struct Mma3T<float> {
  static constexpr bool kRowsByQuarter = true;
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mfma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ float read(float v, int byte_addr) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(byte_addr, __float_as_int(v)));
  }
};
template <> struct Mma3T<double> {
  static constexpr bool kRowsByQuarter = false;
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mfma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ double read(double v, int byte_addr) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(byte_addr, (int)(u & 0xffffffffLL));
    const int hi = __builtin_amdgcn_ds_bpermute(byte_addr, (int)(u >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  }
};

// node b: y0, y1, y2, Re c, Im c, edge factor of dimension 1 and of
// dimension 2 (0 off a grid plane), and a word: -(l1 + 1) in bits 0-7,
// -(l2 + 1) in bits 8-15, the edge flag of dimension 0 in bit 16, l0 from
// bit 20
template <typename R> struct alignas(8 * sizeof(R)) Mma3Node {
  R y0, y1, y2, cx, cy, e1, e2;
  int bits;
};

// sign-extended 8-bit field
__device__ __forceinline__ int sext8(int v) { return (v << 24) >> 24; }

}  // namespace

// Nodes staged per batch; one wave per work item.
constexpr int k3MmaBatch = 256;
constexpr int k3MmaT = 8;

template <typename R, int MW>
__global__ __launch_bounds__(64) void spread3_mma_kernel(SpreadArgs<R> a) {
  constexpr int K2 = 2 * MW;
  constexpr int T = k3MmaT;
  constexpr int P = T + K2;
  constexpr int NB = k3MmaBatch;
  constexpr int DEG = PolyDeg<R>::value;
  typedef typename Mma3T<R>::v4 v4;
  constexpr bool QR = Mma3T<R>::kRowsByQuarter;
  static_assert(P <= 16, "a plane of the padded tile is one 16 x 16 block");
  // the staged nodes; entry NB is a node with c = 0 for the missing members
  // of a row's last group
  __shared__ Mma3Node<R> st[NB + 1];
  __shared__ int st_rs[T + 1];

  const int item = blockIdx.x;
  const int rhs = blockIdx.y;
  const int lane = threadIdx.x;
  const int kq = lane >> 4;    // node of the group of four; accumulator row quarter
  const int j = lane & 15;     // row i1 (A), column i2 (B), polynomial (Horner)
  const int lrow = lane & 48;  // first lane of this lane's 16-lane row
  const int pc = (j & 7) < K2 ? (j & 7) : K2 - 1;
  const bool lo8 = j < 8;

  R cf[DEG + 1];
#pragma unroll
  for (int q = 0; q <= DEG; ++q) cf[q] = a.coef[pc * (DEG + 1) + q];

  v4 acc[P][2];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    acc[i][0] = v4{(R)0, (R)0, (R)0, (R)0};
    acc[i][1] = acc[i][0];
  }

  const int64_t N = a.g.N;
  const int start = a.item_start[item];
  const int cnt = a.item_count[item];
  const cplx<R>* f = a.f + rhs * a.f_rs;
  const R edge = a.edge;

  if (lane == 0) st[NB] = Mma3Node<R>{(R)0, (R)0, (R)0, (R)0, (R)0, (R)0, (R)0, 0};
  for (int b0 = 0; b0 < cnt; b0 += NB) {
    const int nb = (cnt - b0) < NB ? (cnt - b0) : NB;
    __syncthreads();  // the previous batch is consumed
    // two nodes a lane per step, so that their loads are in flight together
#pragma unroll 2
    for (int t = lane; t < nb; t += 64) {
      const int i = start + b0 + t;
      const cplx<R> wv = a.w[i];
      const cplx<R> fv = f[a.perm[i]];
      const uint32_t L = a.loc[i];
      const int l0 = (int)(L & kLocMask);
      const int l1 = (int)((L >> kLocBits) & kLocMask);
      const int l2 = (int)((L >> (2 * kLocBits)) & kLocMask);
      st[t] = Mma3Node<R>{(R)2 * a.frac[i] - (R)1, (R)2 * a.frac[N + i] - (R)1,
                          (R)2 * a.frac[2 * N + i] - (R)1, wv.x * fv.x - wv.y * fv.y,
                          wv.x * fv.y + wv.y * fv.x,
                          ((L >> (kEdgeShift + 1)) & 1u) ? edge : (R)0,
                          ((L >> (kEdgeShift + 2)) & 1u) ? edge : (R)0,
                          ((-(l1 + 1)) & 0xff) | (((-(l2 + 1)) & 0xff) << 8) |
                              (int)(((L >> kEdgeShift) & 1u) << 16) | (l0 << 20)};
    }
    __syncthreads();
    // first node of each tile row (the batch is sorted by l0)
    for (int t = lane; t < nb; t += 64) {
      const int rt = st[t].bits >> 20;
      const int rp = t > 0 ? st[t - 1].bits >> 20 : -1;
      for (int r = rp + 1; r <= rt; ++r) st_rs[r] = t;
      if (t == nb - 1)
        for (int r = rt + 1; r <= T; ++r) st_rs[r] = nb;
    }
    __syncthreads();

    static_for<0, T>([&](auto rc) {
      constexpr int r = decltype(rc)::value;
      const int n0 = __builtin_amdgcn_readfirstlane(st_rs[r]);
      const int n1 = __builtin_amdgcn_readfirstlane(st_rs[r + 1]);
      for (int g = n0; g < n1; g += 4) {
        const int n = g + kq;
        const bool valid = n < n1;
        const Mma3Node<R> nd = st[valid ? n : NB];
        const int bits = nd.bits;
        const int q1 = j + sext8(bits & 0xff);         // window cell of row i1 = j
        const int q2 = j + sext8((bits >> 8) & 0xff);  // window cell of column i2 = j
        // lanes p < 8: polynomial p at y0 (hA) and y1 (hB); lanes 8 + p: at y2 (hA)
        const R hA = horner<R>(cf, lo8 ? nd.y0 : nd.y2);
        const R hB = horner<R>(cf, nd.y1);
        const R v1 = Mma3T<R>::read(hB, (lrow | (q1 & 7)) << 2);
        const R v2 = Mma3T<R>::read(hA, (lrow | 8 | (q2 & 7)) << 2);
        const R b1 = (unsigned)q1 < (unsigned)K2 ? v1 : (q1 == -1 ? nd.e1 : (R)0);
        const R e2 = (unsigned)q2 < (unsigned)K2 ? v2 : (q2 == -1 ? nd.e2 : (R)0);
        const R ur = b1 * nd.cx;
        const R ui = b1 * nd.cy;
        static_for<0, K2>([&](auto pc_) {
          constexpr int p = decltype(pc_)::value;
          const R bp = row_bcast<p>(hA) * e2;  // a_kq(p) e_kq[i2]
          acc[r + 1 + p][0] = Mma3T<R>::mfma(ur, bp, acc[r + 1 + p][0]);
          acc[r + 1 + p][1] = Mma3T<R>::mfma(ui, bp, acc[r + 1 + p][1]);
        });
        // closed-edge plane r of nodes on a grid plane of dimension 0
        const bool e0 = valid && ((bits >> 16) & 1);
        if (__builtin_amdgcn_ballot_w64(e0)) {
          const R be = e0 ? edge * e2 : (R)0;
          acc[r][0] = Mma3T<R>::mfma(ur, be, acc[r][0]);
          acc[r][1] = Mma3T<R>::mfma(ui, be, acc[r][1]);
        }
      }
    });
  }

  // accumulator element v of lane l: row i1 = 4 (l >> 4) + v (float64:
  // 4 v + (l >> 4)), column i2 = l & 15
  const int slot = a.item_slot[item];
  constexpr int Ptot = P * P * P;
  cplx<R>* out = slot < 0 ? a.tilep + rhs * a.tile_rs + (int64_t)a.item_bin[item] * Ptot
                          : a.itemp + rhs * a.item_rs + (int64_t)slot * Ptot;
#pragma unroll
  for (int i0 = 0; i0 < P; ++i0)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i1 = QR ? 4 * kq + v : 4 * v + kq;
      if (i1 < P && j < P) out[(i0 * P + i1) * P + j] = mkc<R>(acc[i0][0][v], acc[i0][1][v]);
    }
}

bool spread3_mma_supported(int d, int T, bool f64, int m) {
  (void)f64;  // float32 and float64
  return d == 3 && T == k3MmaT && m >= 1 && k3MmaT + 2 * m <= 16;
}

// the kernel's staging arrays (static LDS)
size_t spread3_mma_lds_bytes(bool f64) {
  return (size_t)(k3MmaBatch + 1) * (f64 ? sizeof(Mma3Node<double>) : sizeof(Mma3Node<float>)) +
         (k3MmaT + 1) * sizeof(int);
}

template <typename R>
hipError_t launch_spread3_mma(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  if (!spread3_mma_supported(a.g.d, a.g.T, !std::is_same<R, float>::value, a.g.m))
    return hipErrorInvalidValue;
  if (a.g.nsub == 0) return hipSuccess;
  const dim3 grid(a.g.nsub, nrhs);
  switch (a.g.m) {
    case 1: hipLaunchKernelGGL((spread3_mma_kernel<R, 1>), grid, dim3(64), 0, s, a); break;
    case 2: hipLaunchKernelGGL((spread3_mma_kernel<R, 2>), grid, dim3(64), 0, s, a); break;
    case 3: hipLaunchKernelGGL((spread3_mma_kernel<R, 3>), grid, dim3(64), 0, s, a); break;
    case 4: hipLaunchKernelGGL((spread3_mma_kernel<R, 4>), grid, dim3(64), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_spread3_mma<float>(const SpreadArgs<float>&, int, hipStream_t);
template hipError_t launch_spread3_mma<double>(const SpreadArgs<double>&, int, hipStream_t);

}  // namespace nfft
