// Spreading for d = 2 on the matrix cores (float32 and float64), the nodes
// of a work item taken one tile row at a time (Algorithm 2.4 step 1 with the
// weights of (3.7)).
//
// A node in tile row r (tile-local cell (r, l1)) reaches the padded rows
// r .. r + 2m of the item's padded tile (P = 16 + 2m rows and columns): row
// r only for a node on a grid line (closed edge), rows r+1 .. r+2m with the
// window factors a_0 .. a_{2m-1}. For 2m + 1 <= 16 the nodes of one tile row
// therefore update a block of 16 rows x 32 padded columns,
//     G[i][c] += sum_n A_n[i] B_n[c] c_n,
// a product whose inner dimension runs over the nodes. v_mfma_f32_16x16x4f32
// (v_mfma_f64_16x16x4f64 in float64) takes four nodes at a time: lane (k, i) supplies A_k[i] (row factor times
// the real or the imaginary part of c_k = w_k f_k) and B_k[i] (column
// factor), and four operations per four nodes cover the two column blocks
// (padded columns 0..15 and 16..31) times the real and imaginary parts.
// The accumulator rows are slots: slot s holds the padded row congruent to s
// modulo 16 within the block of the current tile row, so the block of row
// r + 1 reuses the slots of row r shifted by one; after the nodes of row r
// the slot of padded row r is complete, is written to the wave's tile in LDS
// and cleared, and takes padded row r + 16 from then on. The window factors
// are evaluated per call: lane (k, p) evaluates polynomial p at node k's two
// offsets, and ds_bpermute moves the values to the slots and columns that
// need them. Nodes of a tile are sorted by row at plan time; the groups of
// four of all rows are dealt to the waves in turn. At the end the waves'
// tiles are summed in LDS in wave order (the result does not depend on
// timing) and the padded tile is written out like the other kernels' (the
// split-tile sums and the first FFT pass merge them).
#include "spread_common.hpp"

namespace nfft {

namespace {

// Per precision: the accumulator block of v_mfma_*_16x16x4 (four elements a
// lane, column l & 15 of the 16 x 16 block; row 4 (l >> 4) + v for element v
// of lane l in float32, row 4 v + (l >> 4) in float64), the operation, and a
// lane read.
template <typename R> struct MmaT;
template <> struct MmaT<float> {
  static constexpr bool kRowsByQuarter = true;  // row 4 (l >> 4) + v
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mfma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ float read(float v, int byte_addr) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(byte_addr, __float_as_int(v)));
  }
};
template <> struct MmaT<double> {
  static constexpr bool kRowsByQuarter = false;  // row 4 v + (l >> 4)
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

// y0, y1, Re c, Im c of a staged node
template <typename R> struct alignas(4 * sizeof(R)) MmaNode {
  R y0, y1, cx, cy;
};

}  // namespace

// Nodes staged per batch (a work item of up to 512 nodes in one batch).
constexpr int kMmaBatch = 512;

template <typename R, int MW, int NW>
struct MmaLds {
  static constexpr int P = 16 + 2 * MW;
  // staging, NB + 1 entries (the last one a node with c = 0 for the missing
  // members of a row's last group): offsets and c_j; the closed-edge factors
  // of the row and the column; the column shift and the tile row in one
  // word; the first node of every tile row in the batch (17 entries, 32
  // reserved); rounded up to 16 bytes. In float32 four work-groups of four
  // waves fit in a compute unit's LDS for m <= 6.
  static constexpr size_t staging =
      ((size_t)(kMmaBatch + 1) * (6 * sizeof(R) + 4) + 32 * 4 + 15) / 16 * 16;
  // one padded tile per wave
  static constexpr size_t tiles = (size_t)NW * P * P * sizeof(cplx<R>);
  static constexpr size_t bytes = staging + tiles;
};

template <typename R, int MW, int NW>
__global__ __launch_bounds__(64 * NW) void spread_mma_kernel(SpreadArgs<R> a) {
  constexpr int K2 = 2 * MW;
  constexpr int P = 16 + K2;
  constexpr int NT = 64 * NW;
  constexpr int NB = kMmaBatch;
  constexpr int DEG = PolyDeg<R>::value;
  typedef typename MmaT<R>::v4 v4;
  constexpr bool QR = MmaT<R>::kRowsByQuarter;
  static_assert(K2 + 1 <= 16, "the rows of one tile row's nodes fit in 16 slots");
  static_assert((P * P) % 2 == 0 && P % 2 == 0, "tiles are summed two cells at a time");
  extern __shared__ double lds_d[];
  MmaNode<R>* st_n = reinterpret_cast<MmaNode<R>*>(lds_d);
  cplx<R>* st_e = reinterpret_cast<cplx<R>*>(st_n + (NB + 1));  // edge factors (0 off a grid line)
  int* st_q = reinterpret_cast<int*>(st_e + (NB + 1));          // -(l1 + 1) in bits 0-15, tile row above
  int* st_rs = st_q + (NB + 1);                                  // row starts [17]
  cplx<R>* tiles = reinterpret_cast<cplx<R>*>(
      reinterpret_cast<char*>(lds_d) + MmaLds<R, MW, NW>::staging);  // [NW][P][P]

  const int item = blockIdx.x;
  const int rhs = blockIdx.y;
  const int tid = threadIdx.x;
  // wave-uniform, so that the group loop below is a scalar branch
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int kq = lane >> 4;       // node of the group of four; accumulator row quarter
  const int j = lane & 15;        // slot (A), column in a block (B), polynomial (Horner)
  const int lrow = lane & 48;     // first lane of this lane's 16-lane row
  const int pc = j < K2 ? j : K2 - 1;
  const bool hi_in = 16 + j < P;  // padded column 16 + j exists

  R cf[DEG + 1];
#pragma unroll
  for (int q = 0; q <= DEG; ++q) cf[q] = a.coef[pc * (DEG + 1) + q];

  v4 acc0r = {(R)0, (R)0, (R)0, (R)0}, acc0i = acc0r, acc1r = acc0r, acc1i = acc0r;
  cplx<R>* mine = tiles + wave * (P * P);

  const int64_t N = a.g.N;
  const int start = a.item_start[item];
  const int cnt = a.item_count[item];
  const cplx<R>* f = a.f + rhs * a.f_rs;
  const R edge = a.edge;

  if (tid == 0) {
    // the node with c = 0: its products are zero whatever its (finite)
    // window factors
    st_n[NB] = MmaNode<R>{(R)0, (R)0, (R)0, (R)0};
    st_e[NB] = mkc<R>(0, 0);
    st_q[NB] = 0xffff;
  }
  for (int b0 = 0; b0 < cnt; b0 += NB) {
    const int nb = (cnt - b0) < NB ? (cnt - b0) : NB;
    const bool first = b0 == 0;
    __syncthreads();  // the previous batch is consumed
#pragma unroll 2
    for (int t = tid; t < nb; t += NT) {
      const int i = start + b0 + t;
      const cplx<R> wv = a.w[i];
      const cplx<R> fv = f[a.perm[i]];
      const uint32_t L = a.loc[i];
      st_n[t] = MmaNode<R>{(R)2 * a.frac[i] - (R)1, (R)2 * a.frac[N + i] - (R)1,
                           wv.x * fv.x - wv.y * fv.y, wv.x * fv.y + wv.y * fv.x};
      st_e[t] = mkc<R>(((L >> kEdgeShift) & 1u) ? edge : (R)0,
                       ((L >> (kEdgeShift + 1)) & 1u) ? edge : (R)0);
      st_q[t] = ((-(int)((L >> kLocBits) & kLocMask) - 1) & 0xffff) | (int)((L & kLocMask) << 16);
    }
    __syncthreads();
    // first node of each tile row (the batch is sorted by row): node t opens
    // the rows after its predecessor's up to its own; the last node closes
    // the rest
    for (int t = tid; t < nb; t += NT) {
      const int rt = st_q[t] >> 16;
      const int rp = t > 0 ? st_q[t - 1] >> 16 : -1;
      for (int r = rp + 1; r <= rt; ++r) st_rs[r] = t;
      if (t == nb - 1)
        for (int r = rt + 1; r <= 16; ++r) st_rs[r] = nb;
    }
    __syncthreads();

    // groups of four consecutive nodes within each row; the groups of all
    // rows are numbered in row order and wave w takes groups w, w + NW, ...
    int gbase = 0;  // groups of the rows before r
    static_for<0, 16>([&](auto rc) {
      constexpr int r = decltype(rc)::value;
      const int n0 = __builtin_amdgcn_readfirstlane(st_rs[r]);
      const int n1 = __builtin_amdgcn_readfirstlane(st_rs[r + 1]);
      const int ng = (n1 - n0 + 3) >> 2;
      // slot j holds padded row r + sA: the closed-edge row (sA = 0), window
      // row sA - 1 (sA = 1 .. 2m) or nothing
      const int sA = (j - r) & 15;
      const bool inA = sA >= 1 && sA <= K2;
      const bool edA = sA == 0;
      const int addrA = (lrow | ((sA - 1) & 15)) << 2;
      int q = wave - gbase % NW;
      q = q < 0 ? q + NW : q;
      for (; q < ng; q += NW) {
        const int n = n0 + 4 * q + kq;
        const int nn = n < n1 ? n : NB;  // past the row: the node with c = 0
        const MmaNode<R> nd = st_n[nn];
        const cplx<R> ne = st_e[nn];
        const int qoff = (st_q[nn] << 16) >> 16;
        const R h0 = horner<R>(cf, nd.y0);
        const R h1 = horner<R>(cf, nd.y1);
        // row factor of slot j, column factors of padded columns j and 16 + j
        const R ra = MmaT<R>::read(h0, addrA);
        const int qB = j + qoff;
        const R cb = MmaT<R>::read(h1, (lrow | (qB & 15)) << 2);
        const R A = inA ? ra : (edA ? ne.x : (R)0);
        const R B0 = (unsigned)qB < (unsigned)K2 ? cb : (qB == -1 ? ne.y : (R)0);
        const R B1 = qB < K2 - 16 ? cb : (R)0;
        const R ar = A * nd.cx;
        const R ai = A * nd.cy;
        acc0r = MmaT<R>::mfma(ar, B0, acc0r);
        acc1r = MmaT<R>::mfma(ar, B1, acc1r);
        acc0i = MmaT<R>::mfma(ai, B0, acc0i);
        acc1i = MmaT<R>::mfma(ai, B1, acc1i);
      }
      gbase += ng;
      // padded row r is complete for this wave: slot r (accumulator element
      // v of lane l is slot 4 (l >> 4) + v in float32, 4 v + (l >> 4) in
      // float64; column l & 15 of its block)
      constexpr int v = QR ? (r & 3) : (r >> 2);
      const bool done = kq == (QR ? (r >> 2) : (r & 3));
      cplx<R> lo = mkc<R>(acc0r[v], acc0i[v]);
      cplx<R> hi = mkc<R>(acc1r[v], acc1i[v]);
      if (done) {
        cplx<R>* rowp = mine + r * P;
        if (!first) {
          const cplx<R> u = rowp[j];
          lo.x += u.x;
          lo.y += u.y;
          if (hi_in) {
            const cplx<R> w = rowp[16 + j];
            hi.x += w.x;
            hi.y += w.y;
          }
        }
        rowp[j] = lo;
        if (hi_in) rowp[16 + j] = hi;
      }
      // only element v of the finished quarter is cleared (a select, so that
      // the other accumulator elements stay where they are)
      acc0r[v] = done ? (R)0 : acc0r[v];
      acc0i[v] = done ? (R)0 : acc0i[v];
      acc1r[v] = done ? (R)0 : acc1r[v];
      acc1i[v] = done ? (R)0 : acc1i[v];
    });
    // padded rows 16 .. P-1: slot s holds padded row 16 + s
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 + (QR ? 4 * kq + v : 4 * v + kq);
      if (row < P) {
        cplx<R>* rowp = mine + row * P;
        cplx<R> lo = mkc<R>(acc0r[v], acc0i[v]);
        cplx<R> hi = mkc<R>(acc1r[v], acc1i[v]);
        if (!first) {
          const cplx<R> u = rowp[j];
          lo.x += u.x;
          lo.y += u.y;
          if (hi_in) {
            const cplx<R> w = rowp[16 + j];
            hi.x += w.x;
            hi.y += w.y;
          }
        }
        rowp[j] = lo;
        if (hi_in) rowp[16 + j] = hi;
      }
    }
    acc0r = v4{(R)0, (R)0, (R)0, (R)0};
    acc0i = acc0r;
    acc1r = acc0r;
    acc1i = acc0r;
  }

  // the waves' tiles summed in wave order: a fixed order, so the result does
  // not depend on timing (float32: two cells at a time)
  __syncthreads();
  const int slot = a.item_slot[item];
  cplx<R>* out = slot < 0 ? a.tilep + rhs * a.tile_rs + (int64_t)a.item_bin[item] * (P * P)
                          : a.itemp + rhs * a.item_rs + (int64_t)slot * (P * P);
  if constexpr (std::is_same<R, float>::value) {
    const float4* t4 = reinterpret_cast<const float4*>(tiles);
    float4* o4 = reinterpret_cast<float4*>(out);
    for (int i = tid; i < P * P / 2; i += NT) {
      float4 s = t4[i];
#pragma unroll
      for (int w = 1; w < NW; ++w) {
        const float4 u = t4[w * (P * P / 2) + i];
        s.x += u.x;
        s.y += u.y;
        s.z += u.z;
        s.w += u.w;
      }
      o4[i] = s;
    }
  } else {
    for (int i = tid; i < P * P; i += NT) {
      cplx<R> s = tiles[i];
#pragma unroll
      for (int w = 1; w < NW; ++w) {
        const cplx<R> u = tiles[w * (P * P) + i];
        s.x += u.x;
        s.y += u.y;
      }
      out[i] = s;
    }
  }
}

bool spread_mma_supported(int d, int T, bool f64, int m) {
  (void)f64;  // float32 and float64
  return d == 2 && T == 16 && m >= 1 && 2 * m + 1 <= 16;
}

// 64 or 128 threads: two waves; 256: four; 512: eight
static int mma_waves(int nt) { return nt >= 512 ? 8 : nt >= 256 ? 4 : 2; }

template <typename R, int MW>
static size_t mma_lds_m(int nw) {
  return nw == 8 ? MmaLds<R, MW, 8>::bytes
                 : nw == 4 ? MmaLds<R, MW, 4>::bytes : MmaLds<R, MW, 2>::bytes;
}

template <typename R>
static size_t mma_lds(int m, int nw) {
  switch (m) {
    case 1: return mma_lds_m<R, 1>(nw);
    case 2: return mma_lds_m<R, 2>(nw);
    case 3: return mma_lds_m<R, 3>(nw);
    case 4: return mma_lds_m<R, 4>(nw);
    case 5: return mma_lds_m<R, 5>(nw);
    case 6: return mma_lds_m<R, 6>(nw);
    case 7: return mma_lds_m<R, 7>(nw);
    default: return 0;
  }
}

size_t spread_mma_lds_bytes(int m, int nt, bool f64) {
  const int nw = mma_waves(nt);
  return f64 ? mma_lds<double>(m, nw) : mma_lds<float>(m, nw);
}

template <typename R, int MW>
static hipError_t spread_mma_m(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  const dim3 grid(a.g.nsub, nrhs);
  const int nw = mma_waves(a.nt);
  if (nw == 8)
    hipLaunchKernelGGL((spread_mma_kernel<R, MW, 8>), grid, dim3(512), (MmaLds<R, MW, 8>::bytes),
                       s, a);
  else if (nw == 4)
    hipLaunchKernelGGL((spread_mma_kernel<R, MW, 4>), grid, dim3(256), (MmaLds<R, MW, 4>::bytes),
                       s, a);
  else
    hipLaunchKernelGGL((spread_mma_kernel<R, MW, 2>), grid, dim3(128), (MmaLds<R, MW, 2>::bytes),
                       s, a);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_spread_mma(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  if (!spread_mma_supported(a.g.d, a.g.T, !std::is_same<R, float>::value, a.g.m))
    return hipErrorInvalidValue;
  if (a.g.nsub == 0) return hipSuccess;
  switch (a.g.m) {
    case 1: return spread_mma_m<R, 1>(a, nrhs, s);
    case 2: return spread_mma_m<R, 2>(a, nrhs, s);
    case 3: return spread_mma_m<R, 3>(a, nrhs, s);
    case 4: return spread_mma_m<R, 4>(a, nrhs, s);
    case 5: return spread_mma_m<R, 5>(a, nrhs, s);
    case 6: return spread_mma_m<R, 6>(a, nrhs, s);
    case 7: return spread_mma_m<R, 7>(a, nrhs, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_spread_mma<float>(const SpreadArgs<float>&, int, hipStream_t);
template hipError_t launch_spread_mma<double>(const SpreadArgs<double>&, int, hipStream_t);

}  // namespace nfft
