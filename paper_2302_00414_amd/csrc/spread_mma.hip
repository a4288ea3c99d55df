// Spreading for d = 2 in float32 on the matrix cores, the nodes of a work
// item taken one tile row at a time (Algorithm 2.4 step 1 with the weights
// of (3.7)).
//
// A node in tile row r (tile-local cell (r, l1)) reaches the padded rows
// r .. r + 2m of the item's padded tile (P = 16 + 2m rows and columns): row
// r only for a node on a grid line (closed edge), rows r+1 .. r+2m with the
// window factors a_0 .. a_{2m-1}. For 2m + 1 <= 16 the nodes of one tile row
// therefore update a block of 16 rows x 32 padded columns,
//     G[i][c] += sum_n A_n[i] B_n[c] c_n,
// a product whose inner dimension runs over the nodes. v_mfma_f32_16x16x4f32
// takes four nodes at a time: lane (k, i) supplies A_k[i] (row factor times
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

typedef float mma_v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float lane_read(float v, int byte_addr) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(byte_addr, __float_as_int(v)));
}

}  // namespace

// Nodes staged per batch (a work item of up to 512 nodes in one batch).
constexpr int kMmaBatch = 512;

template <int MW, int NW>
struct MmaLds {
  static constexpr int P = 16 + 2 * MW;
  // staging, NB + 1 entries (the last one a node with c = 0 for the missing
  // members of a row's last group): offsets and c_j as one float4; the
  // closed-edge factors of the row and the column; the column shift and the
  // tile row in one word; the first node of every tile row in the batch (17
  // entries, 32 reserved); rounded up to 16 bytes. Four work-groups of four
  // waves fit in a compute unit's LDS for m <= 6.
  static constexpr size_t staging = ((size_t)(kMmaBatch + 1) * 28 + 32 * 4 + 15) / 16 * 16;
  // one padded tile per wave
  static constexpr size_t tiles = (size_t)NW * P * P * sizeof(float2);
  static constexpr size_t bytes = staging + tiles;
};

template <int MW, int NW>
__global__ __launch_bounds__(64 * NW) void spread_mma_kernel(SpreadArgs<float> a) {
  constexpr int K2 = 2 * MW;
  constexpr int P = 16 + K2;
  constexpr int NT = 64 * NW;
  constexpr int NB = kMmaBatch;
  constexpr int DEG = PolyDeg<float>::value;
  static_assert(K2 + 1 <= 16, "the rows of one tile row's nodes fit in 16 slots");
  static_assert((P * P) % 2 == 0 && P % 2 == 0, "tiles are summed two cells at a time");
  extern __shared__ float lds_f[];
  float4* st_n = reinterpret_cast<float4*>(lds_f);  // y0, y1, Re c, Im c
  float2* st_e = reinterpret_cast<float2*>(st_n + (NB + 1));  // edge factors (0 off a grid line)
  int* st_q = reinterpret_cast<int*>(st_e + (NB + 1));        // -(l1 + 1) in bits 0-15, tile row above
  int* st_rs = st_q + (NB + 1);                                // row starts [17]
  float2* tiles = reinterpret_cast<float2*>(
      reinterpret_cast<char*>(lds_f) + MmaLds<MW, NW>::staging);  // [NW][P][P]

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

  float cf[DEG + 1];
#pragma unroll
  for (int q = 0; q <= DEG; ++q) cf[q] = a.coef[pc * (DEG + 1) + q];

  mma_v4f acc0r = {0.0f, 0.0f, 0.0f, 0.0f}, acc0i = acc0r, acc1r = acc0r, acc1i = acc0r;
  float2* mine = tiles + wave * (P * P);

  const int64_t N = a.g.N;
  const int start = a.item_start[item];
  const int cnt = a.item_count[item];
  const float2* f = a.f + rhs * a.f_rs;
  const float edge = a.edge;

  if (tid == 0) {
    // the node with c = 0: its products are zero whatever its (finite)
    // window factors
    st_n[NB] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    st_e[NB] = make_float2(0.0f, 0.0f);
    st_q[NB] = 0xffff;
  }
  for (int b0 = 0; b0 < cnt; b0 += NB) {
    const int nb = (cnt - b0) < NB ? (cnt - b0) : NB;
    const bool first = b0 == 0;
    __syncthreads();  // the previous batch is consumed
#pragma unroll 2
    for (int t = tid; t < nb; t += NT) {
      const int i = start + b0 + t;
      const float2 wv = a.w[i];
      const float2 fv = f[a.perm[i]];
      const uint32_t L = a.loc[i];
      st_n[t] = make_float4(2.0f * a.frac[i] - 1.0f, 2.0f * a.frac[N + i] - 1.0f,
                            wv.x * fv.x - wv.y * fv.y, wv.x * fv.y + wv.y * fv.x);
      st_e[t] = make_float2(((L >> kEdgeShift) & 1u) ? edge : 0.0f,
                            ((L >> (kEdgeShift + 1)) & 1u) ? edge : 0.0f);
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
        const float4 nd = st_n[nn];
        const float2 ne = st_e[nn];
        const int qoff = (st_q[nn] << 16) >> 16;
        const float h0 = horner<float>(cf, nd.x);
        const float h1 = horner<float>(cf, nd.y);
        // row factor of slot j, column factors of padded columns j and 16 + j
        const float ra = lane_read(h0, addrA);
        const int qB = j + qoff;
        const float cb = lane_read(h1, (lrow | (qB & 15)) << 2);
        const float A = inA ? ra : (edA ? ne.x : 0.0f);
        const float B0 = (unsigned)qB < (unsigned)K2 ? cb : (qB == -1 ? ne.y : 0.0f);
        const float B1 = qB < K2 - 16 ? cb : 0.0f;
        const float ar = A * nd.z;
        const float ai = A * nd.w;
        acc0r = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, B0, acc0r, 0, 0, 0);
        acc1r = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, B1, acc1r, 0, 0, 0);
        acc0i = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, B0, acc0i, 0, 0, 0);
        acc1i = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, B1, acc1i, 0, 0, 0);
      }
      gbase += ng;
      // padded row r is complete for this wave: slot r, element r % 4 of the
      // lanes of row quarter r / 4 (accumulator element v of lane l is slot
      // 4 (l >> 4) + v, column l & 15 of its block)
      constexpr int v = r & 3;
      const bool done = kq == (r >> 2);
      float2 lo = make_float2(acc0r[v], acc0i[v]);
      float2 hi = make_float2(acc1r[v], acc1i[v]);
      if (done) {
        float2* rowp = mine + r * P;
        if (!first) {
          const float2 u = rowp[j];
          lo.x += u.x;
          lo.y += u.y;
          if (hi_in) {
            const float2 w = rowp[16 + j];
            hi.x += w.x;
            hi.y += w.y;
          }
        }
        rowp[j] = lo;
        if (hi_in) rowp[16 + j] = hi;
      }
      // only element v of the finished quarter is cleared (a select, so that
      // the other accumulator elements stay where they are)
      acc0r[v] = done ? 0.0f : acc0r[v];
      acc0i[v] = done ? 0.0f : acc0i[v];
      acc1r[v] = done ? 0.0f : acc1r[v];
      acc1i[v] = done ? 0.0f : acc1i[v];
    });
    // padded rows 16 .. P-1: slot s holds padded row 16 + s
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 + 4 * kq + v;
      if (row < P) {
        float2* rowp = mine + row * P;
        float2 lo = make_float2(acc0r[v], acc0i[v]);
        float2 hi = make_float2(acc1r[v], acc1i[v]);
        if (!first) {
          const float2 u = rowp[j];
          lo.x += u.x;
          lo.y += u.y;
          if (hi_in) {
            const float2 w = rowp[16 + j];
            hi.x += w.x;
            hi.y += w.y;
          }
        }
        rowp[j] = lo;
        if (hi_in) rowp[16 + j] = hi;
      }
    }
    acc0r = mma_v4f{0.0f, 0.0f, 0.0f, 0.0f};
    acc0i = acc0r;
    acc1r = acc0r;
    acc1i = acc0r;
  }

  // the waves' tiles summed in wave order, two cells at a time: a fixed
  // order, so the result does not depend on timing
  __syncthreads();
  const int slot = a.item_slot[item];
  float2* out = slot < 0 ? a.tilep + rhs * a.tile_rs + (int64_t)a.item_bin[item] * (P * P)
                         : a.itemp + rhs * a.item_rs + (int64_t)slot * (P * P);
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
}

bool spread_mma_supported(int d, int T, bool f64, int m) {
  return d == 2 && T == 16 && !f64 && m >= 1 && 2 * m + 1 <= 16;
}

// 64 or 128 threads: two waves; 256: four; 512: eight
static int mma_waves(int nt) { return nt >= 512 ? 8 : nt >= 256 ? 4 : 2; }

template <int MW>
static size_t mma_lds_m(int nw) {
  return nw == 8 ? MmaLds<MW, 8>::bytes : nw == 4 ? MmaLds<MW, 4>::bytes : MmaLds<MW, 2>::bytes;
}

size_t spread_mma_lds_bytes(int m, int nt) {
  const int nw = mma_waves(nt);
  switch (m) {
    case 1: return mma_lds_m<1>(nw);
    case 2: return mma_lds_m<2>(nw);
    case 3: return mma_lds_m<3>(nw);
    case 4: return mma_lds_m<4>(nw);
    case 5: return mma_lds_m<5>(nw);
    case 6: return mma_lds_m<6>(nw);
    case 7: return mma_lds_m<7>(nw);
    default: return 0;
  }
}

template <int MW>
static hipError_t spread_mma_m(const SpreadArgs<float>& a, int nrhs, hipStream_t s) {
  const dim3 grid(a.g.nsub, nrhs);
  const int nw = mma_waves(a.nt);
  if (nw == 8)
    hipLaunchKernelGGL((spread_mma_kernel<MW, 8>), grid, dim3(512), (MmaLds<MW, 8>::bytes), s, a);
  else if (nw == 4)
    hipLaunchKernelGGL((spread_mma_kernel<MW, 4>), grid, dim3(256), (MmaLds<MW, 4>::bytes), s, a);
  else
    hipLaunchKernelGGL((spread_mma_kernel<MW, 2>), grid, dim3(128), (MmaLds<MW, 2>::bytes), s, a);
  return hipGetLastError();
}

hipError_t launch_spread_mma(const SpreadArgs<float>& a, int nrhs, hipStream_t s) {
  if (!spread_mma_supported(a.g.d, a.g.T, false, a.g.m)) return hipErrorInvalidValue;
  if (a.g.nsub == 0) return hipSuccess;
  switch (a.g.m) {
    case 1: return spread_mma_m<1>(a, nrhs, s);
    case 2: return spread_mma_m<2>(a, nrhs, s);
    case 3: return spread_mma_m<3>(a, nrhs, s);
    case 4: return spread_mma_m<4>(a, nrhs, s);
    case 5: return spread_mma_m<5>(a, nrhs, s);
    case 6: return spread_mma_m<6>(a, nrhs, s);
    case 7: return spread_mma_m<7>(a, nrhs, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nfft
