// Spreading for d = 2 in float32 with the padded tile of a work item held in
// registers (Algorithm 2.4 step 1 with the weights of (3.7)).
//
// The LDS spreading kernels update a node's (2m)^2 footprint by
// read-modify-write of LDS cells, and a lane group's next node has to wait
// for those writes. Here every wave keeps a whole padded tile (P = 16 + 2m
// rows and columns) in registers instead: lane c of a 32-lane half owns
// padded column c and holds its P cells, real and imaginary part, in 2P
// registers. A wave takes two nodes at a time, one per half. For a node with
// tile-local cell (l0, l1) the rows l0+1 .. l0+2m are updated by
//     acc[l0 + 1 + i] += a_i * (b_c * c_j),        i < 2m,
// with a_i the row factor (dimension 0) broadcast to the lanes by the DPP
// operand of the multiply-add, b_c the column factor of lane c (zero outside
// the footprint) and c_j = w_j f_j. Register indices must be static: the
// nodes of a tile are sorted by row at plan time, and the node loop runs
// inside an unrolled loop over the 16 tile rows, so that for row r the
// updated registers are the constants r+1 .. r+2m. The two nodes of a wave
// step come from the same row (pairs of consecutive nodes of the row; the
// pairs of all rows are dealt to the waves in turn). Nothing is written to
// LDS inside the node loop; at the end the waves' tiles are summed in LDS in
// a fixed order (the result does not depend on timing) and the padded tile
// is written out like the other kernels' (tile_reduce and the first FFT pass
// merge them).
// The window factors are evaluated per call from the node's offsets (lane p
// of the half's first 16-lane row evaluates polynomial p at the dimension-0
// offset, lane p of its second row at the dimension-1 offset; the factors
// reach their lanes by ds_bpermute).
// Nodes exactly on a grid line get the closed-edge row l0 / column l1.
#include "spread_common.hpp"

namespace nfft {

namespace {

// acc[OFF + i] += (v of lane i of this lane's 16-lane row) * x, i < K: the
// row broadcast is the DPP operand modifier of the multiply-add. The leading
// s_nop covers the wait states of a DPP read after a VALU write of v (two)
// or a scalar write of EXEC (five). All 64 lanes are active.
#define NFFT_REG_FMAC(I, NOP)                                                                   \
  if constexpr (K > I)                                                                          \
  asm volatile(NOP "v_fmac_f32_dpp %0, %1, %2 row_newbcast:" #I " row_mask:0xf bank_mask:0xf" \
               : "+v"(acc[OFF + I])                                                             \
               : "v"(v), "v"(x))
template <int OFF, int K, int P>
__device__ __forceinline__ void fmac_rows(float (&acc)[P], float v, float x) {
  static_assert(K >= 1 && K <= 16 && OFF + K <= P, "rows inside the padded tile");
  NFFT_REG_FMAC(0, "s_nop 4\n");
  NFFT_REG_FMAC(1, "");
  NFFT_REG_FMAC(2, "");
  NFFT_REG_FMAC(3, "");
  NFFT_REG_FMAC(4, "");
  NFFT_REG_FMAC(5, "");
  NFFT_REG_FMAC(6, "");
  NFFT_REG_FMAC(7, "");
  NFFT_REG_FMAC(8, "");
  NFFT_REG_FMAC(9, "");
  NFFT_REG_FMAC(10, "");
  NFFT_REG_FMAC(11, "");
  NFFT_REG_FMAC(12, "");
  NFFT_REG_FMAC(13, "");
  NFFT_REG_FMAC(14, "");
  NFFT_REG_FMAC(15, "");
}
#undef NFFT_REG_FMAC

__device__ __forceinline__ float lane_pick(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

}  // namespace

// Nodes staged per batch (a work item of up to 512 nodes in one batch).
constexpr int kRegBatch = 512;

template <int MW>
struct RegLds {
  static constexpr int K2 = 2 * MW;
  static constexpr int P = 16 + K2;
  // staging: c_j (2 floats), cell word and the two offsets per node; the
  // first node of every tile row in the batch (17 entries)
  static constexpr size_t per_node = 3 * 4 + 2 * 4;
  static constexpr size_t staging = kRegBatch * per_node + 32 * 4;
  static constexpr size_t combine = 2 * (size_t)P * P * sizeof(float2);
  static constexpr size_t bytes = staging > combine ? staging : combine;
};

template <int MW, int NW>
__global__ __launch_bounds__(64 * NW) void spread_reg_kernel(SpreadArgs<float> a) {
  constexpr int K2 = 2 * MW;
  constexpr int P = 16 + K2;
  constexpr int NT = 64 * NW;
  constexpr int NB = kRegBatch;
  constexpr int DEG = PolyDeg<float>::value;
  extern __shared__ float lds_f[];
  float* st_cx = lds_f;
  float* st_cy = st_cx + NB;
  uint32_t* st_loc = reinterpret_cast<uint32_t*>(st_cy + NB);
  float* st_w = reinterpret_cast<float*>(st_loc + NB);  // offsets [2][NB]
  int* st_rs = reinterpret_cast<int*>(st_w + 2 * NB);    // row starts [17]

  const int item = blockIdx.x;
  const int rhs = blockIdx.y;
  const int tid = threadIdx.x;
  // wave-uniform (a scalar register), so that the node loop and the row
  // dispatch below are scalar branches and EXEC stays full
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int half = lane >> 5;
  const int col = lane & 31;     // padded column of this lane
  const int p = lane & 15;       // position in the 16-lane row
  const bool rowB = (lane & 16) != 0;
  const int pc = p < K2 ? p : K2 - 1;

  float cf[DEG + 1];
#pragma unroll
  for (int q = 0; q <= DEG; ++q) cf[q] = a.coef[pc * (DEG + 1) + q];

  float ar[P], ai[P];
#pragma unroll
  for (int r = 0; r < P; ++r) {
    ar[r] = 0.0f;
    ai[r] = 0.0f;
  }

  const int64_t N = a.g.N;
  const int start = a.item_start[item];
  const int cnt = a.item_count[item];
  const float2* f = a.f + rhs * a.f_rs;
  const float edge = a.edge;

  for (int b0 = 0; b0 < cnt; b0 += NB) {
    const int nb = (cnt - b0) < NB ? (cnt - b0) : NB;
    __syncthreads();  // the previous batch is consumed
#pragma unroll 2
    for (int t = tid; t < nb; t += NT) {
      const int i = start + b0 + t;
      const float2 wv = a.w[i];
      const float2 fv = f[a.perm[i]];
      st_cx[t] = wv.x * fv.x - wv.y * fv.y;
      st_cy[t] = wv.x * fv.y + wv.y * fv.x;
      st_loc[t] = a.loc[i];
      st_w[t] = 2.0f * a.frac[i] - 1.0f;
      st_w[NB + t] = 2.0f * a.frac[N + i] - 1.0f;
    }
    __syncthreads();
    // first node of each tile row (the batch is sorted by row): node t opens
    // the rows after its predecessor's up to its own; the last node closes
    // the rest
    for (int t = tid; t < nb; t += NT) {
      const int rt = (int)(st_loc[t] & kLocMask);
      const int rp = t > 0 ? (int)(st_loc[t - 1] & kLocMask) : -1;
      for (int r = rp + 1; r <= rt; ++r) st_rs[r] = t;
      if (t == nb - 1)
        for (int r = rt + 1; r <= 16; ++r) st_rs[r] = nb;
    }
    __syncthreads();

    // pairs of consecutive nodes within each row; the pairs of all rows are
    // numbered in row order and wave w takes pairs w, w + NW, ...
    int pbase = 0;  // pairs of the rows before r
    static_for<0, 16>([&](auto rc) {
      constexpr int r = decltype(rc)::value;
      const int n0 = __builtin_amdgcn_readfirstlane(st_rs[r]);
      const int n1 = __builtin_amdgcn_readfirstlane(st_rs[r + 1]);
      const int np = (n1 - n0 + 1) >> 1;
      // first pair of this row that belongs to this wave
      int q = wave - pbase % NW;
      q = q < 0 ? q + NW : q;
      for (; q < np; q += NW) {
        const int n = n0 + 2 * q + half;
        const bool valid = n < n1;
        const int nn = valid ? n : n1 - 1;
        // nn is a node of this batch: the reads need no guard
        const uint32_t L = st_loc[nn];
        const float sx = st_cx[nn], sy = st_cy[nn];
        const float cx = valid ? sx : 0.0f;
        const float cy = valid ? sy : 0.0f;
        const int l1 = (int)((L >> kLocBits) & kLocMask);
        const bool e0 = valid && ((L >> kEdgeShift) & 1u);
        const bool e1 = (L >> (kEdgeShift + 1)) & 1u;
        const int k = col - l1 - 1;  // footprint column of this lane
        // first row of the half: factor p of dimension 0; second row: of dimension 1
        const float y = rowB ? st_w[NB + nn] : st_w[nn];
        const float hv = horner<float>(cf, y);
        const float av = lane_pick(hv, (lane & 32) | p);
        const float bk = lane_pick(hv, (lane & 32) | 16 | (k & 15));
        const float bv = (k >= 0 && k < K2) ? bk : ((e1 && col == l1) ? edge : 0.0f);
        const float vx = bv * cx;
        const float vy = bv * cy;
        fmac_rows<r + 1, K2, P>(ar, av, vx);
        fmac_rows<r + 1, K2, P>(ai, av, vy);
        // closed-edge row of nodes on a grid line in dimension 0
        if (__builtin_amdgcn_ballot_w64(e0)) {
          ar[r] += e0 ? edge * vx : 0.0f;
          ai[r] += e0 ? edge * vy : 0.0f;
        }
      }
      pbase += np;
    });
  }

  // the waves' tiles summed in LDS in wave order, one tile per half, then the
  // two halves added: a fixed order, so the result does not depend on timing
  __syncthreads();
  float2* tile0 = reinterpret_cast<float2*>(lds_f);
  float2* tile1 = tile0 + P * P;
  float2* mine = half ? tile1 : tile0;
#pragma unroll 1
  for (int w = 0; w < NW; ++w) {
    if (wave == w && col < P) {
      if (w == 0) {
#pragma unroll
        for (int r = 0; r < P; ++r) mine[r * P + col] = make_float2(ar[r], ai[r]);
      } else {
#pragma unroll
        for (int r = 0; r < P; ++r) {
          float2 v = mine[r * P + col];
          v.x += ar[r];
          v.y += ai[r];
          mine[r * P + col] = v;
        }
      }
    }
    __syncthreads();
  }
  const int slot = a.item_slot[item];
  float2* out = slot < 0 ? a.tilep + rhs * a.tile_rs + (int64_t)a.item_bin[item] * (P * P)
                         : a.itemp + rhs * a.item_rs + (int64_t)slot * (P * P);
  for (int i = tid; i < P * P; i += NT) {
    const float2 u = tile0[i], v = tile1[i];
    out[i] = make_float2(u.x + v.x, u.y + v.y);
  }
}

bool spread_reg_supported(int d, int T, bool f64) { return d == 2 && T == 16 && !f64; }

size_t spread_reg_lds_bytes(int m) {
  switch (m) {
#define NFFT_REG_LDS(MW) \
  case MW:               \
    return RegLds<MW>::bytes;
    NFFT_REG_LDS(1) NFFT_REG_LDS(2) NFFT_REG_LDS(3) NFFT_REG_LDS(4)
    NFFT_REG_LDS(5) NFFT_REG_LDS(6) NFFT_REG_LDS(7) NFFT_REG_LDS(8)
#undef NFFT_REG_LDS
    default: return 0;
  }
}

template <int MW>
static hipError_t spread_reg_m(const SpreadArgs<float>& a, int nrhs, hipStream_t s) {
  const dim3 grid(a.g.nsub, nrhs);
  const size_t lds = RegLds<MW>::bytes;
  // 64 or 128 threads: two waves; 256: four; 512: eight
  if (a.nt == 512)
    hipLaunchKernelGGL((spread_reg_kernel<MW, 8>), grid, dim3(512), lds, s, a);
  else if (a.nt == 256)
    hipLaunchKernelGGL((spread_reg_kernel<MW, 4>), grid, dim3(256), lds, s, a);
  else
    hipLaunchKernelGGL((spread_reg_kernel<MW, 2>), grid, dim3(128), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_spread_reg(const SpreadArgs<float>& a, int nrhs, hipStream_t s) {
  if (!spread_reg_supported(a.g.d, a.g.T, false)) return hipErrorInvalidValue;
  if (a.g.nsub == 0) return hipSuccess;
  switch (a.g.m) {
    case 1: return spread_reg_m<1>(a, nrhs, s);
    case 2: return spread_reg_m<2>(a, nrhs, s);
    case 3: return spread_reg_m<3>(a, nrhs, s);
    case 4: return spread_reg_m<4>(a, nrhs, s);
    case 5: return spread_reg_m<5>(a, nrhs, s);
    case 6: return spread_reg_m<6>(a, nrhs, s);
    case 7: return spread_reg_m<7>(a, nrhs, s);
    case 8: return spread_reg_m<8>(a, nrhs, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nfft
