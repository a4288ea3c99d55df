// Spreading of many right-hand sides by tiles of the output grid (d = 2,
// float32; Algorithm 2.4 step 1 with the weights of (3.7), Remark 3.1 (ii)).
//
// Right-hand sides that share a node set share every node's cell and window
// factors; only c_j^(r) = w_j f_j^(r) differs. Here a work-group owns one
// 16 x 16 tile of the oversampled grid and 32 right-hand sides, and lane
// r + 32 c of each wave holds component c (real, imaginary) of right-hand
// side r: every lane does useful work on every node, and the node's window
// factors are the same for all lanes (LDS broadcasts). Wave w keeps the tile
// rows 4w .. 4w+3, all 16 columns, in 64 registers. The nodes whose window
// support reaches a tile (its own and those of the eight neighbouring tiles
// that come within m cells; the window spans 2m + 1 <= 17 cells, so no
// farther tile can) are listed per tile at plan time, with the footprint
// origin relative to the tile. A work unit is a run of at most item_nodes
// entries of one tile's list: the work-group stages their window factors and
// samples in LDS and adds
//     acc[row][col] += (c_j * a_q) * b_k
// for the footprint row q and column k that fall on the wave's cells.
// Register indices must be static: each tile's list is sorted at plan time by
// the column offset of the footprint inside the tile, and the node loop runs
// inside an unrolled loop over the 16 + 2m possible offsets, so that for
// offset C the updated registers are constants and only the cells a node
// reaches are updated. The samples are first copied node-major (32 samples of
// a node in 256 contiguous bytes), so that the staging reads whole lines. A tile with one unit writes its grid
// cells directly; a tile whose list was cut into several units (the crowded
// tiles) writes one 16 x 16 partial per unit, and a second kernel sums the
// partials in unit order with compensation (Neumaier) into the grid. Each
// partial is one float32 sum per cell in a fixed node order, so the result
// does not depend on timing; no halo is written or merged.
#include "spread_common.hpp"

namespace nfft {

namespace {

constexpr int kGatherRhs = 32;  // right-hand sides per work-group
constexpr int kGatherNb = 64;   // list entries staged per round

template <int MW>
struct GatherLds {
  static constexpr int K = 2 * MW + 1;             // footprint cells per dimension
  static constexpr int XS = (K + 3) / 4 * 4;       // column factors stored per node
  static constexpr int YS = (K + 8 + 3) / 4 * 4;   // row factors: 4 zeros, K values, 4 zeros
  static constexpr int NC = 16 + 2 * MW;           // column offsets
  // per entry: header, caller index, two offsets, weight, factors, samples
  static constexpr size_t staging =
      kGatherNb * (2 * sizeof(int) + 4 * sizeof(float) + (XS + YS) * sizeof(float) +
                   2 * kGatherRhs * sizeof(float)) +
      (NC + 1) * sizeof(int);
  // one wave's tile for the output transpose: [rhs][65 cells][2] floats
  static constexpr size_t transpose = (size_t)kGatherRhs * 65 * 2 * sizeof(float);
  static constexpr size_t bytes = staging > transpose ? staging : transpose;
};

// acc[i][col] += t_i * b_k for the footprint columns k whose tile column
// col = C - 2m + k lies in 0..15 (C: the case of the column dispatch), rows
// i of the wave that the node reaches.
template <int C, int MW>
__device__ __forceinline__ void gather_cols(float (&acc)[4][16], const float (&t)[4],
                                            const bool (&act)[4], const float (&bx)[2 * MW + 1]) {
  static_for<0, 4>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if (act[i]) {
      static_for<0, 2 * MW + 1>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int col = C - 2 * MW + k;
        if constexpr (col >= 0 && col < 16) acc[i][col] = fmaf(t[i], bx[k], acc[i][col]);
      });
    }
  });
}

}  // namespace

template <int MW>
__global__ __launch_bounds__(256) void spread_gather_kernel(
    SpreadArgs<float> a, const int32_t* __restrict__ units, const int32_t* __restrict__ gl_node,
    const int32_t* __restrict__ gl_hdr, const float2* __restrict__ fT, float2* __restrict__ grid,
    int64_t grid_rs, float2* __restrict__ part, int64_t part_rs, int nrhs) {
  constexpr int K = 2 * MW + 1;
  constexpr int XS = GatherLds<MW>::XS;
  constexpr int NB = kGatherNb;
  constexpr int DEG = PolyDeg<float>::value;
  extern __shared__ float lds_f[];
  int* s_hdr = reinterpret_cast<int*>(lds_f);  // packed footprint origin and edge flags
  int* s_perm = s_hdr + NB;                     // caller index
  float* s_y = reinterpret_cast<float*>(s_perm + NB);  // offsets 2 frac - 1, [2][NB]
  float2* s_w = reinterpret_cast<float2*>(s_y + 2 * NB);  // weights
  constexpr int YS = GatherLds<MW>::YS;
  float* s_ay = reinterpret_cast<float*>(s_w + NB);  // row factors [NB][YS], entry q at 4 + q
  float* s_bx = s_ay + NB * YS;                         // column factors [NB][XS]
  float* s_c = s_bx + NB * XS;                          // samples [NB][re 32 | im 32]
  int* s_cs = reinterpret_cast<int*>(s_c + NB * 2 * kGatherRhs);  // first entry per offset
  constexpr int NC = GatherLds<MW>::NC;
  __shared__ float s_cf[2 * MW * (DEG + 1)];

  const int* u = units + 4 * (int64_t)blockIdx.x;
  const int tile = u[0], e_begin = u[1], e_end = u[2], slot = u[3];
  if (tile < 0) return;  // padding of the unit list
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nb = a.g.nb;
  const int t0 = tile / nb, t1 = tile - (tile / nb) * nb;
  const int rhs0 = blockIdx.y * kGatherRhs;
  const int64_t N = a.g.N;
  for (int i = tid; i < 2 * MW * (DEG + 1); i += 256) s_cf[i] = a.coef[i];

  float acc[4][16];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[i][j] = 0.0f;

  for (int c0 = e_begin; c0 < e_end; c0 += NB) {
    const int nk = (e_end - c0) < NB ? (e_end - c0) : NB;
    __syncthreads();  // the previous round is consumed
    // per entry its node's data (every load of a thread issued together)
    if (tid < nk) {
      const int hd = gl_hdr[c0 + tid];
      const int hp = tid > 0 ? gl_hdr[c0 + tid - 1] : 0;
      const int i = gl_node[c0 + tid];
      const float fr0 = a.frac[i], fr1 = a.frac[N + i];
      const float2 wv = a.w[i];
      const int pm = a.perm[i];
      s_hdr[tid] = hd;
      s_perm[tid] = pm;
      s_y[tid] = 2.0f * fr0 - 1.0f;
      s_y[NB + tid] = 2.0f * fr1 - 1.0f;
      s_w[tid] = wv;
      // first entry of every column offset (the list is sorted by offset):
      // entry t opens the offsets after its predecessor's up to its own, the
      // last entry closes the rest
      const int ct = ((hd >> 8) & 0xff) - 64 + 2 * MW;
      const int cp = tid > 0 ? ((hp >> 8) & 0xff) - 64 + 2 * MW : -1;
      for (int c = cp + 1; c <= ct; ++c) s_cs[c] = tid;
      if (tid == nk - 1)
        for (int c = ct + 1; c <= NC; ++c) s_cs[c] = nk;
    }
    __syncthreads();
    // samples c_j = w_j f_j of the work-group's right-hand sides, from the
    // node-major copy (a node's 32 samples are 256 contiguous bytes): item
    // e = tid + 256 j is right-hand side e mod 32 of entry e / 32
    {
      constexpr int SPT = NB * kGatherRhs / 256;
      const float2* fg = fT + (int64_t)blockIdx.y * N * kGatherRhs;
      float2 fv[SPT];
#pragma unroll
      for (int j = 0; j < SPT; ++j) {
        const int e = tid + 256 * j;
        const int k = e / kGatherRhs, r = e % kGatherRhs;
        fv[j] = make_float2(0.0f, 0.0f);
        if (k < nk) fv[j] = fg[(int64_t)s_perm[k] * kGatherRhs + r];
      }
#pragma unroll
      for (int j = 0; j < SPT; ++j) {
        const int e = tid + 256 * j;
        const int k = e / kGatherRhs, r = e % kGatherRhs;
        if (k < nk) {
          const float2 wv = s_w[k];
          s_c[k * 2 * kGatherRhs + r] = wv.x * fv[j].x - wv.y * fv[j].y;
          s_c[k * 2 * kGatherRhs + kGatherRhs + r] = wv.x * fv[j].y + wv.y * fv[j].x;
        }
      }
    }
    // window factors: entry 0 the closed-edge cell, 1 + i polynomial i; the
    // row factors with four zeros on either side, so that the four rows of a
    // wave are read unconditionally
    for (int e = tid; e < nk * 2 * K; e += 256) {
      const int k = e / (2 * K);
      const int rem = e - k * (2 * K);
      const int dim = rem >= K ? 1 : 0;
      const int q = rem - dim * K;
      const float hv = horner<float>(s_cf + (q > 0 ? q - 1 : 0) * (DEG + 1), s_y[dim * NB + k]);
      const float v = q == 0 ? (((s_hdr[k] >> (16 + dim)) & 1) ? a.edge : 0.0f) : hv;
      if (dim)
        s_bx[k * XS + q] = v;
      else
        s_ay[k * YS + 4 + q] = v;
    }
    for (int e = tid; e < nk * 8; e += 256) {
      const int k = e >> 3, z = e & 7;
      s_ay[k * YS + (z < 4 ? z : K + z)] = 0.0f;
    }
    __syncthreads();
    int cs[NC + 1];
#pragma unroll
    for (int c = 0; c <= NC; ++c) cs[c] = s_cs[c];
    static_for<0, NC>([&](auto cc) {
      constexpr int C = decltype(cc)::value;
      const int k0 = __builtin_amdgcn_readfirstlane(cs[C]);
      const int k1 = __builtin_amdgcn_readfirstlane(cs[C + 1]);
      int hd_next = k0 < k1 ? s_hdr[k0] : 0;
      for (int k = k0; k < k1; ++k) {
        const int hd = __builtin_amdgcn_readfirstlane(hd_next);
        if (k + 1 < k1) hd_next = s_hdr[k + 1];  // the next header, read ahead
        const int b0 = (hd & 0xff) - 64;
        const int qlo = ((hd >> 16) & 1) ? 0 : 1;
        const int q0 = 4 * wave - b0;  // footprint row of the wave's first row
        if (q0 + 3 < qlo || q0 > 2 * MW) continue;
        const float cv = s_c[k * 2 * kGatherRhs + lane];
        float bx[K];
#pragma unroll
        for (int q = 0; q < K; ++q) bx[q] = s_bx[k * XS + q];
        // rows q0 .. q0+3 of the padded row factors (zeros outside the footprint)
        const float* ay = s_ay + k * YS + 4 + q0;
        float t[4];
        bool act[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int q = q0 + i;
          act[i] = q >= qlo && q <= 2 * MW;
          t[i] = cv * ay[i];
        }
        gather_cols<C, MW>(acc, t, act, bx);
      }
    });
  }

  // output: each wave in turn transposes its rows through LDS so that a
  // store writes 16 consecutive cells of one right-hand side: to the grid,
  // or to the unit's partial slot (cells in tile order)
  float* tr = lds_f;
  const int r = lane & 31, comp = lane >> 5;
  for (int w = 0; w < 4; ++w) {
    __syncthreads();
    if (wave == w) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 16; ++j) tr[(r * 65 + i * 16 + j) * 2 + comp] = acc[i][j];
    }
    __syncthreads();
    if (wave == w) {
      const int i = lane >> 4, j = lane & 15;
      float2* dst;
      int64_t rs;
      if (slot < 0) {
        dst = grid + (int64_t)(16 * t0 + 4 * w + i) * a.g.Ms + 16 * t1 + j;
        rs = grid_rs;
      } else {
        dst = part + (int64_t)slot * 256 + 64 * w + lane;
        rs = part_rs;
      }
      for (int rr = 0; rr < kGatherRhs && rhs0 + rr < nrhs; ++rr) {
        const float* src = tr + (rr * 65 + lane) * 2;
        dst[(int64_t)(rhs0 + rr) * rs] = make_float2(src[0], src[1]);
      }
    }
  }
}

// The samples of every group of 32 right-hand sides node-major: fT[g][j][r]
// = f[32 g + r][j] (caller order; zero for right-hand sides past nrhs), by
// tiles of 32 right-hand sides x 64 nodes through LDS, both sides coalesced.
__global__ __launch_bounds__(256) void gather_transpose_kernel(const float2* __restrict__ f,
                                                               int64_t f_rs, int64_t N, int nrhs,
                                                               float2* __restrict__ fT) {
  __shared__ float2 t[64][kGatherRhs + 1];
  const int64_t j0 = (int64_t)blockIdx.x * 64;
  const int g = blockIdx.y;
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int e = tid + 256 * q;
    const int r = e / 64, jj = e % 64;
    const int rg = g * kGatherRhs + r;
    t[jj][r] = (rg < nrhs && j0 + jj < N) ? f[(int64_t)rg * f_rs + j0 + jj] : make_float2(0.f, 0.f);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int e = tid + 256 * q;
    const int jj = e / kGatherRhs, r = e % kGatherRhs;
    if (j0 + jj < N) fT[((int64_t)g * N + j0 + jj) * kGatherRhs + r] = t[jj][r];
  }
}

// The partials of a tile cut into several units, summed in unit order with
// compensation into the tile's grid cells. split: per tile (tile, first
// slot, slots, unused); one work-group per tile and right-hand side, one
// thread per cell.
__global__ __launch_bounds__(256) void gather_reduce_kernel(const int32_t* __restrict__ split,
                                                            const float2* __restrict__ part,
                                                            int64_t part_rs, float2* __restrict__ grid,
                                                            int64_t grid_rs, int nb, int Ms) {
  const int* sp = split + 4 * (int64_t)blockIdx.x;
  const int tile = sp[0], first = sp[1], cnt = sp[2];
  const int r = blockIdx.y;
  const int cell = threadIdx.x;
  const float2* src = part + (int64_t)r * part_rs + (int64_t)first * 256 + cell;
  KSum<float> sx, sy;
  for (int k = 0; k < cnt; ++k) {
    const float2 v = src[(int64_t)k * 256];
    sx.add(v.x);
    sy.add(v.y);
  }
  const int t0 = tile / nb, t1 = tile - (tile / nb) * nb;
  grid[(int64_t)r * grid_rs + (int64_t)(16 * t0 + (cell >> 4)) * Ms + 16 * t1 + (cell & 15)] =
      make_float2(sx.value(), sy.value());
}

bool spread_gather_supported(int d, int T, bool f64, int m) {
  return d == 2 && T == 16 && !f64 && m >= 1 && m <= 8;
}

size_t spread_gather_lds_bytes(int m) {
  switch (m) {
#define NFFT_GATHER_LDS(MW) \
  case MW:                  \
    return GatherLds<MW>::bytes;
    NFFT_GATHER_LDS(1) NFFT_GATHER_LDS(2) NFFT_GATHER_LDS(3) NFFT_GATHER_LDS(4)
    NFFT_GATHER_LDS(5) NFFT_GATHER_LDS(6) NFFT_GATHER_LDS(7) NFFT_GATHER_LDS(8)
#undef NFFT_GATHER_LDS
    default: return 0;
  }
}

template <int MW>
static hipError_t spread_gather_m(const SpreadArgs<float>& a, const GatherArgs& ga, int nrhs,
                                  hipStream_t s) {
  const dim3 blocks(ga.nunits, (nrhs + kGatherRhs - 1) / kGatherRhs);
  hipLaunchKernelGGL((spread_gather_kernel<MW>), blocks, dim3(256), GatherLds<MW>::bytes, s, a,
                     ga.units, ga.gl_node, ga.gl_hdr, ga.fT, ga.grid, ga.grid_rs, ga.part,
                     ga.part_rs, nrhs);
  return hipGetLastError();
}

hipError_t launch_spread_gather(const SpreadArgs<float>& a, const GatherArgs& ga, int nrhs,
                                hipStream_t s) {
  if (!spread_gather_supported(a.g.d, a.g.T, false, a.g.m)) return hipErrorInvalidValue;
  if (ga.nunits == 0) return hipSuccess;
  const int groups = (nrhs + kGatherRhs - 1) / kGatherRhs;
  hipLaunchKernelGGL(gather_transpose_kernel, dim3((unsigned)((a.g.N + 63) / 64), groups), dim3(256),
                     0, s, a.f, a.f_rs, a.g.N, nrhs, ga.fT);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (a.g.m) {
    case 1: return spread_gather_m<1>(a, ga, nrhs, s);
    case 2: return spread_gather_m<2>(a, ga, nrhs, s);
    case 3: return spread_gather_m<3>(a, ga, nrhs, s);
    case 4: return spread_gather_m<4>(a, ga, nrhs, s);
    case 5: return spread_gather_m<5>(a, ga, nrhs, s);
    case 6: return spread_gather_m<6>(a, ga, nrhs, s);
    case 7: return spread_gather_m<7>(a, ga, nrhs, s);
    case 8: return spread_gather_m<8>(a, ga, nrhs, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gather_reduce(const GatherArgs& ga, int nb, int Ms, int nrhs, hipStream_t s) {
  if (ga.nsplit == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_reduce_kernel, dim3(ga.nsplit, nrhs), dim3(256), 0, s, ga.split,
                     ga.part, ga.part_rs, ga.grid, ga.grid_rs, nb, Ms);
  return hipGetLastError();
}

}  // namespace nfft
