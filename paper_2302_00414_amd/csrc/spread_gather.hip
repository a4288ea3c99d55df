// Spreading of many right-hand sides by tiles of the output grid (d = 2,
// float32; Algorithm 2.4 step 1 with the weights of (3.7), Remark 3.1 (ii)).
//
// Right-hand sides that share a node set share every node's cell and window
// factors; only c_j^(r) = w_j f_j^(r) differs. For a tile of grid cells and
// 32 right-hand sides the spreading is the contraction
//     g[m][cell] = sum_j C[m][j] W_j[cell],   m = (component, rhs) < 64,
// C[m][j] the real or imaginary part of c_j^(r), W_j[cell] = a_q b_k the
// window factor of node j at that cell (zero outside its footprint): a
// product of a 64 x n and an n x cells matrix, with about 24 flops per byte
// of input. A work-group owns one 16 x 16 tile of the oversampled grid,
// split into sixteen 4 x 4 sub-tiles; each of its eight waves owns two
// sub-tiles and keeps their 64 x 16 sums as four 16 x 16 blocks each
// (v_mfma_f32_16x16x4f32 accumulators, 32 registers). The nodes whose window
// support reaches the tile (its own and those of the eight neighbouring tiles
// that come within m cells; 2m + 1 <= 17, so no farther tile can) are listed
// per tile at plan time with the footprint origin relative to the tile. A
// work unit is a run of at most item_nodes entries of one tile's list; the
// work-group stages 128 entries at a time in LDS (window factors, and the
// samples of the 32 right-hand sides, read from a node-major copy so that a
// node's 32 samples are 256 contiguous bytes), each wave ballots for its two
// sub-tiles the staged entries that reach them and feeds those entries four
// at a time (K = 4) to the matrix cores: lane (k, cell) forms W_k[cell],
// lane (k, m) loads C[m][k]. A tile with one unit writes its grid
// cells directly; a tile whose list was cut into several units (the crowded
// tiles) writes one 16 x 16 partial per unit, and a second kernel sums the
// partials in unit order with compensation (Neumaier) into the grid. Every
// sum runs in a fixed order, so the result does not depend on timing; no halo
// is written or merged.
#include "spread_common.hpp"

namespace nfft {

namespace {

constexpr int kGatherRhs = 32;  // right-hand sides per work-group
constexpr int kGatherNb = 128;  // list entries staged per round
constexpr int kGatherNt = 512;  // threads per work-group (8 waves)

template <int MW>
struct GatherLds {
  static constexpr int K = 2 * MW + 1;             // footprint cells per dimension
  // factors stored per node and dimension: 4 zeros, K values, 4 or more zeros
  static constexpr int YS = (K + 8 + 3) / 4 * 4;
  static constexpr int XS = YS;
  // per entry: header, caller index, two offsets; factors and samples also
  // for entry kGatherNb, all zeros (the padding of the lists)
  static constexpr size_t staging =
      kGatherNb * (2 * sizeof(int) + 2 * sizeof(float)) +
      (kGatherNb + 1) * ((XS + YS) * sizeof(float) + 2 * kGatherRhs * sizeof(float));
  // the output transpose, per band of four tile rows and half of the
  // right-hand sides: [rhs][65 cells][2] floats
  static constexpr size_t transpose = (size_t)4 * (kGatherRhs / 2) * 65 * 2 * sizeof(float);
  static constexpr size_t bytes = staging > transpose ? staging : transpose;
};

typedef float gather_v4f __attribute__((ext_vector_type(4)));

}  // namespace

template <int MW>
__global__ __launch_bounds__(kGatherNt) void spread_gather_kernel(
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
  constexpr int YS = GatherLds<MW>::YS;
  float* s_ay = s_y + 2 * NB;  // row factors [NB + 1][YS], cell q at 4 + q
  float* s_bx = s_ay + (NB + 1) * YS;                   // column factors [NB + 1][XS], likewise
  // samples: component row m = 32 c + r (c: real 0, imaginary 1; r: rhs) of
  // entry k at s_c[k][m mod 16][m / 16], so that a lane's four A values (one
  // per 16-row block) are one 16-byte read; [NB + 1][64]
  float* s_c = s_bx + (NB + 1) * XS;
  __shared__ float s_cf[2 * MW * (DEG + 1)];
  // staged entries that reach each 4 x 4 sub-tile, in entry order, padded
  // to a multiple of 4 items; each wave lists its own two sub-tiles. An item packs the entry index (bits 0-7) with the
  // footprint origin relative to the tile plus 64 (bits 8-15 rows, 16-23
  // columns); a padding item names the zero entry NB at the sub-tile's own
  // origin.
  __shared__ int s_list[16][NB];
  constexpr int NH = NB / 64;  // ballots of 64 entries per round
  static_assert(NB % 64 == 0 && NB <= 128 && kGatherNt == 512, "eight waves, 64-entry ballots");
  constexpr int NT = kGatherNt;

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
  for (int i = tid; i < 2 * MW * (DEG + 1); i += NT) s_cf[i] = a.coef[i];
  // the factor rows start zero (only cells 0 .. 2m are written per round),
  // and entry NB is zero throughout
  for (int i = tid; i < (NB + 1) * (XS + YS); i += NT) s_ay[i] = 0.0f;
  if (tid < 2 * kGatherRhs) s_c[NB * 2 * kGatherRhs + tid] = 0.0f;

  // acc[q][mb]: sub-tile 2 wave + q, rows mb*16 .. mb*16+15 of the 64 x 16 sums
  gather_v4f acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = gather_v4f{0.0f, 0.0f, 0.0f, 0.0f};

  // node data of a round's entries, loaded by waves 0 and 1 (one entry per lane)
  // one round ahead, so that its latency hides behind the round before
  int p_hd = 0, p_pm = 0;
  float p_y0 = 0.0f, p_y1 = 0.0f;
  auto fetch = [&](int cb) {
    if (tid < NB && cb + tid < e_end) {
      p_hd = gl_hdr[cb + tid];
      const int i = gl_node[cb + tid];
      p_y0 = 2.0f * a.frac[i] - 1.0f;
      p_y1 = 2.0f * a.frac[N + i] - 1.0f;
      p_pm = a.perm[i];
    }
  };
  fetch(e_begin);
  for (int c0 = e_begin; c0 < e_end; c0 += NB) {
    const int nk = (e_end - c0) < NB ? (e_end - c0) : NB;
    __syncthreads();  // the previous round is consumed
    // the prefetched entries into LDS (waves 0 and 1)
    if (tid < NB) {
      if (tid < nk) {
        s_hdr[tid] = p_hd;
        s_perm[tid] = p_pm;
        s_y[tid] = p_y0;
        s_y[NB + tid] = p_y1;
      }
      fetch(c0 + NB);  // the next round's entries, in flight from here
    }
    __syncthreads();
    // samples c_j = w_j f_j of the work-group's right-hand sides, from the
    // weighted node-major copy, which holds a node's 32 in the layout of s_c
    // (256 contiguous bytes): float4 e = tid + NT j is float4 e mod 16 of
    // entry e / 16; the window factors are evaluated while the loads are in
    // flight
    constexpr int SPT = NB * 16 / NT;
    const float4* fg = reinterpret_cast<const float4*>(fT) + (int64_t)blockIdx.y * N * 16;
    float4 fv[SPT];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      const int e = tid + NT * j;
      const int k = e >> 4;
      fv[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (k < nk) fv[j] = fg[(int64_t)s_perm[k] * 16 + (e & 15)];
    }
    // window factors: cell 0 the closed-edge cell, 1 + i polynomial i (both
    // dimensions stored from index 4). Thread (k, part), k = tid / 4, takes
    // entry k in dimension part / 2 and evaluates half part % 2 of the 2m
    // polynomials at its offset (m independent Horner chains)
    static_assert(NB * 4 == NT, "four threads an entry");
    {
      const int k = tid >> 2, dim = (tid >> 1) & 1, half = tid & 1;
      if (k < nk) {
        const float y = s_y[dim * NB + k];
        float* dst = (dim ? s_bx + k * XS : s_ay + k * YS) + 4;
        if (half == 0) dst[0] = ((s_hdr[k] >> (16 + dim)) & 1) ? a.edge : 0.0f;
#pragma unroll
        for (int i = 0; i < MW; ++i) {
          const int pi = half * MW + i;
          dst[1 + pi] = horner<float>(s_cf + pi * (DEG + 1), y);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      const int e = tid + NT * j;
      if ((e >> 4) < nk) reinterpret_cast<float4*>(s_c)[e] = fv[j];
    }
    __syncthreads();
    // the wave's two sub-tiles: the lists of staged entries whose footprint
    // reaches each (a ballot per half round), then those entries four at a
    // time. The lists are this wave's own: written and read by it alone.
    const int kk = lane >> 4, j = lane & 15;
    int hd2[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) hd2[h] = 64 * h + lane < nk ? s_hdr[64 * h + lane] : -1;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int st = 2 * wave + q;
      const int row = 4 * (st >> 2) + (j >> 2);  // tile cell of lane (kk, j) in B
      const int col = 4 * (st & 3) + (j & 3);
      int cnt = 0;
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int hd = hd2[h];
        // footprint rows b0 + (edge ? 0 : 1) .. b0 + 2m against the
        // sub-tile's rows 4 sr .. 4 sr + 3, likewise for the columns
        const int b0 = (hd & 0xff) - 64, b1 = ((hd >> 8) & 0xff) - 64;
        const int r0 = b0 + (((hd >> 16) & 1) ? 0 : 1), k0 = b1 + (((hd >> 17) & 1) ? 0 : 1);
        const int sr = 4 * (st >> 2), sc = 4 * (st & 3);
        const bool in = hd >= 0 && r0 <= sr + 3 && b0 + 2 * MW >= sr && k0 <= sc + 3 &&
                        b1 + 2 * MW >= sc;
        const uint64_t bal = __builtin_amdgcn_ballot_w64(in);
        const int pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
        if (in) s_list[st][cnt + pos] = (64 * h + lane) | ((hd & 0xffff) << 8);
        cnt += __popcll(bal);
      }
      const int c4 = (cnt + 3) & ~3;  // <= NB
      if (lane < c4 - cnt)
        s_list[st][cnt + lane] = NB | ((64 + 4 * (st >> 2)) << 8) | ((64 + 4 * (st & 3)) << 16);
      __builtin_amdgcn_wave_barrier();
      for (int g = 0; g < c4; g += 4) {
        // lane (kk, j) takes item g + kk of the sub-tile's list. An entry on
        // the list reaches the sub-tile, so the cell offsets row - origin
        // and col - origin lie in [-3, 2m + 3] and index the zero-padded
        // factor rows; cells outside the footprint read a zero factor, and a
        // padding item reads entry NB (zero factors and samples).
        const int it = s_list[st][g + kk];
        const int kc = it & 0xff;
        const float fa = s_ay[kc * YS + 4 + row + 64 - ((it >> 8) & 0xff)];
        const float fb = s_bx[kc * XS + 4 + col + 64 - ((it >> 16) & 0xff)];
        const float bw = fa * fb;
        const float4 a4 = *reinterpret_cast<const float4*>(s_c + kc * 2 * kGatherRhs + j * 4);
        const float av[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
          acc[q][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mb], bw, acc[q][mb], 0, 0, 0);
      }
    }
  }

  // output, in two passes of 16 right-hand sides: the two waves of each
  // band of four tile rows transpose their sub-tiles through the band's LDS
  // area, so that a store writes 16 consecutive cells of one right-hand
  // side: to the grid, or to the unit's partial slot (cells in tile order).
  // (Accumulator element v of lane l in block mb: row m = 16 mb + 4 (l >> 4)
  // + v of the 64 (m < 32: real part of right-hand side m, else imaginary
  // part of m - 32), cell l & 15 of the sub-tile; pass p takes the blocks p
  // and 2 + p, right-hand sides 16 p + 4 (l >> 4) + v.)
  const int band = wave >> 1;
  constexpr int RH = kGatherRhs / 2;
  float* tr = lds_f + band * (RH * 65 * 2);
  const int cj = lane & 15;
  float* base = tr + (4 * (lane >> 4) * 65 + (cj >> 2) * 16 + (cj & 3)) * 2;
  float2* dst;
  int64_t rs;
  if (slot < 0) {
    dst = grid + (int64_t)(16 * t0 + 4 * band + (lane >> 4)) * a.g.Ms + 16 * t1 + cj;
    rs = grid_rs;
  } else {
    dst = part + (int64_t)slot * 256 + 64 * band + lane;
    rs = part_rs;
  }
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    __syncthreads();  // the LDS is free: the rounds, or the previous pass, are done with it
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int sc = (2 * wave + q) & 3;
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) base[(v * 65 + 4 * sc) * 2 + c] = acc[q][p + 2 * c][v];
    }
    __syncthreads();
    // the band's two waves store 8 right-hand sides each
    const int r0 = (RH / 2) * (wave & 1);
    const int r1 = min(r0 + RH / 2, nrhs - rhs0 - RH * p);
    float2* d = dst + (int64_t)(rhs0 + RH * p + r0) * rs;
#pragma unroll 2
    for (int rr = r0; rr < r1; ++rr, d += rs) {
      const float* src = tr + (rr * 65 + lane) * 2;
      *d = make_float2(src[0], src[1]);
    }
  }
}

// The weighted samples c = w f of every group of 32 right-hand sides
// node-major: fT[g][j] = 16 float4, float4 q = (Re c_q, Re c_16+q, Im c_q,
// Im c_16+q) with c_r = w_j f[32 g + r][j] (caller order j, its weight found
// through the inverse node permutation; zero for right-hand sides past nrhs),
// the layout in which the gather stages them. Tiles of 32 right-hand sides x
// 64 nodes through LDS, loads and stores coalesced.
__global__ __launch_bounds__(256) void gather_transpose_kernel(const float2* __restrict__ f,
                                                               int64_t f_rs, int64_t N, int nrhs,
                                                               const float2* __restrict__ w,
                                                               const int32_t* __restrict__ iperm,
                                                               float4* __restrict__ fT) {
  __shared__ float2 t[64][kGatherRhs + 1];
  __shared__ float2 s_wv[64];
  const int64_t j0 = (int64_t)blockIdx.x * 64;
  const int g = blockIdx.y;
  const int tid = threadIdx.x;
  if (tid < 64) s_wv[tid] = j0 + tid < N ? w[iperm[j0 + tid]] : make_float2(0.f, 0.f);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int e = tid + 256 * q;
    const int r = e / 64, jj = e % 64;
    const int rg = g * kGatherRhs + r;
    t[jj][r] = (rg < nrhs && j0 + jj < N) ? f[(int64_t)rg * f_rs + j0 + jj] : make_float2(0.f, 0.f);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + 256 * q;
    const int jj = e >> 4, qq = e & 15;
    if (j0 + jj < N) {
      const float2 wv = s_wv[jj], u = t[jj][qq], v = t[jj][16 + qq];
      fT[((int64_t)g * N + j0 + jj) * 16 + qq] =
          make_float4(wv.x * u.x - wv.y * u.y, wv.x * v.x - wv.y * v.y, wv.x * u.y + wv.y * u.x,
                      wv.x * v.y + wv.y * v.x);
    }
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
  // the loads of up to 8 units are issued before their adds (unit order kept)
  for (int k0 = 0; k0 < cnt; k0 += 8) {
    float2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      v[u] = k0 + u < cnt ? src[(int64_t)(k0 + u) * 256] : make_float2(0.0f, 0.0f);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (k0 + u < cnt) {
        sx.add(v[u].x);
        sy.add(v[u].y);
      }
    }
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
  hipLaunchKernelGGL((spread_gather_kernel<MW>), blocks, dim3(kGatherNt), GatherLds<MW>::bytes, s, a,
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
                     0, s, a.f, a.f_rs, a.g.N, nrhs, reinterpret_cast<const float2*>(a.w), ga.iperm,
                     reinterpret_cast<float4*>(ga.fT));
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
