// Spreading (adjoint NFFT step 1) and window sums (NFFT step 3).
//
// Work decomposition: the oversampled grid is cut into tiles of T^d cells;
// the nodes, sorted by tile at plan time, form work items of at most a few
// hundred nodes of one tile. A work-group owns one work item and one
// right-hand side. Its nodes touch only the padded tile of (T + 2m)^d cells
// around the tile, which lives in LDS:
//   spread : nodes are spread into the LDS tile by groups of lanes, each
//            lane owning footprint cells (d <= 2: 16-lane groups per node,
//            d = 3: one wave per node); the finished padded tile is written
//            out whole. Tiles split into several work items are summed by
//            tile_reduce, and the first FFT pass merges the tile partials
//            into grid cells.
//   sums   : the padded tile is gathered from the grid (periodically
//            wrapped) into LDS, and every thread evaluates its nodes' sums.
// Nodes exactly on a grid line (offset zero) get the extra closed-edge cell;
// a wave takes the (2m+1)-wide loop only when one of its lanes needs it.
#include <type_traits>

#include "spread_common.hpp"
#include "spread_group.hpp"

namespace nfft {

// ----------------------------------------------------------------------------
// Spreading for d = 3, one wave per node. A batch of SB nodes is staged in LDS
// (the 2m window factors of each dimension by Horner, c_j and the packed
// cells), the jobs spread over the work-group. A wave then takes one node at a
// time; its lanes own cells (i1, i2) of the footprint plane (64 at a time) and
// walk the 2m footprint planes i0, whose factor every lane holds in registers.
//   float32: two waves, one per component: each keeps a float32 plane of its
//            own (real or imaginary part) and updates it by batched
//            read-modify-write; no two lanes touch one cell, and float32 LDS
//            atomics, far slower on this target, are not used.
//   float64: four waves share one tile through float64 LDS atomics.
// A node on a grid line (extra closed-edge cells) takes a slower path over
// the full (2m+1)^3 footprint.
template <typename R, int MW>
struct Stage3 {
  static constexpr int SB = 64;                   // nodes per staged batch (one per lane)
  static constexpr int K2 = 2 * MW;
  static constexpr int SW = 3 * K2;               // psi_0, psi_1, psi_2
  static constexpr size_t bytes = (size_t)SB * SW * sizeof(R);
};

// Value of lane n (uniform n) of a wave-wide register.
__device__ __forceinline__ uint32_t lane_value(uint32_t v, int n) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, n);
}
__device__ __forceinline__ float lane_value(float v, int n) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), n));
}
__device__ __forceinline__ double lane_value(double v, int n) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), n);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), n);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <typename R, int MW, int NW, int TT>
__global__ __launch_bounds__(64 * NW) void spread3_kernel(SpreadArgs<R> a) {
  constexpr int NT = 64 * NW;
  constexpr int K2 = 2 * MW;
  constexpr int KP = K2 * K2;                 // footprint cells of the (1,2) plane
  constexpr int NPASS = (KP + 63) / 64;
  constexpr int DEG = PolyDeg<R>::value;
  constexpr int SB = Stage3<R, MW>::SB;
  constexpr int SW = Stage3<R, MW>::SW;
  constexpr bool SPLIT = std::is_same<R, float>::value;  // one component per wave
  static_assert(!SPLIT || NW == 2, "float32: one wave per component");
  extern __shared__ double lds_d[];
  const int item = blockIdx.x;
  const int rhs = blockIdx.y;
  // padded tile edge: a compile-time constant for the usual tile edge
  const int P = TT > 0 ? TT + 2 * MW : a.g.P;
  const int PP = P * P;
  const int Ptot = a.g.Ptot;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const size_t acc_bytes = (size_t)2 * Ptot * sizeof(R);
  R* stage = reinterpret_cast<R*>(reinterpret_cast<unsigned char*>(lds_d) + acc_bytes);
  for (int i = tid; i < (int)(acc_bytes / sizeof(double)); i += NT) lds_d[i] = 0.0;

  const int64_t N = a.g.N;
  const int start = a.item_start[item];
  const int cnt = a.item_count[item];
  const cplx<R>* f = a.f + rhs * a.f_rs;
  const R edge = a.edge;
  // float32: this wave's component plane; float64: both planes, shared
  R* plane = reinterpret_cast<R*>(lds_d) + (SPLIT ? (wave & 1) * Ptot : 0);
  const int comp = SPLIT ? (wave & 1) : 0;
  const int first = SPLIT ? 0 : wave;         // first node of this wave in a batch
  constexpr int NS = SPLIT ? 1 : NW;          // node stride

  // With a padded edge of 16 the 2m rows a wave touches would share LDS
  // banks (a row is 16 elements; 32 banks of 4 bytes). The column index is
  // XOR-ed with 8 on every other row, or pair of rows, so that the rows one
  // LDS cycle serves fall on distinct banks: float64 planes (8-byte accesses,
  // 16 lanes = 2 rows per cycle) flip on row bit 0, float32 planes (4-byte
  // accesses, 32 lanes = 4 rows per cycle, two rows per 32 banks) on row
  // bit 1.
  const bool swz = P == 16;
  constexpr int SWB = SPLIT ? 5 : 4;  // bit of the cell index that flips the column
  auto sw = [swz](int c) { return swz ? c ^ (((c >> SWB) & 1) << 3) : c; };

  // this lane's cell of the footprint plane in each pass
  int q1[NPASS], q2[NPASS];
#pragma unroll
  for (int pass = 0; pass < NPASS; ++pass) {
    const int q = lane + 64 * pass;
    q1[pass] = q < KP ? q / K2 : 0;
    q2[pass] = q < KP ? q % K2 : 0;
  }

  // Node data of the staged batch in registers: lane l holds node b0 + l
  // (cell word and c_j). A wave reads node n's with readlane, so a node's
  // addresses never wait on LDS, where they would queue behind the previous
  // node's writes (LDS operations complete in order).
  uint32_t myloc = 0;
  R myc0 = 0, myc1 = 0;  // float32: this wave's component; float64: re, im

  // per-node values a wave needs, read one node ahead
  struct Hdr {
    uint32_t L;
    R c0, c1;  // float32: this wave's component (c1 unused); float64: re, im
    R w1[NPASS], w2[NPASS];  // psi_1, psi_2 at this lane's cells (product taken at use)
    R p0[K2];
  };
  auto load_hdr = [&](int n) {
    Hdr h;
    const R* o = stage + n * SW;
    h.L = lane_value(myloc, n);
    h.c0 = lane_value(myc0, n);
    h.c1 = SPLIT ? (R)0 : lane_value(myc1, n);
#pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
      h.w1[pass] = o[K2 + q1[pass]];
      h.w2[pass] = o[2 * K2 + q2[pass]];
    }
#pragma unroll
    for (int i0 = 0; i0 < K2; ++i0) h.p0[i0] = o[i0];
    return h;
  };

  auto spread_node = [&](const Hdr& h, int n) {
    const uint32_t L = h.L;
    const int l0 = (int)(L & kLocMask);
    const int l1 = (int)((L >> kLocBits) & kLocMask);
    const int l2 = (int)((L >> (2 * kLocBits)) & kLocMask);
    if (((L >> kEdgeShift) & 7u) == 0) {
#pragma unroll
      for (int pass = 0; pass < NPASS; ++pass) {
        if (lane + 64 * pass >= KP) continue;
        // the swizzle depends on the row only, not on the plane
        const int cell0 = sw((l0 + 1) * PP + (l1 + 1 + q1[pass]) * P + (l2 + 1 + q2[pass]));
        if constexpr (SPLIT) {
          const R v = h.c0 * (h.w1[pass] * h.w2[pass]);
          R* t = plane + cell0;
          R cur[K2];
#pragma unroll
          for (int i0 = 0; i0 < K2; ++i0) cur[i0] = t[i0 * PP];
#pragma unroll
          for (int i0 = 0; i0 < K2; ++i0) cur[i0] += v * h.p0[i0];
#pragma unroll
          for (int i0 = 0; i0 < K2; ++i0) t[i0 * PP] = cur[i0];
        } else {
          const R w12 = h.w1[pass] * h.w2[pass];
          const R vx = h.c0 * w12, vy = h.c1 * w12;
#pragma unroll
          for (int i0 = 0; i0 < K2; ++i0) {
            lds_add(lds_d + cell0 + i0 * PP, vx * h.p0[i0]);
            lds_add(lds_d + Ptot + cell0 + i0 * PP, vy * h.p0[i0]);
          }
        }
      }
    } else {
      // full closed footprint: index 0 of each dimension is the edge cell
      const R* o = stage + n * SW;
      const bool e0 = (L >> kEdgeShift) & 1u, e1 = (L >> (kEdgeShift + 1)) & 1u,
                 e2 = (L >> (kEdgeShift + 2)) & 1u;
      constexpr int KE = K2 + 1;
      for (int q = lane; q < KE * KE * KE; q += 64) {
        const int k0 = q / (KE * KE), k1 = (q / KE) % KE, k2 = q % KE;
        const R w0 = k0 ? o[k0 - 1] : (e0 ? edge : (R)0);
        const R w1 = k1 ? o[K2 + k1 - 1] : (e1 ? edge : (R)0);
        const R w2 = k2 ? o[2 * K2 + k2 - 1] : (e2 ? edge : (R)0);
        const R wv = w0 * w1 * w2;
        const int cell = sw(((l0 + k0) * P + (l1 + k1)) * P + (l2 + k2));
        if constexpr (SPLIT) {
          plane[cell] += h.c0 * wv;
        } else {
          lds_add(lds_d + cell, h.c0 * wv);
          lds_add(lds_d + Ptot + cell, h.c1 * wv);
        }
      }
    }
  };

  for (int b0 = 0; b0 < cnt; b0 += SB) {
    const int nb = (cnt - b0) < SB ? (cnt - b0) : SB;
    __syncthreads();  // tile zeroed / previous batch consumed
    for (int job = tid; job < 3 * SB; job += NT) {
      const int n = job % SB, kind = job / SB;
      if (n >= nb) continue;
      const int i = start + b0 + n;
      R* o = stage + n * SW;
      const R y = (R)2 * a.frac[kind * N + i] - (R)1;
#pragma unroll
      for (int q = 0; q < K2; ++q) o[kind * K2 + q] = horner<R>(a.coef + q * (DEG + 1), y);
    }
    if (lane < nb) {
      const int i = start + b0 + lane;
      myloc = a.loc[i];
      const cplx<R> c = cmul<R>(a.w[i], f[a.perm[i]]);
      myc0 = (SPLIT && comp) ? c.y : c.x;
      myc1 = c.y;
    }
    __syncthreads();
    // two nodes per trip with the header of the next one loaded ahead; the
    // loads are issued on every trip (for the last node again past the end,
    // then unused) and headers are never copied, so no wait for them joins
    // paths or falls behind the previous node's LDS writes
    if (first >= nb) continue;
    Hdr h0 = load_hdr(first), h1;
    for (int n = first; n < nb; n += 2 * NS) {
      h1 = load_hdr(n + NS < nb ? n + NS : nb - 1);
      spread_node(h0, n);
      if (n + NS >= nb) break;
      h0 = load_hdr(n + 2 * NS < nb ? n + 2 * NS : nb - 1);
      spread_node(h1, n + NS);
    }
  }
  __syncthreads();
  const int slot = a.item_slot[item];
  cplx<R>* out = slot < 0 ? a.tilep + rhs * a.tile_rs + (int64_t)a.item_bin[item] * Ptot
                          : a.itemp + rhs * a.item_rs + (int64_t)slot * Ptot;
  const R* re = reinterpret_cast<const R*>(lds_d);
  for (int i = tid; i < Ptot; i += NT) out[i] = mkc<R>(re[sw(i)], re[Ptot + sw(i)]);
}

template <typename R>
__global__ __launch_bounds__(256) void tile_reduce_kernel(ReduceArgs<R> a) {
  const int Ptot = a.g.Ptot;
  const int chunks = (Ptot + blockDim.x - 1) / blockDim.x;
  const int tix = blockIdx.x / chunks;
  const int cell = (blockIdx.x - tix * chunks) * blockDim.x + threadIdx.x;
  if (cell >= Ptot) return;
  const int s0 = a.multi_first[tix], s1 = a.multi_first[tix + 1];
  const cplx<R>* itemp = a.itemp + blockIdx.y * a.item_rs;
  // slot k goes to compensated sum (k - s0) mod 4; the four are combined in
  // a fixed order, so the result does not depend on timing. The loads of up
  // to 16 slots are issued before the first add (one memory latency for a
  // tile of at most 16 items).
  KSum<R> sx[4], sy[4];
  for (int base = s0; base < s1; base += 16) {
    cplx<R> v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      v[u] = base + u < s1 ? itemp[(int64_t)(base + u) * Ptot + cell] : mkc<R>(0, 0);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (base + u < s1) {
        sx[u & 3].add(v[u].x);
        sy[u & 3].add(v[u].y);
      }
    }
  }
  KSum<R> tx, ty;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    tx.add(sx[u].s);
    tx.add(sx[u].c);
    ty.add(sy[u].s);
    ty.add(sy[u].c);
  }
  a.tilep[blockIdx.y * a.tile_rs + (int64_t)a.multi_bin[tix] * Ptot + cell] =
      mkc<R>(tx.value(), ty.value());
}

template <typename R>
hipError_t launch_tile_reduce(const ReduceArgs<R>& a, int nrhs, hipStream_t s) {
  if (a.nmulti == 0) return hipSuccess;
  const int chunks = (a.g.Ptot + 255) / 256;
  hipLaunchKernelGGL(tile_reduce_kernel<R>, dim3(a.nmulti * chunks, nrhs), dim3(256), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_tile_reduce<float>(const ReduceArgs<float>&, int, hipStream_t);
template hipError_t launch_tile_reduce<double>(const ReduceArgs<double>&, int, hipStream_t);

template <typename R, int D, int MW, bool EDGE>
__device__ __forceinline__ cplx<R> sum_node(const cplx<R>* tile, int P, const int* l,
                                            const R (*psi)[2 * MW + 1]) {
  constexpr int K0 = EDGE ? 0 : 1;
  constexpr int KE = 2 * MW + 1;
  R sx = 0, sy = 0;
  if constexpr (D == 1) {
#pragma unroll
    for (int i0 = K0; i0 < KE; ++i0) {
      const cplx<R> v = tile[l[0] + i0];
      sx += v.x * psi[0][i0];
      sy += v.y * psi[0][i0];
    }
  } else if constexpr (D == 2) {
#pragma unroll
    for (int i0 = K0; i0 < KE; ++i0) {
      const cplx<R>* row = tile + (l[0] + i0) * P + l[1];
      R rx = 0, ry = 0;
#pragma unroll
      for (int i1 = K0; i1 < KE; ++i1) {
        const cplx<R> v = row[i1];
        rx += v.x * psi[1][i1];
        ry += v.y * psi[1][i1];
      }
      sx += rx * psi[0][i0];
      sy += ry * psi[0][i0];
    }
  } else {
#pragma unroll
    for (int i0 = K0; i0 < KE; ++i0) {
      R px = 0, py = 0;
#pragma unroll
      for (int i1 = K0; i1 < KE; ++i1) {
        const cplx<R>* row = tile + ((l[0] + i0) * P + (l[1] + i1)) * P + l[2];
        R rx = 0, ry = 0;
#pragma unroll
        for (int i2 = K0; i2 < KE; ++i2) {
          const cplx<R> v = row[i2];
          rx += v.x * psi[2][i2];
          ry += v.y * psi[2][i2];
        }
        px += rx * psi[1][i1];
        py += ry * psi[1][i1];
      }
      sx += px * psi[0][i0];
      sy += py * psi[0][i0];
    }
  }
  return mkc<R>(sx, sy);
}

template <typename R, int D, int MW>
__global__ __launch_bounds__(256) void interp_kernel(InterpArgs<R> a) {
  extern __shared__ unsigned char smem_raw[];
  cplx<R>* tile = reinterpret_cast<cplx<R>*>(smem_raw);
  const int item = blockIdx.x;
  const int rhs = blockIdx.y;
  const int P = a.g.P;
  const int Ptot = a.g.Ptot;
  const int Ms = a.g.Ms;
  const int nb = a.g.nb;
  // tile origin (in cells) of this work item's tile, per dimension
  int org[3] = {0, 0, 0};
  {
    int bb = a.item_bin[item];
    for (int t = D - 1; t >= 0; --t) {
      org[t] = (bb % nb) * a.g.T - a.g.m;
      bb /= nb;
    }
  }
  const cplx<R>* grid = a.grid + rhs * a.grid_rs;
  // rem / P as floor((rem + 1/2) / P) in float: for rem < 2^22 the rounding
  // error (about rem / P * 2^-23) stays below the distance 1/(2P) of the
  // exact quotient to an integer, and a tile in LDS has far fewer cells;
  // the tile edge divides M_sigma, so tile cells lie in [-m, M_sigma + m)
  // with m <= M_sigma and one wrap each way suffices
  const float invP = 1.0f / (float)P;
  for (int i = threadIdx.x; i < Ptot; i += blockDim.x) {
    int rem = i;
    int64_t lin = 0;
    int p[3] = {0, 0, 0};
    for (int t = D - 1; t >= 0; --t) {
      const int q = (int)(((float)rem + 0.5f) * invP);
      p[t] = rem - q * P;
      rem = q;
    }
    for (int t = 0; t < D; ++t) {
      int c = org[t] + p[t];
      c = c < 0 ? c + Ms : (c >= Ms ? c - Ms : c);
      lin = lin * Ms + c;
    }
    tile[i] = grid[lin];
  }
  // float64: the window polynomials beside the tile (every lane of a wave
  // reads the same coefficient, an LDS broadcast; measured faster than the
  // cached device reads in float64, slower in float32)
  constexpr bool kLdsCoef = std::is_same<R, double>::value;
  constexpr int NCF = 2 * MW * (PolyDeg<R>::value + 1);
  R* cf = reinterpret_cast<R*>(tile + Ptot);
  if constexpr (kLdsCoef)
    for (int i = threadIdx.x; i < NCF; i += blockDim.x) cf[i] = a.coef[i];
  __syncthreads();

  const int64_t N = a.g.N;
  const int start = a.item_start[item];
  const int cnt = a.item_count[item];
  cplx<R>* f = a.f + rhs * a.f_rs;
  for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
    const int i = start + k;
    const uint32_t L = a.loc[i];
    int l[D];
    R psi[D][2 * MW + 1];
    bool any_edge = false;
    // the plan's window factor table (pairs per footprint cell) holds the
    // same values as the polynomials
    const bool tab = D == 2 && a.psi != nullptr;
    R pairs[4 * MW];
    if (tab) load_factors<R, 4 * MW>(pairs, a.psi + (int64_t)i * (4 * MW));
    R y[D];
    bool e[D];
#pragma unroll
    for (int t = 0; t < D; ++t) {
      l[t] = (int)((L >> (kLocBits * t)) & kLocMask);
      e[t] = (L >> (kEdgeShift + t)) & 1u;
      any_edge |= e[t];
      y[t] = tab ? (R)0 : (R)2 * a.frac[t * N + i] - (R)1;
      if (tab) {
        psi[t][0] = e[t] ? a.edge : (R)0;
#pragma unroll
        for (int c = 0; c < 2 * MW; ++c) psi[t][1 + c] = pairs[2 * c + t];
      }
    }
    if (!tab) kb_poly<R, MW, D>(y, e, a.edge, kLdsCoef ? cf : a.coef, psi);
    cplx<R> v;
    if (__any(any_edge))
      v = sum_node<R, D, MW, true>(tile, P, l, psi);
    else
      v = sum_node<R, D, MW, false>(tile, P, l, psi);
    const int j = a.perm[i];
    if (a.sub) {
      const cplx<R> u = a.sub[rhs * a.f_rs + j];
      v = mkc<R>(u.x - v.x, u.y - v.y);
    }
    f[j] = v;
  }
}

template <typename R, int D, int MW>
static hipError_t spread_dm(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  if constexpr (D <= 2) {
    // float32: private group tiles, 64 / 128 / 256 threads; float64: 256
    // threads sharing one tile
    if constexpr (std::is_same<R, float>::value) {
      if (a.planes == 2) {
        if (a.nt == 64) return spread_group_nt<R, D, MW, 64, true, 0>(a, nrhs, s);
        if (a.nt == 256) return spread_group_nt<R, D, MW, 256, true, 0>(a, nrhs, s);
        return spread_group_nt<R, D, MW, 128, true, 0>(a, nrhs, s);
      }
      if (a.nt == 64) return spread_group_nt<R, D, MW, 64, false, 0>(a, nrhs, s);
      if (a.nt == 256) return spread_group_nt<R, D, MW, 256, false, 0>(a, nrhs, s);
      return spread_group_nt<R, D, MW, 128, false, 0>(a, nrhs, s);
    } else {
      return spread_group_nt<R, D, MW, 256, false, 0>(a, nrhs, s);
    }
  } else {
    // d = 3: float32 two waves, one component plane each; float64 four
    // waves sharing one tile
    constexpr int NW = std::is_same<R, float>::value ? 2 : 4;
    const size_t lds = (size_t)2 * a.g.Ptot * sizeof(R) + Stage3<R, MW>::bytes;
    if (a.g.T == 8)
      hipLaunchKernelGGL((spread3_kernel<R, MW, NW, 8>), dim3(a.g.nsub, nrhs), dim3(64 * NW), lds, s, a);
    else
      hipLaunchKernelGGL((spread3_kernel<R, MW, NW, 0>), dim3(a.g.nsub, nrhs), dim3(64 * NW), lds, s, a);
  }
  return hipGetLastError();
}

template <typename R, int D, int MW>
static hipError_t interp_dm(const InterpArgs<R>& a, int nrhs, hipStream_t s) {
  size_t lds = (size_t)a.g.Ptot * sizeof(cplx<R>) +
               (std::is_same<R, double>::value ? 2 * MW * (PolyDeg<R>::value + 1) * sizeof(R) : 0);
  hipLaunchKernelGGL((interp_kernel<R, D, MW>), dim3(a.g.nsub, nrhs), dim3(256), lds, s, a);
  return hipGetLastError();
}

#define NFFT_DISPATCH_M(FN, R, D, ARGS, NRHS, S)   \
  switch (ARGS.g.m) {                              \
    case 1: return FN<R, D, 1>(ARGS, NRHS, S);     \
    case 2: return FN<R, D, 2>(ARGS, NRHS, S);     \
    case 3: return FN<R, D, 3>(ARGS, NRHS, S);     \
    case 4: return FN<R, D, 4>(ARGS, NRHS, S);     \
    case 5: return FN<R, D, 5>(ARGS, NRHS, S);     \
    case 6: return FN<R, D, 6>(ARGS, NRHS, S);     \
    case 7: return FN<R, D, 7>(ARGS, NRHS, S);     \
    case 8: return FN<R, D, 8>(ARGS, NRHS, S);     \
    default: return hipErrorInvalidValue;          \
  }

size_t spread_multi_lds_bytes(bool f64, int Ptot, int nr);

size_t spread_lds_bytes(int d, bool f64, int m, int T, int Ptot, int nt, int nr, int planes) {
  (void)T;
  const size_t rb = f64 ? 8 : 4;
  if (d <= 2) {
    if (nr > 1) return spread_multi_lds_bytes(f64, Ptot, nr);
    if (nr != 1) return 0;
    if (f64) return (size_t)2 * Ptot * 8 + (size_t)256 * (4 * rb + 4);
    if (nt != 64 && nt != 128 && nt != 256) return 0;
    // float32 private tiles: complex (8 bytes a cell) or one plane (4 bytes)
    return (size_t)(nt / 16) * Ptot * (planes == 2 ? 4 : 8) + (size_t)nt * (4 * rb + 4);
  }
  if (nr != 1) return 0;
  // Stage3: 64 nodes of 3 * 2m reals (cell words and c_j stay in registers)
  return (size_t)2 * Ptot * rb + (size_t)64 * (3 * 2 * m) * rb;
}

template <typename R>
hipError_t launch_spread(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  if (a.g.nsub == 0) return hipSuccess;
  if (a.mode == 2 && spread_rows_supported(a.g.d, a.g.P)) return launch_spread_rows<R>(a, nrhs, s);
  if (a.nr > 1 && a.g.d <= 2) return launch_spread_multi<R>(a, nrhs, s);
  if (a.mode == 7 && spread_mma_supported(a.g.d, a.g.T, !std::is_same<R, float>::value, a.g.m))
    return launch_spread_mma<R>(a, nrhs, s);
  if (a.mode == 7 && spread3_mma_supported(a.g.d, a.g.T, !std::is_same<R, float>::value, a.g.m))
    return launch_spread3_mma<R>(a, nrhs, s);
  if constexpr (std::is_same<R, float>::value) {
    if (a.mode == 5 && spread_reg_supported(a.g.d, a.g.T, false))
      return launch_spread_reg(a, nrhs, s);
  }
  if (a.mode == 3 && a.psi && a.g.d == 2) return launch_spread_pre<R>(a, nrhs, s);
  if (a.mode == 4 && a.g.d == 2) return launch_spread_late<R>(a, nrhs, s);
  switch (a.g.d) {
    case 1: NFFT_DISPATCH_M(spread_dm, R, 1, a, nrhs, s)
    case 2: NFFT_DISPATCH_M(spread_dm, R, 2, a, nrhs, s)
    case 3: NFFT_DISPATCH_M(spread_dm, R, 3, a, nrhs, s)
    default: return hipErrorInvalidValue;
  }
}

template <typename R>
hipError_t launch_interp(const InterpArgs<R>& a, int nrhs, hipStream_t s) {
  if (a.g.nsub == 0) return hipSuccess;
  switch (a.g.d) {
    case 1: NFFT_DISPATCH_M(interp_dm, R, 1, a, nrhs, s)
    case 2: NFFT_DISPATCH_M(interp_dm, R, 2, a, nrhs, s)
    case 3: NFFT_DISPATCH_M(interp_dm, R, 3, a, nrhs, s)
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_spread<float>(const SpreadArgs<float>&, int, hipStream_t);
template hipError_t launch_spread<double>(const SpreadArgs<double>&, int, hipStream_t);
template hipError_t launch_interp<float>(const InterpArgs<float>&, int, hipStream_t);
template hipError_t launch_interp<double>(const InterpArgs<double>&, int, hipStream_t);

}  // namespace nfft
