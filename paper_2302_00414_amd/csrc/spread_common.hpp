// Device helpers shared by the spreading kernels: float64 LDS atomics,
// compensated sums, DPP row broadcasts, Horner evaluation of the window
// polynomials and the per-node preparation of the lane-group kernels.
#pragma once

#include <type_traits>

#include "internal.hpp"
#include "window.hpp"

namespace nfft {

__device__ __forceinline__ void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Compensated (Neumaier) accumulation of one component.
template <typename R>
struct KSum {
  R s = 0, c = 0;
  __device__ __forceinline__ void add(R v) {
    const R t = s + v;
    if (fabs(s) >= fabs(v))
      c += (s - t) + v;
    else
      c += (v - t) + s;
    s = t;
  }
  __device__ __forceinline__ R value() const { return s + c; }
};

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// Value of lane I of this lane's 16-lane row (DPP row broadcast; every lane
// of the row reads an existing lane, so no lane keeps an old value and the
// move writes a fresh register).
template <int I>
__device__ __forceinline__ float row_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + I, 0xf, 0xf, false));
}
template <int I>
__device__ __forceinline__ double row_bcast(double v) {
  const long long b = __double_as_longlong(v);
  const int l = (int)(b & 0xffffffffLL), u = (int)(b >> 32);
  const int lo = __builtin_amdgcn_update_dpp(l, l, 0x150 + I, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(u, u, 0x150 + I, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <typename R>
__device__ __forceinline__ R horner(const R* c, R y) {
  constexpr int DEG = PolyDeg<R>::value;
  R v = c[DEG];
#pragma unroll
  for (int p = DEG - 1; p >= 0; --p) v = v * y + c[p];
  return v;
}

template <typename R> struct GroupAcc;
// float32: private padded tile per group, plain read-modify-write
template <> struct GroupAcc<float> {
  float2* tile;  // this group's tile
  __device__ __forceinline__ void add(int cell, float x, float y) {
    float2 v = tile[cell];
    v.x += x;
    v.y += y;
    tile[cell] = v;
  }
};
// float64: shared padded tile (real and imaginary planes), LDS atomics
template <> struct GroupAcc<double> {
  double* re;
  double* im;
  __device__ __forceinline__ void add(int cell, double x, double y) {
    lds_add(re + cell, x);
    lds_add(im + cell, y);
  }
};

// Per-node values a group needs for one node: the column factor times c_j
// (vx, vy, lane k), the 2m row factors (rw, broadcast to every lane), the
// node's tile-local cell and its on-grid-line flags.
// acc[i] += (v of lane i of this 16-lane row) * x for i < K (K <= 16): the row
// broadcast is the DPP operand modifier of the multiply-add itself, one
// instruction per footprint row instead of a broadcast move and a
// multiply-add. The leading s_nop covers the wait states a DPP read needs
// after an EXEC write by a scalar instruction (five) or a VGPR write by a
// vector instruction (two); the operands are plain registers, nothing is
// loaded.
#define NFFT_FMAC_BCAST(I, NOP)                                                              \
  asm volatile(NOP "v_fmac_f32_dpp %0, %1, %2 row_newbcast:" #I " row_mask:0xf bank_mask:0xf" \
               : "+v"(acc[I])                                                                \
               : "v"(v), "v"(x))
template <int K>
__device__ __forceinline__ void fmac_row_bcast(float (&acc)[K], float v, float x) {
  static_assert(K >= 1 && K <= 16, "one 16-lane row");
  NFFT_FMAC_BCAST(0, "s_nop 4\n");
  if constexpr (K > 1) NFFT_FMAC_BCAST(1, "");
  if constexpr (K > 2) NFFT_FMAC_BCAST(2, "");
  if constexpr (K > 3) NFFT_FMAC_BCAST(3, "");
  if constexpr (K > 4) NFFT_FMAC_BCAST(4, "");
  if constexpr (K > 5) NFFT_FMAC_BCAST(5, "");
  if constexpr (K > 6) NFFT_FMAC_BCAST(6, "");
  if constexpr (K > 7) NFFT_FMAC_BCAST(7, "");
  if constexpr (K > 8) NFFT_FMAC_BCAST(8, "");
  if constexpr (K > 9) NFFT_FMAC_BCAST(9, "");
  if constexpr (K > 10) NFFT_FMAC_BCAST(10, "");
  if constexpr (K > 11) NFFT_FMAC_BCAST(11, "");
  if constexpr (K > 12) NFFT_FMAC_BCAST(12, "");
  if constexpr (K > 13) NFFT_FMAC_BCAST(13, "");
  if constexpr (K > 14) NFFT_FMAC_BCAST(14, "");
  if constexpr (K > 15) NFFT_FMAC_BCAST(15, "");
}
#undef NFFT_FMAC_BCAST

// Tile-local cell and on-grid-line flags of a d = 2 node.
struct Cell2 {
  int l0, l1;
  bool e0, e1;
};
__device__ __forceinline__ Cell2 decode_cell2(uint32_t L) {
  return {(int)(L & kLocMask), (int)((L >> kLocBits) & kLocMask), ((L >> kEdgeShift) & 1u) != 0,
          ((L >> (kEdgeShift + 1)) & 1u) != 0};
}

template <typename R, int K2>
struct NodePrep {
  R vx, vy, p0, cx, cy;
  R q1;        // column factor of lane k, from the precomputed table
  R y0, y1;    // offsets (late evaluation: the window is evaluated where it is used)
  uint32_t L;  // cell word as loaded (decoded where it is used)
  R rw[K2];
  int l0, l1;
  bool e0, e1;
};

template <typename R, int D, int K2>
__device__ __forceinline__ void prep_node(NodePrep<R, K2>& h, R y0, R y1, R cx, R cy, uint32_t L,
                                          const R* cf) {
  h.cx = cx;
  h.cy = cy;
  h.l0 = (int)(L & kLocMask);
  h.e0 = (L >> kEdgeShift) & 1u;
  h.p0 = horner<R>(cf, y0);
  if constexpr (D == 1) {
    h.vx = cx * h.p0;
    h.vy = cy * h.p0;
    h.l1 = 0;
    h.e1 = false;
  } else {
    h.l1 = (int)((L >> kLocBits) & kLocMask);
    h.e1 = (L >> (kEdgeShift + 1)) & 1u;
    const R p1 = horner<R>(cf, y1);
    h.vx = cx * p1;
    h.vy = cy * p1;
    static_for<0, K2>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      h.rw[I] = row_bcast<I>(h.p0);
    });
  }
}

// K2 consecutive reals of the window factor table into dst: a node's row of
// 2 * K2 reals starts 16-byte aligned, so either half allows these loads.
template <typename R, int K2>
__device__ __forceinline__ void load_factors(R* dst, const R* q) {
  constexpr int VW = (K2 * sizeof(R)) % 16 == 0 ? 16 / sizeof(R) : 8 / sizeof(R);
  using V = typename std::conditional<VW * sizeof(R) == 16, float4, float2>::type;
  static_for<0, K2 / VW>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    const V v = reinterpret_cast<const V*>(q)[I];
    __builtin_memcpy(dst + I * VW, &v, sizeof(V));
  });
}

// The same values from the table of window factors precomputed at plan time:
// q points to the node's 2m pairs (dimension-0 factor, dimension-1 factor) of
// footprint cells 0..2m-1. Lane k loads pair k: p0 is the row factor it
// broadcasts to its group where the factors are used, q1 its column factor
// (rw, vx, vy and the decoded cell word are left to the caller, so nothing
// waits for the loads here).
template <typename R, int K2>
__device__ __forceinline__ void prep_node_pre(NodePrep<R, K2>& h, const R* q, R cx, R cy,
                                              uint32_t L, int k) {
  using V2 = typename std::conditional<std::is_same<R, float>::value, float2, double2>::type;
  h.cx = cx;
  h.cy = cy;
  h.L = L;
  const int kk = k < K2 ? k : 0;
  const V2 pr = reinterpret_cast<const V2*>(q)[kk];
  h.p0 = pr.x;
  h.q1 = pr.y;
}

}  // namespace nfft
