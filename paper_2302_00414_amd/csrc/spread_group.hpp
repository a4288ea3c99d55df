// Spreading for d <= 2 by 16-lane groups (one right-hand side per
// work-group), shared by the kernel that evaluates the window per call and the
// one that reads window factors precomputed at plan time.
#pragma once

#include <type_traits>

#include "spread_common.hpp"

namespace nfft {

// ----------------------------------------------------------------------------
// Spreading for d <= 2 by lane groups. A group is one 16-lane DPP row; it
// takes one node at a time and lane k owns footprint column k (the window
// polynomial k, whose coefficients the lane keeps in registers). The row
// factor of footprint row i is computed by lane i and broadcast to the group
// with a DPP row broadcast, so every cell update is one multiply chain and
// one LDS update of a row segment of consecutive cells.
//   float32: every group accumulates into its own padded tile (plain
//            read-modify-write, no atomics; float32 LDS atomics are slow on
//            this target); the group tiles are summed with compensation at
//            the end.
//   float64: all groups accumulate into one padded tile with float64 LDS
//            atomics.
// A batch of nodes is first staged in LDS by the whole work-group (one node
// per thread: offsets, c_j = w_j f_j and the packed cells).
//   WS (window source, d = 2): 0 = offsets, cell words and c_j staged in
//            LDS, the window evaluated when a node is prepared; 1 = the 2m
//            window factors per dimension from the table precomputed at plan
//            time; 2 = evaluated in the step from offsets loaded from device
//            memory. With 1 and 2 only c_j is staged, the cell word and the
//            factors (or offsets) of a node are loaded from device memory two
//            nodes ahead, and the row factors reach the group by DPP; all three
//            give the same values.

template <typename R, int D, int MW, int NT, int TT, bool CS, int WS>
__global__ __launch_bounds__(NT) void spread_group_kernel(SpreadArgs<R> a) {
  static_assert(D <= 2 && 2 * MW <= 16, "group spreading covers d <= 2, m <= 8");
  static_assert(WS == 0 || D == 2, "the table and the late evaluation are laid out for d = 2");
  constexpr bool PRE = WS != 0;   // node data from device memory, loaded ahead
  constexpr bool TAB = WS == 1;   // window factors from the plan's table
  static_assert(!CS || std::is_same<R, float>::value, "component split is a float32 layout");
  constexpr int DEG = PolyDeg<R>::value;
  constexpr int NG = NT / 16;            // groups per work-group
  constexpr int K2 = 2 * MW;             // footprint columns
  constexpr bool PRIV = std::is_same<R, float>::value;
  // CS: groups 2q and 2q+1 take the same nodes, for the real and the
  // imaginary part, each into a float32 plane of its own (half the LDS of a
  // complex tile per group, so twice the groups fit).
  constexpr int NODE_GROUPS = CS ? NG / 2 : NG;
  extern __shared__ double lds_d[];
  const int item = blockIdx.x;
  const int rhs = blockIdx.y;
  // padded tile edge: a compile-time constant for the usual tile edge
  const int P = TT > 0 ? TT + 2 * MW : a.g.P;
  const int Ptot = a.g.Ptot;
  const int tid = threadIdx.x;
  const int grp = tid >> 4;
  const int k = tid & 15;
  const int comp = CS ? (grp & 1) : 0;
  const int ngrp = CS ? (grp >> 1) : grp;  // node group

  // LDS layout: accumulation tile(s), then the node staging area
  unsigned char* base = reinterpret_cast<unsigned char*>(lds_d);
  const size_t acc_bytes = CS     ? (size_t)NG * Ptot * sizeof(float)
                           : PRIV ? (size_t)NG * Ptot * sizeof(float2)
                                  : (size_t)2 * Ptot * sizeof(double);
  // staged per node: c_j, and with WS = 0 also the offsets and the cell word
  // (with WS = 1, 2 those come from device memory; the smaller staging area
  // lets one more work-group share a compute unit)
  R* st_cx = reinterpret_cast<R*>(base + acc_bytes);
  R* st_cy = st_cx + NT;
  R* st_y0 = st_cy + NT;
  R* st_y1 = st_y0 + NT;
  uint32_t* st_loc = reinterpret_cast<uint32_t*>(st_y1 + NT);
  // CS: this group's component of c_j stands in for cx (cy unused)
  const R* st_c0 = (CS && comp) ? st_cy : st_cx;

  for (int i = tid; i < (int)(acc_bytes / sizeof(double)); i += NT) lds_d[i] = 0.0;
  GroupAcc<R> acc;
  float* ptile = nullptr;  // CS: this group's float32 plane
  if constexpr (CS) {
    ptile = reinterpret_cast<float*>(lds_d) + (size_t)grp * Ptot;
  } else if constexpr (PRIV) {
    acc.tile = reinterpret_cast<float2*>(lds_d) + (size_t)grp * Ptot;
  } else {
    acc.re = lds_d;
    acc.im = lds_d + Ptot;
  }
  auto add1 = [&](int cell, R x, R y) {
    if constexpr (CS) {
      ptile[cell] += x;
    } else {
      acc.add(cell, x, y);
    }
  };

  // this lane's window polynomial (column k; lanes past 2m keep polynomial 0)
  R cf[DEG + 1];
  if constexpr (!TAB) {
    const int kk = k < K2 ? k : 0;
#pragma unroll
    for (int p = 0; p <= DEG; ++p) cf[p] = a.coef[kk * (DEG + 1) + p];
  }
  const R edge = a.edge;
  __syncthreads();

  const int64_t N = a.g.N;
  const int start = a.item_start[item];
  const int cnt = a.item_count[item];
  const cplx<R>* f = a.f + rhs * a.f_rs;
  // one node per thread is loaded into registers one batch ahead, so the
  // global-memory latency of batch b+1 overlaps the spreading of batch b
  R pf0 = 0, pf1 = 0;
  uint32_t pfl = 0;
  cplx<R> pfw = mkc<R>(0, 0), pfs = mkc<R>(0, 0);
  auto issue = [&](int b) {
    if (b + tid < cnt) {
      const int i = start + b + tid;
      if constexpr (!PRE) {
        pf0 = a.frac[i];
        pf1 = D > 1 ? a.frac[N + i] : (R)0;
      }
      if constexpr (!PRE) pfl = a.loc[i];
      pfw = a.w[i];
      pfs = f[a.perm[i]];
    }
  };
  int b0 = 0;  // first node of the staged batch (within the item)
  auto prep = [&](NodePrep<R, K2>& h, int n) {
    if constexpr (PRE) {
      // the cell word from device memory, not the staging area: its wait is
      // then on the vector-memory counter and does not also wait for this
      // group's LDS writes issued since (LDS operations complete in order)
      const int64_t i = start + b0 + n;
      if constexpr (TAB) {
        prep_node_pre<R, K2>(h, a.psi + i * (2 * K2), st_c0[n], CS ? (R)0 : st_cy[n], a.loc[i], k);
      } else {
        h.cx = st_c0[n];
        h.cy = CS ? (R)0 : st_cy[n];
        h.L = a.loc[i];
        h.y0 = a.frac[i];      // offsets; the window is evaluated in the step
        h.y1 = a.frac[N + i];
      }
    } else
      prep_node<R, D, K2>(h, st_y0[n], st_y1[n], st_c0[n], CS ? (R)0 : st_cy[n], st_loc[n], cf);
  };
  // The node's tile-local cell. With WS = 1, 2 the cell word was loaded two
  // nodes ahead and is decoded only here: the empty asm keeps the
  // compiler from decoding it (and waiting for its load) earlier, e.g. where
  // the loop turns around.
  auto cell_of = [&](const NodePrep<R, K2>& h) -> Cell2 {
    if constexpr (PRE) {
      uint32_t L = h.L;
      asm volatile("" : "+v"(L));
      return decode_cell2(L);
    } else {
      return Cell2{h.l0, h.l1, h.e0, h.e1};
    }
  };
  // this lane's row factor (p0, broadcast to the group) and column factor
  // (q1) of a node prepared with WS = 1 or 2
  auto factors = [&](const NodePrep<R, K2>& h, R& p0, R& q1) {
    if constexpr (TAB) {
      p0 = h.p0;
      q1 = h.q1;
    } else {
      p0 = horner<R>(cf, (R)2 * h.y0 - (R)1);
      q1 = horner<R>(cf, (R)2 * h.y1 - (R)1);
    }
  };
  // closed-edge cells of a d = 2 node on a grid line: row 0 and column 0
  auto edges = [&](const NodePrep<R, K2>& h, const Cell2& c, R vx, R vy, int col, R p0) {
    if (c.e0 | c.e1) {
      if (c.e0 && k < K2) add1(c.l0 * P + col, vx * edge, vy * edge);
      if (c.e1 && k < K2) add1((c.l0 + 1 + k) * P + c.l1, h.cx * p0 * edge, h.cy * p0 * edge);
      if (c.e0 && c.e1 && k == 0) add1(c.l0 * P + c.l1, h.cx * edge * edge, h.cy * edge * edge);
    }
  };
  issue(0);
  for (b0 = 0; b0 < cnt; b0 += NT) {
    const int nb = (cnt - b0) < NT ? (cnt - b0) : NT;
    if (tid < nb) {
      const cplx<R> c = cmul<R>(pfw, pfs);
      if constexpr (!PRE) {
        st_y0[tid] = (R)2 * pf0 - (R)1;
        st_y1[tid] = (R)2 * pf1 - (R)1;
      }
      st_cx[tid] = c.x;
      st_cy[tid] = c.y;
      if constexpr (!PRE) st_loc[tid] = pfl;
    }
    if (b0 + NT < cnt) issue(b0 + NT);
    __syncthreads();
    // Software pipeline over this group's nodes n = ngrp, ngrp + NODE_GROUPS,
    // ...: the window factors of the next node are computed while the cell
    // reads of the current node are in flight. LDS operations of a wave
    // execute in order, so the next node's reads always see this node's
    // writes.
    // The next node's header. With WS = 1, 2 its loads are issued on
    // every trip (past the batch end for the last node again, whose header
    // is then unused): a load issued on some paths only would make the
    // compiler wait for all loads in flight where the paths join.
    auto fetch = [&](NodePrep<R, K2>& hn, int nn) {
      if constexpr (PRE)
        prep(hn, nn < nb ? nn : nb - 1);
      else if (nn < nb)
        prep(hn, nn);
    };
    // With WS = 1, 2 the loads are issued two nodes ahead: three
    // headers in turn, so a load has two steps of this group's LDS work to
    // arrive in.
    auto run3 = [&](auto&& step) {
      NodePrep<R, K2> h0, h1, h2;
      int n = ngrp;
      if (n < nb) {
        prep(h0, n);
        fetch(h1, n + NODE_GROUPS);
      }
      while (n < nb) {
        step(h0, h2, n + 2 * NODE_GROUPS);
        n += NODE_GROUPS;
        if (n >= nb) break;
        step(h1, h0, n + 2 * NODE_GROUPS);
        n += NODE_GROUPS;
        if (n >= nb) break;
        step(h2, h1, n + 2 * NODE_GROUPS);
        n += NODE_GROUPS;
      }
    };
    if constexpr (PRIV && D == 2) {
      // two headers in turn, so the next node's window is prepared into the
      // other one and nothing is copied between trips
      auto step = [&](const NodePrep<R, K2>& h, NodePrep<R, K2>& hn, int nn) {
        const Cell2 c = cell_of(h);
        const int col = c.l1 + 1 + k;
        // with WS = 1, 2 the factors are formed here, two steps after their
        // loads were issued, and the column factor multiplied in
        R p0 = h.p0, q1 = h.q1;
        if constexpr (PRE) factors(h, p0, q1);
        const R vx = PRE ? h.cx * q1 : h.vx;
        const R vy = PRE ? h.cy * q1 : h.vy;
        // row factors: lane i of the group holds row i's factor, broadcast
        // here (all 16 lanes of the group are active)
        R rw[K2];
        if constexpr (!(PRE && CS)) {
          static_for<0, K2>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            rw[I] = PRE ? row_bcast<I>(p0) : h.rw[I];
          });
        }
        if constexpr (CS) {
          float* t = ptile + (c.l0 + 1) * P + col;
          float cur[K2];
          if (k < K2) {
#pragma unroll
            for (int i = 0; i < K2; ++i) cur[i] = t[i * P];
          }
          fetch(hn, nn);
          if (k < K2) {
            if constexpr (PRE) {
              // row factor i is lane i's p0, broadcast inside the multiply-add
              fmac_row_bcast<K2>(cur, p0, vx);
            } else {
#pragma unroll
              for (int i = 0; i < K2; ++i) cur[i] += vx * rw[i];
            }
#pragma unroll
            for (int i = 0; i < K2; ++i) t[i * P] = cur[i];
          }
        } else {
          float2* t = acc.tile + (c.l0 + 1) * P + col;
          float2 cur[K2];
          if (k < K2) {
#pragma unroll
            for (int i = 0; i < K2; ++i) cur[i] = t[i * P];
          }
          fetch(hn, nn);
          if (k < K2) {
#pragma unroll
            for (int i = 0; i < K2; ++i) {
              cur[i].x += vx * rw[i];
              cur[i].y += vy * rw[i];
            }
#pragma unroll
            for (int i = 0; i < K2; ++i) t[i * P] = cur[i];
          }
        }
        edges(h, c, vx, vy, col, p0);
      };
      if constexpr (PRE) {
        run3(step);
      } else {
        NodePrep<R, K2> h0, h1;
        int n = ngrp;
        if (n < nb) prep(h0, n);
        while (n < nb) {
          step(h0, h1, n + NODE_GROUPS);
          n += NODE_GROUPS;
          if (n >= nb) break;
          step(h1, h0, n + NODE_GROUPS);
          n += NODE_GROUPS;
        }
      }
    } else if constexpr (PRE) {
      // float64 with WS = 1, 2: the data of the node two ahead is loaded
      // before this node's atomics are issued
      auto step = [&](const NodePrep<R, K2>& h, NodePrep<R, K2>& hn, int nn) {
        fetch(hn, nn);
        const Cell2 c = cell_of(h);
        const int col = c.l1 + 1 + k;
        R p0, q1;
        factors(h, p0, q1);
        const R vx = h.cx * q1;
        const R vy = h.cy * q1;
        R rw[K2];
        static_for<0, K2>([&](auto ic) {
          constexpr int I = decltype(ic)::value;
          rw[I] = row_bcast<I>(p0);
        });
        if (k < K2) {
#pragma unroll
          for (int i = 0; i < K2; ++i) add1((c.l0 + 1 + i) * P + col, vx * rw[i], vy * rw[i]);
        }
        edges(h, c, vx, vy, col, p0);
      };
      run3(step);
    } else {
      // d = 1, and float64 (shared tile, atomics): the next header is
      // prepared into the same registers after this node's updates
      int n = ngrp;
      NodePrep<R, K2> h;
      if (n < nb) prep(h, n);
      for (; n < nb; n += NODE_GROUPS) {
        const int nn = n + NODE_GROUPS;
        if constexpr (D == 1) {
          if (k < K2) add1(h.l0 + 1 + k, h.vx, h.vy);
          if (h.e0 && k == 0) add1(h.l0, h.cx * edge, h.cy * edge);
        } else {
          const int col = h.l1 + 1 + k;
          if (k < K2) {
#pragma unroll
            for (int i = 0; i < K2; ++i) add1((h.l0 + 1 + i) * P + col, h.vx * h.rw[i], h.vy * h.rw[i]);
          }
          edges(h, cell_of(h), h.vx, h.vy, col, h.p0);
        }
        if (nn < nb) prep(h, nn);
      }
    }
    __syncthreads();
  }

  const int slot = a.item_slot[item];
  cplx<R>* out = slot < 0 ? a.tilep + rhs * a.tile_rs + (int64_t)a.item_bin[item] * Ptot
                          : a.itemp + rhs * a.item_rs + (int64_t)slot * Ptot;
  if constexpr (CS) {
    // planes of one component summed in a fixed pairwise order (float64)
    const float* t = reinterpret_cast<const float*>(lds_d);
    for (int i = tid; i < Ptot; i += NT) {
      double sx[NODE_GROUPS], sy[NODE_GROUPS];
#pragma unroll
      for (int g = 0; g < NODE_GROUPS; ++g) {
        sx[g] = t[(size_t)(2 * g) * Ptot + i];
        sy[g] = t[(size_t)(2 * g + 1) * Ptot + i];
      }
#pragma unroll
      for (int w = 1; w < NODE_GROUPS; w *= 2)
#pragma unroll
        for (int g = 0; g + w < NODE_GROUPS; g += 2 * w) {
          sx[g] += sx[g + w];
          sy[g] += sy[g + w];
        }
      out[i] = mkc<R>((R)sx[0], (R)sy[0]);
    }
  } else if constexpr (PRIV) {
    // group tiles summed in a fixed pairwise order (in float64, rounded once)
    const float2* t = reinterpret_cast<const float2*>(lds_d);
    for (int i = tid; i < Ptot; i += NT) {
      double sx[NG], sy[NG];
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const float2 v = t[(size_t)g * Ptot + i];
        sx[g] = v.x;
        sy[g] = v.y;
      }
#pragma unroll
      for (int w = 1; w < NG; w *= 2)
#pragma unroll
        for (int g = 0; g + w < NG; g += 2 * w) {
          sx[g] += sx[g + w];
          sy[g] += sy[g + w];
        }
      out[i] = mkc<R>((R)sx[0], (R)sy[0]);
    }
  } else {
    for (int i = tid; i < Ptot; i += NT) out[i] = mkc<R>((R)acc.re[i], (R)acc.im[i]);
  }
}

// d <= 2 single right-hand side: float32 private group tiles, nt threads
template <typename R, int D, int MW, int NT, bool CS, int WS>
static hipError_t spread_group_nt(const SpreadArgs<R>& a, int nrhs, hipStream_t s) {
  constexpr int NG = NT / 16;
  const size_t acc = CS ? (size_t)NG * a.g.Ptot * 4
                        : std::is_same<R, float>::value ? (size_t)NG * a.g.Ptot * 8
                                                        : (size_t)2 * a.g.Ptot * 8;
  const size_t lds = acc + (size_t)NT * (WS != 0 ? 2 * sizeof(R) : 4 * sizeof(R) + 4);
  const dim3 grid(a.g.nsub, nrhs);
  if constexpr (D == 2) {
    if (a.g.T == 16) {
      hipLaunchKernelGGL((spread_group_kernel<R, D, MW, NT, 16, CS, WS>), grid, dim3(NT), lds, s, a);
      return hipGetLastError();
    }
    if (a.g.T == 8) {
      hipLaunchKernelGGL((spread_group_kernel<R, D, MW, NT, 8, CS, WS>), grid, dim3(NT), lds, s, a);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((spread_group_kernel<R, D, MW, NT, 0, CS, WS>), grid, dim3(NT), lds, s, a);
  return hipGetLastError();
}


}  // namespace nfft
