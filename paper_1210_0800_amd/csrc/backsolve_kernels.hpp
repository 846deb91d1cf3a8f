// Back substitution of Section 6, Figure 3 spread over workgroups: for
// k = n..1, x_k = y_k / r_kk, then y_j -= r_jk x_k for j < k.
//
// Workgroup j is one wave holding rows [64j, 64j + 64) of y, one row per
// lane.  It applies r_ic x_c to its rows for every column c above its
// block as soon as x_c is published, in descending c, then solves its own
// diagonal block: the lane of row c forms x_c (times the reciprocal of
// r_cc, formed up front), every lane gets it by readlane, the owner lane
// publishes it, and the rows above c in the block receive r_ic x_c.  The
// entries of R (and of x above the block) are loaded eight columns ahead,
// so the loads stay off the serial chain.  So
// every y_i receives r_ic x_c in the order c = n, n-1, ..., i+1 with the
// operations of the column-oriented loop, and x is bitwise that of the
// one-workgroup kernel; only the schedule differs: the blocks below are
// already absorbed when a block's turn comes, and x_c reaches the block
// above one entry at a time, so the serial chain is one multiply, one
// broadcast and one update per column plus one hand-off per block.
//
// Publication: x is filled with the empty marker (a signalling NaN, which
// no arithmetic produces) by bs_mark_kernel before the launch; x_c is
// written with device-scope stores and read with device-scope loads until
// no marker is left.  Every wait is bounded by a wall-clock limit
// (MGS_INFO_SYNC_TIMEOUT in info).  The launch is cooperative: every
// workgroup resident.
#pragma once
#include "../../include/mgsqr.h"
#include "resident_kernels.hpp"

namespace mgsq {

constexpr int BP_ROWS = 64;  // rows per workgroup (one wave)
constexpr int BP_RING = 8;   // columns of R (and entries of x) loaded ahead

// x := empty marker (all planes), info := 0; nothing when *skip != 0.
template <int L>
__global__ __launch_bounds__(256) void bs_mark_kernel(int n, double *x, int *info, const int *skip) {
  if (skip != nullptr && *skip != 0) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i == 0 && info != nullptr) *info = 0;
  if (i < n) {
#pragma unroll
    for (int p = 0; p < 2 * L; ++p) x[i + (size_t)p * n] = __longlong_as_double(RES_EMPTY);
  }
}

template <class P>
__device__ __forceinline__ typename P::C bs_coh_load(const double *p, size_t plane, bool &miss) {
  constexpr int NP = 2 * P::L;
  // plane q of the element, gathered in plane order, then read as P::load
  // reads a planar element with plane stride 1
  double t[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    t[q] = coh_load(p + (size_t)q * plane);
    miss = miss || __double_as_longlong(t[q]) == RES_EMPTY;
  }
  return P::load(t, 1);
}
template <class P>
__device__ __forceinline__ void bs_coh_store(double *p, size_t plane, const typename P::C &v) {
  constexpr int NP = 2 * P::L;
  double t[NP];
  P::store(t, 1, v);
#pragma unroll
  for (int q = 0; q < NP; ++q) coh_store(p + (size_t)q * plane, t[q]);
}

template <class P>
__global__ __launch_bounds__(BP_ROWS) void backsolve_pipe_kernel(int n, const double *R, int ldr, size_t planeR,
                                                                 const double *y, size_t planeY, double *x,
                                                                 int *info, const int *skip, long long spin_ticks) {
  if (skip != nullptr && *skip != 0) return;
  using C = typename P::C;
  using Rl = typename P::R;
  const int lane = threadIdx.x;
  const int r0 = blockIdx.x * BP_ROWS;
  const int r1 = r0 + BP_ROWS < n ? r0 + BP_ROWS : n;
  const int i = r0 + lane;
  const bool mine = i < r1;
  C yv = P::czero();
  Rl inv = P::rzero();
  if (mine) {
    yv = P::load(y + i, planeY);
    const C d = P::load(R + (size_t)i * ldr + i, planeR);
    if (!P::ok_norm(d.re) && info != nullptr) info_first_bad(info, i + 1);
    inv = P::recip(d.re);
  }
  // R(i, col) of this lane's row for the columns the lane applies: above the
  // block every row, inside it the rows above col.
  auto rload = [&](int col) __attribute__((always_inline)) {
    const bool use = mine && (col >= r1 || (col >= r0 && i < col));
    return use ? P::load(R + (size_t)col * ldr + i, planeR) : P::czero();
  };
  // Rings of BP_RING columns in flight: slot t serves the columns
  // top - t, top - t - BP_RING, ... (static register indices).
  C rb[BP_RING];  // the block's own columns r1-1, r1-2, ...
#pragma unroll
  for (int t = 0; t < BP_RING; ++t) rb[t] = r1 - 1 - t > r0 ? rload(r1 - 1 - t) : P::czero();
  // 1. Columns above the block, descending, each once x_c is out; R and x
  // loaded BP_RING columns ahead.
  const long long t0 = wall_clock64();
  {
    C ra[BP_RING], xa[BP_RING];
#pragma unroll
    for (int t = 0; t < BP_RING; ++t) {
      const int col = n - 1 - t;
      bool miss = false;
      ra[t] = col >= r1 ? rload(col) : P::czero();
      xa[t] = col >= r1 ? bs_coh_load<P>(x + col, (size_t)n, miss) : P::czero();
    }
    int c = n - 1;
    while (c >= r1) {
#pragma unroll
      for (int t = 0; t < BP_RING; ++t) {
        if (c >= r1) {
          while (true) {  // x_c, unless the early load already saw it
            bool miss = false;
            const double *pv = reinterpret_cast<const double *>(&xa[t]);
#pragma unroll
            for (int q = 0; q < 2 * P::L; ++q) miss = miss || __double_as_longlong(pv[q]) == RES_EMPTY;
            if (__ballot(miss) == 0) break;
            if (wall_clock64() - t0 > spin_ticks) {
              if (lane == 0 && info != nullptr)
                __hip_atomic_store(info, MGS_INFO_SYNC_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              return;
            }
            __builtin_amdgcn_s_sleep(1);
            bool m2 = false;
            xa[t] = bs_coh_load<P>(x + c, (size_t)n, m2);
          }
          if (mine) P::upd(yv, ra[t], xa[t]);
          const int cn = c - BP_RING;
          if (cn >= r1) {
            bool m3 = false;
            ra[t] = rload(cn);
            xa[t] = bs_coh_load<P>(x + cn, (size_t)n, m3);
          }
          --c;
        }
      }
    }
  }
  // 2. The block itself: x_c from its lane, broadcast, published, applied
  // to the rows above it (R from the ring, BP_RING columns ahead).
  int cc = r1 - 1;
  while (cc >= r0) {
#pragma unroll
    for (int t = 0; t < BP_RING; ++t) {
      if (cc >= r0) {
        const C xk = bs_readlane<P>(P::scale(yv, inv), cc - r0);
        if (lane == cc - r0) bs_coh_store<P>(x + cc, (size_t)n, xk);
        if (lane < cc - r0) P::upd(yv, rb[t], xk);
        const int cn = cc - BP_RING;
        if (cn > r0) rb[t] = rload(cn);
        --cc;
      }
    }
  }
}

}  // namespace mgsq
