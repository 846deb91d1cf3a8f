// Back substitution of Section 6, Figure 3 spread over workgroups: for
// k = n..1, x_k = y_k / r_kk, then y_j -= r_jk x_k for j < k (and its
// mirror image, the forward substitution R^H w = g of the adjoint).
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

// True when any limb of v carries the empty marker.
template <class P>
__device__ __forceinline__ bool bs_empty(const typename P::C &v) {
  bool miss = false;
  const double *pv = reinterpret_cast<const double *>(&v);
#pragma unroll
  for (int q = 0; q < 2 * P::L; ++q) miss = miss || __double_as_longlong(pv[q]) == RES_EMPTY;
  return miss;
}

// v when pick, else w, elementwise (selects, no branch).
template <class P>
__device__ __forceinline__ typename P::C bs_pick(bool pick, const typename P::C &v, const typename P::C &w) {
  typename P::C r;
  double *pr = reinterpret_cast<double *>(&r);
  const double *pv = reinterpret_cast<const double *>(&v);
  const double *pw = reinterpret_cast<const double *>(&w);
#pragma unroll
  for (int q = 0; q < 2 * P::L; ++q) pr[q] = pick ? pv[q] : pw[q];
  return r;
}

// The triangular solve across workgroups.  FWD = false: R x = y (back
// substitution, Figure 3: columns descending, rows above the pivot
// updated).  FWD = true: R^H x = y (the adjoint's forward substitution:
// columns ascending, entry (i, c) of R^H is conj(r_ci), rows below the
// pivot updated), with the same operations per row as the one-workgroup
// blocked kernels.
//
// Memory operations in the loops below are unconditional (addresses
// clamped into the arrays, unused values discarded by selects) and the loops
// run whole rings, so that the compiler can count the loads in flight and
// wait only for the one a step consumes.
template <class P, bool FWD>
__global__ __launch_bounds__(BP_ROWS) void trsv_pipe_kernel(int n, const double *R, int ldr, size_t planeR,
                                                            const double *y, size_t planeY, double *x, int *info,
                                                            const int *skip, long long spin_ticks,
                                                            long long *trace, unsigned jitter) {
  if (skip != nullptr && *skip != 0) return;
  using C = typename P::C;
  using Rl = typename P::R;
  constexpr int DIR = FWD ? 1 : -1;  // column order
  const int lane = threadIdx.x;
  const int r0 = blockIdx.x * BP_ROWS;
#ifdef MGS_TRACE
  // diagnostic builds: wall-clock stamps per workgroup (start, phase 1 done,
  // phase 2 done)
  if (trace != nullptr && lane == 0) trace[blockIdx.x * 4] = (long long)wall_clock64();
#else
  (void)trace;
#endif
  const int r1 = r0 + BP_ROWS < n ? r0 + BP_ROWS : n;
  const int i = r0 + lane;
  const bool mine = i < r1;
  const int ic = mine ? i : n - 1;  // clamped row for loads
  C yv = P::load(y + ic, planeY);
  const C dg = P::load(R + (size_t)ic * ldr + ic, planeR);
  Rl inv = P::recip(dg.re);
  if (!mine) {
    yv = P::czero();
    inv = P::rzero();
  }
  if (mine && !P::ok_norm(dg.re) && info != nullptr) info_first_bad(info, i + 1);
  // Entry (row i, column col) of the triangular matrix; col clamped.
  auto rload = [&](int col) __attribute__((always_inline)) {
    const int cl = col < 0 ? 0 : (col >= n ? n - 1 : col);
    if constexpr (FWD)
      return P::conj(P::load(R + (size_t)ic * ldr + cl, planeR));
    else
      return P::load(R + (size_t)cl * ldr + ic, planeR);
  };
  auto xload = [&](int col) __attribute__((always_inline)) {
    bool m = false;
    const int cl = col < 0 ? 0 : (col >= n ? n - 1 : col);
    return res_coh_load<P>(x + cl, (size_t)n, m);
  };
  // The block's own columns in solve order in a ring (slot t: the t-th,
  // (t+8)-th, ... column).
  const int c2 = FWD ? r0 : r1 - 1;
  C rb[BP_RING];
#pragma unroll
  for (int t = 0; t < BP_RING; ++t) rb[t] = rload(c2 + DIR * t);
  // 1. The columns solved before the block (above it for R x = y, left of
  // it for R^H x = y), in solve order, in chunks of CH columns: the entries
  // and x values of the next chunk are loaded while the current one is
  // applied (two buffers, so no register moves between chunks); at the
  // front, where x arrives one entry at a time, each entry is applied as it
  // comes.
  const long long t0 = wall_clock64();
  {
    constexpr int CH = P::L == 4 ? 4 : 8;
    const int ncol = FWD ? r0 : n - r1;  // columns of phase 1
    const int c1 = FWD ? 0 : n - 1;      // the first of them
    C ra0[CH], xa0[CH], ra1[CH], xa1[CH];
    auto fetch = [&](int s0, C (&rr)[CH], C (&xx)[CH]) __attribute__((always_inline)) {
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        rr[u] = rload(c1 + DIR * (s0 + u));
        xx[u] = xload(c1 + DIR * (s0 + u));
      }
    };
    // Applies the chunk starting at step s0, in order, each entry as soon
    // as it (and every earlier one) is out: the entries already applied are
    // kept by the selects, the rest reloaded while waiting.  False on
    // time-out.
    auto consume = [&](int s0, const C (&rr)[CH], C (&xx)[CH]) __attribute__((always_inline)) {
      int done = 0;
      while (true) {
        int avail = 0;
        bool gap = false;
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          const bool here = s0 + u >= ncol || __ballot(bs_empty<P>(xx[u])) == 0;
          gap = gap || !here;
          if (!gap) avail = u + 1;
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          C yn = yv;
          P::upd(yn, rr[u], xx[u]);
          yv = bs_pick<P>(mine && u >= done && u < avail && s0 + u < ncol, yn, yv);
        }
        done = avail;
        if (done == CH) return true;
        if (wall_clock64() - t0 > spin_ticks) {
          if (lane == 0 && info != nullptr)
            __hip_atomic_store(info, MGS_INFO_SYNC_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          return false;
        }
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int u = 0; u < CH; ++u) xx[u] = xload(c1 + DIR * (s0 + u));
      }
    };
    const int nch = (ncol + CH - 1) / CH;
    int s0 = 0;
    fetch(s0, ra0, xa0);
#pragma unroll 1
    for (int k = 0; k < nch; k += 2) {
      res_jitter(jitter, (unsigned)k);
      fetch(s0 + CH, ra1, xa1);
      if (!consume(s0, ra0, xa0)) return;
      s0 += CH;
      if (k + 1 >= nch) break;
      fetch(s0 + CH, ra0, xa0);
      if (!consume(s0, ra1, xa1)) return;
      s0 += CH;
    }
  }
#ifdef MGS_TRACE
  if (trace != nullptr && lane == 0) trace[blockIdx.x * 4 + 1] = (long long)wall_clock64();
#endif
  // 2. The block itself: x_c from its lane, broadcast, applied to the rows
  // it reaches (R from the ring, BP_RING columns ahead).  Each lane keeps
  // its own x (the empty marker until solved) and every step all lanes
  // store theirs, so x_c is out one step after it is formed, with no branch.
  C xown;
  {
    double *po = reinterpret_cast<double *>(&xown);
#pragma unroll
    for (int q = 0; q < 2 * P::L; ++q) po[q] = __longlong_as_double(RES_EMPTY);
  }
  const int rounds2 = (r1 - r0 + BP_RING - 1) / BP_RING;
  int cc = c2;
#pragma unroll 1
  for (int rd = 0; rd < rounds2; ++rd) {
    res_jitter(jitter, 0x10000u + (unsigned)rd);
#pragma unroll
    for (int t = 0; t < BP_RING; ++t) {
      const int k = cc - r0;  // lane of row cc (outside [0, 64) past the block)
      const C xk = bs_readlane<P>(P::scale(yv, inv), k & 63);
      xown = bs_pick<P>(lane == k, xk, xown);
      C yn = yv;
      P::upd(yn, rb[t], xk);
      yv = bs_pick<P>(FWD ? lane > k : lane < k, yn, yv);
      if (mine) res_coh_store<P>(x + i, (size_t)n, xown);
      rb[t] = rload(cc + DIR * BP_RING);
      cc += DIR;
    }
  }
#ifdef MGS_TRACE
  if (trace != nullptr && lane == 0) trace[blockIdx.x * 4 + 2] = (long long)wall_clock64();
#endif
}

}  // namespace mgsq
