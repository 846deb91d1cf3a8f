// Register-resident MGS: the whole factorisation of [A b] in one persistent
// launch, every column held in registers from its first load to the
// moment its q vector is written.
//
// Operations are those of Figure 1 (Section 3) on the augmented matrix of
// Equation (1): column j receives the projections k = 1, 2, ..., j-1 in
// order, then (j <= n) its norm r_jj and q_j = a_j / r_jj.  Only the
// schedule, the reduction trees and one reassociation (below) are new:
//
//  * Every column is its own panel (bw = 1), owned by one workgroup; the
//    NW waves of a workgroup split the rows (thread t holds rows r*64*NW
//    + t, r < RR, of every column it owns), so inner products and norms
//    are block sums over the workgroup.  Columns are dealt to the G
//    workgroups in a reflected cyclic order counted from the last column
//    (workgroup g gets np-1-g, np-1-(2G-1-g), np-1-(2G+g), ...), so that
//    every workgroup owns about the same triangular amount of work; near
//    the reflection points neighbours trade places so that no workgroup
//    owns two columns close together (res_position).
//  * Bulk projections (apply) sum the inner products of all of a
//    workgroup's columns at once: partials through LDS, one wave per
//    column reduces, a second barrier shares the result.  They read q_k
//    from Q once its owner's counter says it is published (device-scope
//    stores, completed before the counter moves; one counter per wave,
//    since wave w of every workgroup holds the same rows).
//  * The critical path (the chain column k -> column k+1) goes another
//    way.  As soon as column k has received its last projection, its
//    owner copies it, not yet normalised, to U and only then normalises
//    it.  The owners of the next `defer` columns poll U[k] directly (Q and
//    U hold a signalling-NaN pattern until written) and, in one block sum
//    with one barrier (DPP scans per wave, the NW wave totals merged by
//    every thread), get both ||a_k||^2 and a_k^H a_j; from these they form
//    r_kk and q_k exactly as the owner does (same partials, same merge
//    tree, same operations) and r_kj = (a_k^H a_j) / r_kk, equal to
//    q_k^H a_j in exact arithmetic.  Their other columns receive these
//    projections later, from Q, in order.
//  * Consecutive columns sit on the same XCD (workgroup numbering is
//    rotated so that logical workgroups 0..G/8-1 land on one XCD).
//
// The launch is cooperative (every workgroup resident); it starts with a
// grid barrier after Q and U are marked empty, and every wait is bounded by
// a wall-clock limit after which the kernel aborts through a flag that all
// waits observe, so no wave can spin forever.
#pragma once
#include "../../include/mgsqr.h"
#include "mgs_kernels.hpp"

namespace mgsq {

struct ResArgs {
  int m, n, ncols;  // ncols = n + 1 when b is augmented
  const double *A;
  int lda;
  size_t planeA;
  const double *b;
  double *Q;
  int ldq;
  size_t planeQ;
  double *R;
  int ldr;
  size_t planeR;
  double *y;
  double *rho;
  int *info;
  double *U;  // workspace: each column after its last projection, before normalisation (n columns)
  int ldu;
  size_t planeU;
  unsigned int *sync;  // RES_SYNC_WORDS words, zero at launch: per-wave counters and the abort flag
  int bw, np, G;  // bw must be 1: every panel is one column
  int xcd_group;        // logical workgroups per XCD (G / 8), 0 for identity numbering
  unsigned jitter;      // race checks: seed of the timing jitter (0: none)
  int kbase;            // column offset of this matrix in the caller's, for info
  int init_info;        // clear info at the start (else keep an earlier status)
  int defer;            // look-ahead window of the critical-path-first rule (columns, >= 1)
  long long spin_ticks;  // wall-clock limit of one wait
#ifdef MGS_TRACE
  long long *trace;  // diagnostic builds only: RES_TRACE_SLOTS wall-clock stamps per column
#endif
};

// Diagnostic builds (-DMGS_TRACE) stamp the wall clock at the steps of the
// critical chain, per column: 0 poll of the hand-off started, 1 hand-off
// data arrived, 2 last projection applied, 3 column handed on (stores
// issued), 4 column normalised and published, 5 block sums of the last
// projection past their barrier, 6 square root and reciprocal done.
constexpr int RES_TRACE_SLOTS = 16;
#ifdef MGS_TRACE
#define RES_TRACE(col, slot)                                                                   \
  do {                                                                                         \
    if (a.trace != nullptr && threadIdx.x == 0)                                                \
      a.trace[(size_t)(col) * RES_TRACE_SLOTS + (slot)] = (long long)wall_clock64();           \
  } while (0)
// The latest of the workgroup's waves to reach this point.
#define RES_TRACE_LAST(col, slot)                                                                         \
  do {                                                                                                    \
    if (a.trace != nullptr && (threadIdx.x & 63) == 0)                                                    \
      __hip_atomic_fetch_max(a.trace + (size_t)(col) * RES_TRACE_SLOTS + (slot), (long long)wall_clock64(), \
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);                                 \
  } while (0)
#else
#define RES_TRACE(col, slot) \
  do {                       \
  } while (0)
#define RES_TRACE_LAST(col, slot) \
  do {                            \
  } while (0)
#endif

// Sentinel column index of an empty slot.
constexpr int RES_NONE = 1 << 30;

// Position (counted from the last panel) of the i-th panel of workgroup g
// among G: the reflected cyclic order g, 2G-1-g, 2G+g, 4G-1-g, ..., which
// balances the triangular work, except near the reflection points, where
// that order gives a workgroup two panels 2g+1 (odd blocks, g small) or
// 2G-1-2g (even blocks, g near G) apart: there the workgroup trades its
// place in that block with the one 2 RES_SEP away, so that no workgroup
// owns two panels fewer than 2 RES_SEP + 1 apart (its second panel would
// otherwise wait for the projections it deferred to favour the first).  The
// trade moves 2 RES_SEP positions per block: the balance changes by a few
// percent.  Shared by the kernel and the host (same arithmetic).
constexpr int RES_SEP = 25;
__host__ __device__ __forceinline__ int res_position(int i, int g, int G) {
  int gg = g;
  if (G >= 6 * RES_SEP) {
    if (i & 1) {
      if (g < RES_SEP)
        gg = g + 2 * RES_SEP;
      else if (g >= 2 * RES_SEP && g < 3 * RES_SEP)
        gg = g - 2 * RES_SEP;
    } else {
      if (g >= G - RES_SEP)
        gg = g - 2 * RES_SEP;
      else if (g >= G - 3 * RES_SEP && g < G - 2 * RES_SEP)
        gg = g + 2 * RES_SEP;
    }
  }
  return 2 * G * (i / 2) + ((i & 1) ? 2 * G - 1 - gg : gg);
}

// Synchronisation words: wave w's counter at 16 w (w < 16, one 64-byte
// line each), the arrival count of the start barrier and the abort flag in
// the last two words.
constexpr int RES_SYNC_WORDS = 256;
constexpr int RES_GRID = RES_SYNC_WORDS - 2;
constexpr int RES_ABORT = RES_SYNC_WORDS - 1;

// Bit pattern written over every q entry of Q before the factorisation: a
// signalling NaN, which no arithmetic produces, so a reader knows an entry
// of q_k has arrived when it differs from it.
constexpr long long RES_EMPTY = 0x7ff4a5a5a5a5a5a5LL;

// v, or a quiet NaN when v carries the empty marker's bit pattern.
__device__ __forceinline__ double res_unmark(double v) {
  return __double_as_longlong(v) == RES_EMPTY ? __longlong_as_double(0x7ff8000000000000LL) : v;
}

// Widest panel the resident schedule factors.
constexpr int RES_BWMAX = 4;

// Device-scope (coherent across XCDs) relaxed loads and stores of one
// double: the q vectors exchanged between workgroups.
__device__ __forceinline__ void coh_store(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double coh_load(const double *p) {
  return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Waits until every vector memory operation of this wave has completed
// (s_waitcnt vmcnt(0), expcnt and lgkmcnt left alone).  Through the builtin,
// not inline asm, so that the compiler knows the loads before it are done:
// with an opaque wait it treats the columns loaded at the start as still in
// flight and waits again (for every store the wave has issued since) each
// time the main loop touches them.
// The empty asm statements keep the compiler from moving memory accesses
// across it.
__device__ __forceinline__ void wait_vmem() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0x0F70);
  asm volatile("" ::: "memory");
}

// The row index of a Q / U access, opaque to the compiler: keeps it from
// hoisting the 64-bit addresses of every plane and row out of the main
// loop, which would hold dozens of registers for the whole kernel.
__device__ __forceinline__ int row_of(int r, int rwg) {
  int i = r * rwg + (int)threadIdx.x;
  asm volatile("" : "+v"(i));
  return i;
}

// info = the smallest 1-based column with a zero or non-finite norm (the
// owner of a later column can get there first, since it does not wait for
// the earlier column's normalisation); a negative status is kept.
__device__ __forceinline__ void info_first_bad(int *info, int v) {
  int old = __hip_atomic_load(info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while (old == 0 || old > v) {
    const int prev = atomicCAS(info, old, v);
    if (prev == old) break;
    old = prev;
  }
}

// Race checks: with seed != 0, a pause of 0..15 x 64 clocks, the same for
// the whole wave, drawn from (seed, workgroup, wave, step) by an integer
// hash.  Results must not change: every reduction order is fixed, so a
// difference under jitter is a race.  seed 0 (the default) costs one
// scalar compare.
__device__ __forceinline__ void res_jitter(unsigned seed, unsigned step) {
  if (seed == 0) return;
  unsigned h = seed * 0x9E3779B1u ^ blockIdx.x * 0x85EBCA77u ^ (threadIdx.x >> 6) * 0xC2B2AE3Du ^ step * 0x27D4EB2Fu;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  const int n = __builtin_amdgcn_readfirstlane((int)(h & 15u));
  for (int i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(1);
}

// Common end of a bounded wait: true (and the abort flag set, info
// written) once the wall-clock limit has passed, or when another wave has
// aborted.
__device__ __forceinline__ bool res_give_up(const ResArgs &a, long long t0) {
  if (__builtin_amdgcn_readfirstlane(
          (int)__hip_atomic_load(a.sync + RES_ABORT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0)
    return true;
  if (wall_clock64() - t0 > a.spin_ticks) {
    __hip_atomic_store(a.sync + RES_ABORT, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(a.info, MGS_INFO_SYNC_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
  }
  return false;
}

// Waits until wave `wave` of the owners has published at least k+1
// columns.  `seen` caches the last observed count (wave-uniform).
// Returns false on abort or time-out.
__device__ __forceinline__ bool res_wait(const ResArgs &a, int k, int wave, int &seen) {
  if (seen > k) return true;
  const long long t0 = wall_clock64();
  unsigned int *cnt = a.sync + 16 * wave;
  while (true) {
    const int v = __builtin_amdgcn_readfirstlane(
        (int)__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (v > k) {
      seen = v;
      asm volatile("" ::: "memory");
      return true;
    }
    if (res_give_up(a, t0)) return false;
    __builtin_amdgcn_s_sleep(1);
  }
}

// Wave reduction by DPP: an inclusive scan inside each row of 16 lanes
// (shifts 1, 2, 4, 8), then the row totals carried across rows; lane 63
// ends with the sum of all 64 lanes (a fixed merge tree, so results are
// reproducible).  Lanes shifted in from outside a row read zero, which
// the accumulator merge adds exactly.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_shift(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// One DPP step of a wave sum for any accumulator: every double of the
// accumulator (the real half only when re_only) moves by CTRL, then the
// merge.  Lanes shifted in from outside a row read zero.
template <class P, int CTRL, int ROWS>
__device__ __forceinline__ void dpp_step_any(typename P::Acc &a, bool re_only) {
  using Acc = typename P::Acc;
  constexpr int NA = sizeof(Acc) / sizeof(double);
  Acc o;
  double *po = reinterpret_cast<double *>(&o);
  const double *pa = reinterpret_cast<const double *>(&a);
#pragma unroll
  for (int c = 0; c < NA; ++c) po[c] = (re_only && c >= NA / 2) ? 0.0 : dpp_shift<CTRL, ROWS>(pa[c]);
  if (re_only)
    P::acc_merge_re(a, o);
  else
    P::acc_merge(a, o);
}
// Wave sum into lane 63 (fixed tree: row scans, then the row totals).
template <class P>
__device__ __forceinline__ void wave_sum_any(typename P::Acc &a, bool re_only) {
  dpp_step_any<P, 0x111, 0xf>(a, re_only);  // row_shr:1
  dpp_step_any<P, 0x112, 0xf>(a, re_only);  // row_shr:2
  dpp_step_any<P, 0x114, 0xf>(a, re_only);  // row_shr:4
  dpp_step_any<P, 0x118, 0xf>(a, re_only);  // row_shr:8
  dpp_step_any<P, 0x142, 0xa>(a, re_only);  // row_bcast:15 into rows 1, 3
  dpp_step_any<P, 0x143, 0xc>(a, re_only);  // row_bcast:31 into rows 2, 3
}

// One complex element of a planar array (2L planes, stride `plane`) with
// device-scope loads / stores, plane by plane; `miss` is set when a plane
// holds the empty marker.
template <class P>
__device__ __forceinline__ typename P::C res_coh_load(const double *p, size_t plane, bool &miss) {
  constexpr int NP = 2 * P::L;
  double t[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    t[q] = coh_load(p + (size_t)q * plane);
    miss = miss || __double_as_longlong(t[q]) == RES_EMPTY;
  }
  return P::load(t, 1);
}
template <class P>
__device__ __forceinline__ void res_coh_store(double *p, size_t plane, const typename P::C &v, bool unmark = false) {
  constexpr int NP = 2 * P::L;
  double t[NP];
  P::store(t, 1, v);
#pragma unroll
  for (int q = 0; q < NP; ++q) coh_store(p + (size_t)q * plane, unmark ? res_unmark(t[q]) : t[q]);
}

template <class P, int RR, int CB, int NW>
struct Resident {
  using C = typename P::C;
  using Acc = typename P::Acc;
  using Rl = typename P::R;
  static constexpr int RWG = 64 * NW;  // threads per workgroup

  const ResArgs &a;
  int tid, wave, lane;
  int cidx[CB];  // column of each slot, ascending; RES_NONE when empty
  C col[CB][RR];
  static constexpr int NA = sizeof(Acc) / sizeof(double);  // doubles per accumulator
  double (*red)[NA][RWG];  // LDS: per-thread partial sums, [CB][NA][RWG]
  Acc *rsum;               // LDS: reduced sums, [CB]
  double (*xch)[RES_BWMAX][NA][NW];  // LDS: wave totals of the panel steps, [2][RES_BWMAX][NA][NW]
  int xb = 0;              // xch buffer of the next panel-step reduction

  __device__ __forceinline__ Resident(const ResArgs &args, double (*r)[NA][RWG], Acc *rs,
                                      double (*x)[RES_BWMAX][NA][NW])
      : a(args), red(r), rsum(rs), xch(x) {
    tid = threadIdx.x;
    wave = tid >> 6;
    lane = tid & 63;
  }

  // Block reductions: every thread stores its partial sum of slot s, then
  // (after a barrier) wave s mod NW alone reduces it: lane l merges the partials
  // of threads l, l+64, ..., l+64(NW-1) in a pairwise tree, then a DPP scan
  // brings the total to lane 63, which writes rsum[s].  A second barrier
  // makes rsum visible.  The merge tree is fixed, so results are
  // reproducible, and each partial is merged once (not once per wave).
  __device__ __forceinline__ void put(int s, const Acc &v) {
    const double *d = reinterpret_cast<const double *>(&v);
#pragma unroll
    for (int c = 0; c < NA; ++c) red[s][c][tid] = d[c];
  }
  // Partials of threads lane + 64 w, w in [W0, W0 + CNT), merged in a
  // fixed pairwise tree.
  template <int W0, int CNT>
  __device__ __forceinline__ Acc red_tree(int s, bool re_only) const {
    if constexpr (CNT == 1) {
      Acc u;
      double *du = reinterpret_cast<double *>(&u);
#pragma unroll
      for (int c = 0; c < NA; ++c) du[c] = red[s][c][lane + 64 * W0];
      return u;
    } else {
      Acc x = red_tree<W0, CNT / 2>(s, re_only);
      const Acc y = red_tree<W0 + CNT / 2, CNT / 2>(s, re_only);
      if (re_only)
        P::acc_merge_re(x, y);
      else
        P::acc_merge(x, y);
      return x;
    }
  }
  __device__ __forceinline__ void reduce_slot(int s, bool re_only) {
    Acc t = red_tree<0, NW>(s, re_only);
    wave_sum_any<P>(t, re_only);
    if (lane == 63) rsum[s] = t;
  }

  // r_kj for the slots s whose column lies in (k, hi) and >= lo: the inner
  // products of q with those columns, one block reduction, the R / y
  // stores and the updates a_j -= r_kj q.
  __device__ __forceinline__ void apply(const C (&q)[RR], int k, int lo, int hi) {
    static_for<CB>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      const int j = cidx[s];
      if (j > k && j >= lo && j < hi) {
        Acc acc;
        P::acc_zero(acc);
#pragma unroll
        for (int r = 0; r < RR; ++r) P::acc_cmulc(acc, q[r], col[s][r]);
        put(s, acc);
      }
    });
    lds_barrier();
    static_for<CB>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      const int j = cidx[s];
      if (j > k && j >= lo && j < hi && wave == s % NW) reduce_slot(s, false);
    });
    lds_barrier();
    static_for<CB>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      const int j = cidx[s];
      if (j > k && j >= lo && j < hi) {
        const C rk = P::acc_value(rsum[s]);
        if (tid == 0) {
          if (j < a.n)
            P::store(a.R + (size_t)j * a.ldr + k, a.planeR, rk);
          else
            P::store(a.y + k, (size_t)a.n, rk);
        }
#pragma unroll
        for (int r = 0; r < RR; ++r) P::upd(col[s][r], rk, q[r]);
      }
    });
  }

  // Block sums on the critical path (the steps that factor a panel), with a
  // single barrier: each wave scans its own partial (DPP), lane 63 stores
  // the wave total, and after the barrier every wave merges the NW wave
  // totals in the same fixed pairwise tree (xch_sum), so all threads hold
  // the same sum.  Two buffers alternate: a wave can only overwrite one
  // after every wave has passed the next barrier, i.e. finished reading it.
  __device__ __forceinline__ void xch_put(int pos, Acc t, bool re_only) {
    wave_sum_any<P>(t, re_only);
    if (lane == 63) {
      const double *d = reinterpret_cast<const double *>(&t);
#pragma unroll
      for (int c = 0; c < NA; ++c) xch[xb][pos][c][wave] = d[c];
    }
  }
  // The merge of the NW wave totals, spread over the lanes: lane l starts
  // from the total of wave l mod NW and log2(NW) butterfly steps merge it
  // with the lane l^1, l^2, l^4 (DPP inside rows of 16 lanes, where the
  // totals repeat with period NW, so that a rotation by 4 reaches the l^4
  // partner's value).  The accumulator merge gives the same bits in either
  // operand order (TwoSum's error term is exact), so every lane ends with
  // the pairwise tree ((w0 w1)(w2 w3))((w4 w5)(w6 w7)), in 3 merges per
  // lane instead of 7 one after another.
  __device__ __forceinline__ Acc xch_sum(int pos, bool re_only) const {
    static_assert(NW == 1 || NW == 2 || NW == 4 || NW == 8, "butterfly over at most 8 waves");
    Acc x;
    double *dx = reinterpret_cast<double *>(&x);
#pragma unroll
    for (int c = 0; c < NA; ++c) dx[c] = xch[xb][pos][c][lane & (NW - 1)];
    if constexpr (NW >= 2) dpp_step_any<P, 0xB1, 0xf>(x, re_only);   // quad_perm [1,0,3,2]: lane l^1
    if constexpr (NW >= 4) dpp_step_any<P, 0x4E, 0xf>(x, re_only);   // quad_perm [2,3,0,1]: lane l^2
    if constexpr (NW >= 8) dpp_step_any<P, 0x124, 0xf>(x, re_only);  // row_ror:4: lane l+-4 within the row
    return x;
  }

  // Publication of q_k: this wave's device-scope stores of its rows are
  // complete before its counter moves to k + 1.  The counter only grows
  // (atomic max): the owners of later columns do not wait for it (they
  // read the unnormalised columns from U), so their stores can land first.
  __device__ __forceinline__ void publish(int k) {
    wait_vmem();
    if (lane == 0)
      __hip_atomic_fetch_max(a.sync + 16 * wave, (unsigned int)(k + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }

  // This thread's rows of the owned column x, with device-scope stores,
  // into U (the hand-off to the owners of the next `defer` columns).
  // Column 0 receives no projection, so its entries are the raw input: an
  // entry with the bit pattern of the empty marker is stored as a quiet
  // NaN instead (every other column has passed through arithmetic, which
  // never yields a signalling NaN), so that readers never wait on it.
  __device__ __forceinline__ void store_u(int x) {
    double *dst = a.U + (size_t)x * a.ldu;
    const bool raw = x == 0;
    static_for<CB>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      if (cidx[s] == x) {
#pragma unroll
        for (int r = 0; r < RR; ++r) {
          const int i = row_of(r, RWG);
          if (i < a.m) {
            res_coh_store<P>(dst + i, a.planeU, col[s][r], raw);
          }
        }
      }
    });
  }

  // Normalisation of the owned column x, which has received all its
  // projections: s2 = ||a_x||^2 (one barrier), r_xx and 1/r_xx, q_x = a_x /
  // r_xx in the slot and in q, the stores of q_x and R(x, x), and the
  // publication of q_x.
  __device__ __forceinline__ void own_norm(int x, C (&q)[RR]) {
    Acc nacc;
    P::acc_zero(nacc);
    static_for<CB>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      if (cidx[s] == x) {
#pragma unroll
        for (int r = 0; r < RR; ++r) P::acc_abs2(nacc, col[s][r]);
      }
    });
    xch_put(0, nacc, true);
    lds_barrier();
    const Rl s2 = P::acc_value_re(xch_sum(0, true));
    xb ^= 1;
    if (!P::ok_norm(s2) && tid == 0) info_first_bad(a.info, a.kbase + x + 1);
    Rl rkk, inv;
    root_and_inverse<P>(s2, rkk, inv);
    static_for<CB>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      if (cidx[s] == x) {
#pragma unroll
        for (int r = 0; r < RR; ++r) {
          col[s][r] = P::scale(col[s][r], inv);
          q[r] = col[s][r];
        }
      }
    });
    double *dst = a.Q + (size_t)x * a.ldq;
#pragma unroll
    for (int r = 0; r < RR; ++r) {
      const int i = row_of(r, RWG);
      if (i < a.m) res_coh_store<P>(dst + i, a.planeQ, q[r]);
    }
    if (tid == 0) {
      C d;
      d.re = rkk;
      d.im = P::rzero();
      P::store(a.R + (size_t)x * a.ldr + x, a.planeR, d);
    }
    publish(x);
  }

  // Critical-path projection of column k onto the owned column ps (k >=
  // ps - defer), from u = a_k after its last projection, read from U (in
  // u's registers, which hold q_k on return).  One block sum gives both
  // ||u||^2 and u^H a_ps; then r_kk and 1/r_kk exactly as the owner of
  // column k computes them (same partials, same merge tree, same
  // operations), q_k = u / r_kk, r_{k,ps} = (u^H a_ps) / r_kk (equal to
  // q_k^H a_ps up to rounding) and a_ps -= r_{k,ps} q_k.  After the last
  // projection (k = ps - 1) column ps is final and is handed on through U
  // before anything else.
  __device__ __forceinline__ void lookahead_step(C (&u)[RR], int k, int ps, bool last) {
    {
      Acc an;
      P::acc_zero(an);
#pragma unroll
      for (int r = 0; r < RR; ++r) P::acc_abs2(an, u[r]);
      xch_put(1, an, true);
    }
    static_for<CB>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      if (cidx[s] == ps) {
        Acc ad;
        P::acc_zero(ad);
#pragma unroll
        for (int r = 0; r < RR; ++r) P::acc_cmulc(ad, u[r], col[s][r]);
        xch_put(0, ad, false);
      }
    });
    if (last) RES_TRACE_LAST(ps, 8);
    lds_barrier();
    if (last) RES_TRACE(ps, 5);
    const Rl s2 = P::acc_value_re(xch_sum(1, true));
    const C d = P::acc_value(xch_sum(0, false));
    xb ^= 1;
    Rl rkk, inv;
    root_and_inverse<P>(s2, rkk, inv);
    if (last) RES_TRACE(ps, 6);
#pragma unroll
    for (int r = 0; r < RR; ++r) u[r] = P::scale(u[r], inv);
    const C rk = P::scale(d, inv);
    static_for<CB>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      if (cidx[s] == ps) {
#pragma unroll
        for (int r = 0; r < RR; ++r) P::upd(col[s][r], rk, u[r]);
      }
    });
    if (last) {
      RES_TRACE(ps, 2);
      RES_TRACE_LAST(ps, 9);
      store_u(ps);
      RES_TRACE(ps, 3);
      RES_TRACE_LAST(ps, 10);
    }
    // R(k, ps) last: stores count towards the same wait counter as loads,
    // so a store issued before the hand-off would hold wave 0's rows of U
    // back until it completes.
    if (tid == 0) P::store(a.R + (size_t)ps * a.ldr + k, a.planeR, rk);
  }

  __device__ __forceinline__ void copy_own(int k, C (&q)[RR]) {
    static_for<CB>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      if (cidx[s] == k) {
#pragma unroll
        for (int r = 0; r < RR; ++r) q[r] = col[s][r];
      }
    });
  }
  // Reads this thread's rows of column k of Q or U, again until none of
  // this wave's entries is still RES_EMPTY (so it also serves as the wait
  // of the critical-path steps, which poll U instead of a counter).
  // Returns false on abort or time-out.
  __device__ __forceinline__ bool load_col(const double *base, size_t ld, size_t plane, int k, C (&q)[RR]) {
    const double *src = base + (size_t)k * ld;
    long long t0 = -1;
    while (true) {
      bool miss = false;
#pragma unroll
      for (int r = 0; r < RR; ++r) {
        const int i = row_of(r, RWG);
        q[r] = P::czero();
        if (i < a.m) q[r] = res_coh_load<P>(src + i, plane, miss);
      }
      if (__ballot(miss) == 0) return true;
      if (t0 < 0) t0 = wall_clock64();
      if (res_give_up(a, t0)) return false;
      __builtin_amdgcn_s_sleep(1);
    }
  }
  // Start of the factorisation: RES_EMPTY over the owned columns of Q and
  // U (after they have been read: Q may be A), then a grid barrier, so that
  // no entry of Q or U is read before it is either empty or final.
  __device__ __forceinline__ bool mark_empty() {
    wait_vmem();  // the columns are in registers
    static_for<CB>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      const int j = cidx[s];
      if (j < a.n) {
        double *dst = a.Q + (size_t)j * a.ldq;
        double *dsu = a.U + (size_t)j * a.ldu;
        const double e = __longlong_as_double(RES_EMPTY);
#pragma unroll
        for (int r = 0; r < RR; ++r) {
          const int i = r * RWG + tid;
          if (i < a.m) {
#pragma unroll
            for (int pl = 0; pl < 2 * P::L; ++pl) {
              coh_store(dst + i + pl * a.planeQ, e);
              coh_store(dsu + i + pl * a.planeU, e);
            }
          }
        }
      }
    });
    wait_vmem();
    __syncthreads();
    bool ok = true;
    if (tid == 0) {
      __hip_atomic_fetch_add(a.sync + RES_GRID, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const long long t0 = wall_clock64();
      while (__hip_atomic_load(a.sync + RES_GRID, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned int)a.G) {
        if (res_give_up(a, t0)) {
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __shared__ int grid_ok;
    if (tid == 0) grid_ok = ok ? 1 : 0;
    __syncthreads();
    return grid_ok != 0;
  }
  // Panel `i` of the owned list in ascending column order: [ps, pe).
  __device__ __forceinline__ void panel(int i, int nq, int g, int &ps, int &pe) const {
    if (i >= nq) {
      ps = pe = RES_NONE;
      return;
    }
    const int u = nq - 1 - i;
    const int qi = res_position(u, g, a.G);
    ps = (a.np - 1 - qi) * a.bw;
    pe = ps + a.bw < a.ncols ? ps + a.bw : a.ncols;
  }

  // The whole schedule of one workgroup as a sequence of steps, each either
  // a normalisation or one projection applied to a range of owned columns,
  // so that the loop body holds a single copy of each (a small code
  // footprint for the instruction cache).
  __device__ void run() {
    const int bid = blockIdx.x;
    const int G = a.G;
    const int g = a.xcd_group ? (bid % 8) * a.xcd_group + bid / 8 : bid;
    // Owned panels: the i-th is q_i = res_position(i, g, G) (reflected
    // order), panel np-1-q_i; ascending columns = descending i.
    int nq = 0;
    while (true) {
      const int qi = res_position(nq, g, G);
      if (qi >= a.np) break;
      ++nq;
    }
    static_for<CB>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      const int jp = s / a.bw, c = s - jp * a.bw;
      int ps, pe;
      panel(jp, nq, g, ps, pe);
      cidx[s] = (ps != RES_NONE && ps + c < pe) ? ps + c : RES_NONE;
    });
    static_for<CB>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      const int j = cidx[s];
      const double *src = nullptr;
      size_t pl = 0;
      if (j < a.n) {
        src = a.A + (size_t)j * a.lda;
        pl = a.planeA;
      } else if (j == a.n) {
        src = a.b;
        pl = (size_t)a.m;
      }
#pragma unroll
      for (int r = 0; r < RR; ++r) {
        const int i = r * RWG + tid;
        col[s][r] = (src != nullptr && i < a.m) ? P::load(src + i, pl) : P::czero();
      }
    });
    int last = -1;
    static_for<CB>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      if (cidx[s] != RES_NONE && cidx[s] > last) last = cidx[s];
    });
    if (!mark_empty()) return;
    if (last < 0) return;
    const int kend = last < a.n ? last + 1 : a.n;

    // States: 0 = projections from other workgroups, 1 = normalising an
    // owned column, 2 = deferred projections (q_kd .. q_{ps-1} from Q, then
    // the column's own q) onto the later owned columns.
    int st = 0, seen = 0, nxt = 0, k = 0;
    int ps = 0, pe = 0, kd = -1, dc = 0;
    int qk = -1;       // q currently holds q_qk (this thread's rows)
    int handed = -1;   // last owned column already copied to U
    C q[RR];
    // Each pass performs one bulk projection (apply), one look-ahead
    // projection or one normalisation; each has a single call site so that
    // the loop body holds one copy of it.
    unsigned pass = 0;
    while (true) {
      res_jitter(a.jitter, pass++);
      int mode = 0;  // 1 apply, 2 lookahead_step, 3 own_norm
      int opk = -1, lo = 0;
      int qsrc = 3;  // q_opk: 0 wait and load from Q, 1 owned column, 2 load from Q (already seen), 3 none, 4 poll U
      if (st == 0) {
        if (k >= kend) break;
        panel(nxt, nq, g, ps, pe);
        if (k == ps) {
          st = 1;
          continue;
        }
        opk = k;
        if (ps < a.n && k + a.defer >= ps) {
          // Critical path first: the next owned column only.
          if (kd < 0) kd = k;
          mode = 2;
          qsrc = 4;
        } else {
          mode = 1;
          qsrc = 0;
          lo = k + 1;
        }
      } else if (st == 1) {
        mode = 3;
        opk = ps;
      } else {
        mode = 1;
        opk = dc;
        qsrc = dc < ps ? 2 : 1;
        lo = pe;
      }

      if (qsrc == 0) {
        if (!res_wait(a, opk, wave, seen)) return;
        if (!load_col(a.Q, a.ldq, a.planeQ, opk, q)) return;
      } else if (qsrc == 1) {
        if (qk != opk) copy_own(opk, q);
      } else if (qsrc == 2) {
        if (!load_col(a.Q, a.ldq, a.planeQ, opk, q)) return;  // already published
      } else if (qsrc == 4) {
        if (opk + 1 == ps) RES_TRACE(ps, 0);
        if (!load_col(a.U, a.ldu, a.planeU, opk, q)) return;
        if (opk + 1 == ps) {
          RES_TRACE(ps, 1);
          RES_TRACE_LAST(ps, 7);
        }
      }
      if (mode == 1) {
        apply(q, opk, lo, RES_NONE);
      } else if (mode == 2) {
        lookahead_step(q, opk, ps, opk + 1 == ps);
        if (opk + 1 == ps) handed = ps;
      } else if (mode == 3) {
        // U[ps] is due unless the last projection was a look-ahead step
        // (not so for column 0, or when q_{ps-1} is this workgroup's own
        // and reached column ps as a deferred projection).
        if (handed != ps) {
          store_u(ps);
          RES_TRACE(ps, 3);
        }
        own_norm(ps, q);
        RES_TRACE(ps, 4);
      }
      qk = opk;

      if (st == 0) {
        ++k;
        if (k == ps && ps < a.n) st = 1;
      } else if (st == 1) {
        if (last >= pe) {
          st = 2;
          dc = kd >= 0 ? kd : ps;
        } else {
          st = 0;
          k = pe;
          ++nxt;
          kd = -1;
        }
      } else {
        ++dc;
        if (dc >= pe) {
          st = 0;
          k = pe;
          ++nxt;
          kd = -1;
        }
      }
    }

    // rho = ||b - Q y|| after the last projection (Equation (1)).
    if (a.rho != nullptr && last == a.n) {
      copy_own(a.n, q);
      Acc nacc;
      P::acc_zero(nacc);
#pragma unroll
      for (int r = 0; r < RR; ++r) P::acc_abs2(nacc, q[r]);
      put(0, nacc);
      lds_barrier();
      if (wave == 0) reduce_slot(0, true);
      lds_barrier();
      const Acc t = rsum[0];
      if (tid == 0) {
        const Rl s2 = P::acc_value_re(t);
        P::store_real(a.rho, 1, P::ok_norm(s2) ? P::sqrt_(s2) : P::rzero());
      }
    }
    // Zeros below the diagonal of the owned columns of R.
    static_for<CB>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      const int j = cidx[s];
      if (j < a.n) {
        for (int i = j + 1 + tid; i < a.n; i += RWG) P::store(a.R + (size_t)j * a.ldr + i, a.planeR, P::czero());
      }
    });
  }
};

template <class P, int RR, int CB, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW < 4 ? 1 : NW / 4, NW < 4 ? 1 : NW / 4))) void mgs_resident_kernel(
    ResArgs a) {
  using Acc = typename P::Acc;
  constexpr int NA = sizeof(Acc) / sizeof(double);
  __shared__ double red[CB][NA][64 * NW];
  __shared__ Acc rsum[CB];
  __shared__ double xch[2][RES_BWMAX][NA][NW];
  Resident<P, RR, CB, NW> st(a, red, rsum, xch);
  st.run();
}

// Clears the publication counters, the abort flag and (optionally) info
// (one workgroup of RES_SYNC_WORDS threads).
__global__ void resident_init_kernel(unsigned int *sync, int *info, int init_info) {
  if (threadIdx.x < RES_SYNC_WORDS) sync[threadIdx.x] = 0u;
  if (threadIdx.x == 0 && init_info) *info = 0;
}

}  // namespace mgsq
