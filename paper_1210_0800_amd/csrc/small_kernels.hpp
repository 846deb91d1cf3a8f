// MGS of a small [A b] (dd, m <= 64 rows, at most 64 columns) in one
// workgroup: the operations of Figure 1 (Section 3) on the augmented matrix
// of Equation (1), column j receiving the projections k = 1, ..., j-1 in
// order, then its norm and q_j = a_j / r_jj.
//
// Sixteen waves, one row per lane; column j lives in the registers of wave
// j mod 16.  Inner products and norms are wave sums (DPP scan, total in
// lane 63, broadcast by readlane), with no block barrier.  q_k passes from
// its owner to the other waves through LDS with a per-column flag; the
// owner of column k+1 applies q_k to that column first, normalises and
// publishes it, and only then applies q_k to its later columns, so the
// serial chain is one projection and one normalisation per column.  Every
// wait is bounded by a wall-clock limit (MGS_INFO_SYNC_TIMEOUT in info).
#pragma once
#include "../../include/mgsqr.h"
#include "resident_kernels.hpp"

namespace mgsq {

constexpr int SMALL_WAVES = 16;
constexpr int SMALL_CPW = 4;  // columns per wave
constexpr int SMALL_MAX_ROWS = 64;
constexpr int SMALL_MAX_COLS = SMALL_WAVES * SMALL_CPW;

struct SmallArgs {
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
  long long spin_ticks;  // wall-clock limit of one wait
  unsigned jitter;       // race checks: seed of the timing jitter (0: none)
};

__device__ __forceinline__ PrecDD::Acc small_lane63(const PrecDD::Acc &v) {
  PrecDD::Acc r;
  r.sr = __shfl(v.sr, 63);
  r.cr = __shfl(v.cr, 63);
  r.si = __shfl(v.si, 63);
  r.ci = __shfl(v.ci, 63);
  return r;
}

__global__ __launch_bounds__(64 * SMALL_WAVES) void mgs_small_kernel(SmallArgs a) {
  using P = PrecDD;
  using C = P::C;
  using Acc = P::Acc;
  using Rl = P::R;
  __shared__ double qs[SMALL_MAX_COLS][4][SMALL_MAX_ROWS];  // published q vectors, planar
  __shared__ int flag[SMALL_MAX_COLS];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const bool row = lane < a.m;
  if (tid < SMALL_MAX_COLS) flag[tid] = 0;
  if (tid == 0) *a.info = 0;
  C col[SMALL_CPW];
  static_for<SMALL_CPW>([&](auto sI) __attribute__((always_inline)) {
    constexpr int s = decltype(sI)::value;
    const int j = w + SMALL_WAVES * s;
    col[s] = P::czero();
    if (row && j < a.n)
      col[s] = P::load(a.A + (size_t)j * a.lda + lane, a.planeA);
    else if (row && j == a.n && a.ncols > a.n)
      col[s] = P::load(a.b + lane, (size_t)a.m);
  });
  __syncthreads();

  // r_cc = ||a_c||, q_c = a_c / r_cc in slot s; q_c stored to Q and LDS,
  // R(c, c), then the flag.  Returns q_c in q.
  auto normalise = [&](int c, C &q) __attribute__((always_inline)) {
    static_for<SMALL_CPW>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      if (w + SMALL_WAVES * s == c) {
        Acc t;
        P::acc_zero(t);
        P::acc_abs2(t, col[s]);
        wave_sum_any<PrecDD>(t, true);
        const Rl s2 = P::acc_value_re(small_lane63(t));
        if (!P::ok_norm(s2) && lane == 0) atomicCAS(a.info, 0, c + 1);
        Rl rkk, inv;
        P::sqrt_recip(s2, rkk, inv);
        col[s] = P::scale(col[s], inv);
        q = col[s];
        if (row) {
          P::store(a.Q + (size_t)c * a.ldq + lane, a.planeQ, q);
          qs[c][0][lane] = q.re.h;
          qs[c][1][lane] = q.im.h;
          qs[c][2][lane] = q.re.l;
          qs[c][3][lane] = q.im.l;
        }
        if (lane == 0) {
          C d;
          d.re = rkk;
          d.im = P::rzero();
          P::store(a.R + (size_t)c * a.ldr + c, a.planeR, d);
        }
        lds_wait();
        if (lane == 0) __hip_atomic_store(&flag[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    });
  };
  // r_kj = q_k^H a_j and a_j -= r_kj q_k for slot s (column j).
  auto project = [&](int s_j, int j, int k, const C &q) __attribute__((always_inline)) {
    static_for<SMALL_CPW>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      if (s == s_j) {
        Acc t;
        P::acc_zero(t);
        P::acc_cmulc(t, q, col[s]);
        wave_sum_any<PrecDD>(t, false);
        const C rk = P::acc_value(small_lane63(t));
        if (lane == 0) {
          if (j < a.n)
            P::store(a.R + (size_t)j * a.ldr + k, a.planeR, rk);
          else
            P::store(a.y + k, (size_t)a.n, rk);
        }
        P::upd(col[s], rk, q);
      }
    });
  };

  C q = P::czero();
  if (w == 0 && a.n > 0) normalise(0, q);
  for (int k = 0; k < a.n; ++k) {
    res_jitter(a.jitter, (unsigned)k);
    // this wave's last column; nothing left to do once it is <= k
    const int lastj = w + SMALL_WAVES * ((a.ncols - 1 - w) / SMALL_WAVES);
    if (w >= a.ncols || lastj <= k) break;
    if (k % SMALL_WAVES != w) {
      const long long t0 = wall_clock64();
      while (__hip_atomic_load(&flag[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0) {
        if (wall_clock64() - t0 > a.spin_ticks) {
          if (lane == 0) atomicExch(a.info, MGS_INFO_SYNC_TIMEOUT);
          return;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      q = P::czero();
      if (row) {
        q.re.h = qs[k][0][lane];
        q.im.h = qs[k][1][lane];
        q.re.l = qs[k][2][lane];
        q.im.l = qs[k][3][lane];
      }
    } else {
      static_for<SMALL_CPW>([&](auto sI) __attribute__((always_inline)) {
        constexpr int s = decltype(sI)::value;
        if (w + SMALL_WAVES * s == k) q = col[s];
      });
    }
    // Critical path first: column k+1, if it is this wave's, receives q_k,
    // is normalised and published before the wave's later columns.
    const int c1 = k + 1;
    const bool own_next = c1 < a.n && c1 % SMALL_WAVES == w;
    C qn = P::czero();
    if (own_next) {
      project(c1 / SMALL_WAVES, c1, k, q);
      normalise(c1, qn);
    }
    for (int s = 0; s < SMALL_CPW; ++s) {
      const int j = w + SMALL_WAVES * s;
      if (j > k && j < a.ncols && !(own_next && j == c1)) project(s, j, k, q);
    }
  }
  // rho = ||b - Q y|| (Equation (1)), by the owner of b.
  if (a.rho != nullptr && a.ncols > a.n && a.n % SMALL_WAVES == w) {
    static_for<SMALL_CPW>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      if (w + SMALL_WAVES * s == a.n) {
        Acc t;
        P::acc_zero(t);
        P::acc_abs2(t, col[s]);
        wave_sum_any<PrecDD>(t, true);
        const Rl s2 = P::acc_value_re(small_lane63(t));
        if (lane == 0) P::store_real(a.rho, 1, P::ok_norm(s2) ? P::sqrt_(s2) : P::rzero());
      }
    });
  }
  // Zeros below the diagonal of the owned columns of R.
  for (int s = 0; s < SMALL_CPW; ++s) {
    const int j = w + SMALL_WAVES * s;
    if (j < a.n && lane > j && lane < a.n) P::store(a.R + (size_t)j * a.ldr + lane, a.planeR, P::czero());
  }
}

}  // namespace mgsq
