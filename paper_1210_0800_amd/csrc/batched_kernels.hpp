// Batched least squares: many independent small systems [A_s b_s], one
// workgroup each (the many paths of a homotopy, Section 2; the data stays on
// the card between them, Section 7).
//
// Per system the operations are those of Figure 1 (Section 3) on the
// augmented matrix of Equation (1): column j receives the projections
// k = 1, ..., j-1 in order, then its norm r_jj and q_j = a_j / r_jj; then
// the back substitution of Section 6, Figure 3 on y = the projections of b.
//
// NW waves, one row per lane (m <= 64); column j of [A b] lives in the
// registers of wave j mod NW (slot j / NW).  Inner products and norms are
// wave sums (DPP scan, total read from lane 63), with no block barrier.
// q_k passes from its owner to the other waves through LDS with a
// per-column flag; the owner of column k+1 applies q_k to that column
// first, normalises and publishes it, and only then applies q_k to its
// later columns, so a system's serial chain is one projection and one
// normalisation per column, and the other systems on the compute unit fill
// its waits.  The projections of b (y) go to y (or to x), then the first
// wave writes x = R^{-1} y, column oriented.  Every wait is bounded by a
// wall-clock limit (MGS_INFO_SYNC_TIMEOUT in that system's info).
#pragma once
#include "../../include/mgsqr.h"
#include "resident_kernels.hpp"

namespace mgsq {

constexpr int BAT_MAX_ROWS = 64;
constexpr int BAT_MAX_COLS = 64;          // columns of [A b]
constexpr size_t BAT_LDS_BYTES = 160 * 1024 - 1024;  // q vectors of one system (flags take the rest)

struct BatArgs {
  int batch, m, n, ncols;  // ncols = n + 1 when b is given
  const double *A;         // [batch][L][2][n][lda]
  int lda;
  const double *b;  // [batch][L][2][m] or null
  double *Q;        // [batch][L][2][n][ldq]
  int ldq;
  double *R;  // [batch][L][2][n][ldr]
  int ldr;
  double *y;    // [batch][L][2][n] or null: the projections of b
  double *x;    // [batch][L][2][n] or null: R^{-1} y (b given)
  double *rho;  // [batch][L] or null
  int *info;    // [batch]
  long long spin_ticks;
  unsigned jitter;  // race checks: seed of the timing jitter (0: none)
};

// Lane 63's accumulator, wave-uniform.
template <class P>
__device__ __forceinline__ typename P::Acc acc_lane63(const typename P::Acc &v) {
  using Acc = typename P::Acc;
  constexpr int NA = sizeof(Acc) / sizeof(double);
  Acc r;
  double *pr = reinterpret_cast<double *>(&r);
  const double *pv = reinterpret_cast<const double *>(&v);
#pragma unroll
  for (int c = 0; c < NA; ++c) {
    const long long bits = __double_as_longlong(pv[c]);
    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), 63);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), 63);
    pr[c] = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
  return r;
}

template <class P, int NW, int CPW>
__global__ __launch_bounds__(64 * NW) void mgs_batched_kernel(BatArgs a) {
  using C = typename P::C;
  using Acc = typename P::Acc;
  using Rl = typename P::R;
  constexpr int NP = 2 * P::L;  // planes of a complex element
  extern __shared__ double qs[];  // published q vectors of this system, [column][plane][row]
  __shared__ int flag[BAT_MAX_COLS];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int sys = blockIdx.x;
  const int m = a.m, n = a.n;
  const bool row = lane < m;
  const size_t planeA = (size_t)a.lda * n, planeQ = (size_t)a.ldq * n, planeR = (size_t)a.ldr * n;
  const double *A = a.A + (size_t)sys * NP * planeA;
  double *Q = a.Q + (size_t)sys * NP * planeQ;
  double *R = a.R + (size_t)sys * NP * planeR;
  double *x = a.x != nullptr ? a.x + (size_t)sys * NP * n : nullptr;
  double *y = a.y != nullptr ? a.y + (size_t)sys * NP * n : x;  // y_k lands here
  int *info = a.info + sys;
  if (tid < BAT_MAX_COLS) flag[tid] = 0;
  if (tid == 0) *info = 0;
  C col[CPW];
  static_for<CPW>([&](auto sI) __attribute__((always_inline)) {
    constexpr int s = decltype(sI)::value;
    const int j = w + NW * s;
    col[s] = P::czero();
    if (row && j < n)
      col[s] = P::load(A + (size_t)j * a.lda + lane, planeA);
    else if (row && j == n && a.ncols > n)
      col[s] = P::load(a.b + (size_t)sys * NP * m + lane, (size_t)m);
  });
  __syncthreads();

  // r_cc = ||a_c||, q_c = a_c / r_cc in its slot; q_c to Q and LDS, R(c, c),
  // then the flag.  Returns q_c in q.
  auto normalise = [&](int c, C &q) __attribute__((always_inline)) {
    static_for<CPW>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      if (w + NW * s == c) {
        Acc t;
        P::acc_zero(t);
        P::acc_abs2(t, col[s]);
        wave_sum_any<P>(t, true);
        const Rl s2 = P::acc_value_re(acc_lane63<P>(t));
        if (!P::ok_norm(s2) && lane == 0) atomicCAS(info, 0, c + 1);
        Rl rkk, inv;
        root_and_inverse<P>(s2, rkk, inv);
        col[s] = P::scale(col[s], inv);
        q = col[s];
        if (row) {
          P::store(Q + (size_t)c * a.ldq + lane, planeQ, q);
          P::store(qs + (size_t)c * NP * m + lane, (size_t)m, q);
        }
        if (lane == 0) {
          C d;
          d.re = rkk;
          d.im = P::rzero();
          P::store(R + (size_t)c * a.ldr + c, planeR, d);
        }
        lds_wait();
        if (lane == 0) __hip_atomic_store(&flag[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    });
  };
  // r_kj = q_k^H a_j and a_j -= r_kj q_k for slot s_j (column j); y_k = r_kn
  // goes to y (to x when no y is asked for).
  auto project = [&](int s_j, int j, int k, const C &q) __attribute__((always_inline)) {
    static_for<CPW>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      if (s == s_j) {
        Acc t;
        P::acc_zero(t);
        P::acc_cmulc(t, q, col[s]);
        wave_sum_any<P>(t, false);
        const C rk = P::acc_value(acc_lane63<P>(t));
        if (lane == 0) {
          if (j < n)
            P::store(R + (size_t)j * a.ldr + k, planeR, rk);
          else
            P::store(y + k, (size_t)n, rk);
        }
        P::upd(col[s], rk, q);
      }
    });
  };

  bool alive = true;
  C q = P::czero();
  if (w == 0) normalise(0, q);
  const int lastj = w < a.ncols ? w + NW * ((a.ncols - 1 - w) / NW) : -1;  // this wave's last column
  for (int k = 0; k < n && k < lastj; ++k) {
    res_jitter(a.jitter, (unsigned)k);
    if (k % NW != w) {
      const long long t0 = wall_clock64();
      while (__hip_atomic_load(&flag[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0) {
        if (wall_clock64() - t0 > a.spin_ticks) {
          if (lane == 0) atomicExch(info, MGS_INFO_SYNC_TIMEOUT);
          alive = false;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (!alive) break;
      q = row ? P::load(qs + (size_t)k * NP * m + lane, (size_t)m) : P::czero();
    } else {
      static_for<CPW>([&](auto sI) __attribute__((always_inline)) {
        constexpr int s = decltype(sI)::value;
        if (w + NW * s == k) q = col[s];
      });
    }
    // Critical path first: column k+1, if it is this wave's, receives q_k,
    // is normalised and published before the wave's later columns.
    const int c1 = k + 1;
    const bool own_next = c1 < n && c1 % NW == w;
    C qn = P::czero();
    if (own_next) {
      project(c1 / NW, c1, k, q);
      normalise(c1, qn);
    }
    for (int s = 0; s < CPW; ++s) {
      const int j = w + NW * s;
      if (j > k && j < a.ncols && !(own_next && j == c1)) project(s, j, k, q);
    }
  }
  // rho = ||b - Q y|| (Equation (1)), by the owner of b.
  if (alive && a.rho != nullptr && a.ncols > n && n % NW == w) {
    static_for<CPW>([&](auto sI) __attribute__((always_inline)) {
      constexpr int s = decltype(sI)::value;
      if (w + NW * s == n) {
        Acc t;
        P::acc_zero(t);
        P::acc_abs2(t, col[s]);
        wave_sum_any<P>(t, true);
        const Rl s2 = P::acc_value_re(acc_lane63<P>(t));
        if (lane == 0) P::store_real(a.rho + (size_t)sys * P::L, 1, P::ok_norm(s2) ? P::sqrt_(s2) : P::rzero());
      }
    });
  }
  // Zeros below the diagonal of the owned columns of R.
  for (int s = 0; s < CPW; ++s) {
    const int j = w + NW * s;
    if (j < n && lane > j && lane < n) P::store(R + (size_t)j * a.ldr + lane, planeR, P::czero());
  }
  if (a.ncols == n || x == nullptr) return;
  // Back substitution (Figure 3) by wave 0 once every wave is done: lane j
  // holds y_j; for k = n-1 .. 0, x_k = y_k / r_kk (times the reciprocal),
  // then y_j -= r_jk x_k for j < k (column k of R read coalesced, the next
  // one in flight).  Skipped when the factorisation reported a problem.
  __syncthreads();
  if (w != 0 || __hip_atomic_load(info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0) return;
  C yv = lane < n ? P::load(y + lane, (size_t)n) : P::czero();
  C rc = lane < n ? P::load(R + (size_t)(n - 1) * a.ldr + lane, planeR) : P::czero();
#pragma unroll 1
  for (int k = n - 1; k >= 0; --k) {
    const C rn = (k > 0 && lane < k) ? P::load(R + (size_t)(k - 1) * a.ldr + lane, planeR) : P::czero();
    Rl inv = P::rzero();
    if (lane == k) inv = P::recip(rc.re);
    const C xk = bs_readlane<P>(P::scale(yv, inv), k);
    if (lane == k) P::store(x + k, (size_t)n, xk);
    if (lane < k) P::upd(yv, rc, xk);
    rc = rn;
  }
}

}  // namespace mgsq
