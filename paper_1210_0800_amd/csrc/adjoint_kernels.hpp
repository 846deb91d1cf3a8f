// Adjoint of the least-squares solution x = argmin ||b - A x|| for a loss
// L(x) with gradient g = dL/dRe(x) + i dL/dIm(x):
//   w  = R^{-H} g      (forward substitution)
//   z  = R^{-1} w      (back substitution of Section 6, Figure 3)
//   gb = Q w           (= A z, the gradient with respect to b)
//   r  = b - A x
//   gA = r z^H - gb x^H
// with z = (A^H A)^{-1} g for A = Q R of full column rank.
#pragma once
#include "mgs_kernels.hpp"

namespace mgsq {

// w = R^{-H} g, column oriented: for k = 0..n-1, w_k = g_k / r_kk, then
// g_j -= conj(r_kj) w_k for j > k (the lower-triangular counterpart of the
// back substitution of Figure 3).  Blocked like backsolve_blocked_kernel,
// from the top: one workgroup of BS_T threads, thread t holding g_j for
// j = s*BS_T + t; for each block [k0, k0 + B) of columns
//   1. its upper triangle of R is staged in LDS;
//   2. the wave holding rows k0 .. k0+B-1 solves it: w_k = g_k / r_kk
//      (owner lane), broadcast by readlane, g_j -= conj(r_kj) w_k for the
//      block rows j > k;
//   3. every thread with j >= k0 + B applies g_j -= conj(r_kj) w_k for the
//      block's k in ascending order (its R entries are consecutive in
//      memory, read BQ at a time).
// Each g_j receives conj(r_kj) w_k in the order k = 0, 1, ..., j-1 with the
// operations of the column-oriented loop, so w is bitwise that loop's.
template <class P, int NY>
__global__ __launch_bounds__(BS_T) void fwdsub_blocked_kernel(int n, const double *R, int ldr, size_t planeR,
                                                              const double *g, double *w, int *info) {
  using C = typename P::C;
  using Rl = typename P::R;
  constexpr int NP = 2 * P::L;
  constexpr int BS_B = bs_block(P::L);
  __shared__ double rb[NP * BS_B * BS_B];  // block of R, planar [p][col][row]
  __shared__ double xs[NP * BS_B];         // w of the block, planar [p][k]
  __shared__ int bad;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (tid == 0) bad = 0x7fffffff;
  __syncthreads();
  C gv[NY];
  Rl inv[NY];
#pragma unroll
  for (int s = 0; s < NY; ++s) {
    const int j = s * BS_T + tid;
    if (j < n) {
      gv[s] = P::load(g + j, (size_t)n);
      const C d = P::load(R + (size_t)j * ldr + j, planeR);
      if (!P::ok_norm(d.re)) atomicMin(&bad, j + 1);
      inv[s] = P::recip(d.re);
    } else {
      gv[s] = P::czero();
      inv[s] = P::rzero();
    }
  }
  __syncthreads();
  if (tid == 0 && info != nullptr) *info = (bad == 0x7fffffff) ? 0 : bad;
  const int nblk = (n + BS_B - 1) / BS_B;
#pragma unroll 1
  for (int kb = 0; kb < nblk; ++kb) {
    const int k0 = kb * BS_B;
    const int k1 = k0 + BS_B < n ? k0 + BS_B : n;
    const int nb = k1 - k0;
    // 1. R(k0 + r, k0 + c) for r <= c < nb into LDS.
    for (int e = tid; e < BS_B * BS_B; e += BS_T) {
      const int c = e / BS_B, r = e - c * BS_B;
      if (c < nb && r <= c) {
        const C v = P::load(R + (size_t)(k0 + c) * ldr + (k0 + r), planeR);
        P::store(rb + c * BS_B + r, (size_t)BS_B * BS_B, v);
      }
    }
    __syncthreads();
    // 2. The wave holding rows k0 .. k1-1 (one slot s, consecutive lanes).
    const int sk = k0 / BS_T, tk = k0 - sk * BS_T;
    if (wave == tk / 64) {
      const int l0 = tk % 64;
#pragma unroll
      for (int s = 0; s < NY; ++s) {
        if (s == sk) {
          const int i = lane - l0;  // block row of this lane
#pragma unroll 1
          for (int c = 0; c < nb; ++c) {
            const C xl = P::scale(gv[s], inv[s]);
            const C xk = bs_readlane<P>(xl, l0 + c);
            if (i == c) {
              P::store(w + k0 + c, (size_t)n, xk);
              P::store(xs + c, (size_t)BS_B, xk);
            }
            if (i > c && i < nb) P::upd(gv[s], P::conj(P::load(rb + i * BS_B + c, (size_t)BS_B * BS_B)), xk);
          }
        }
      }
    }
    __syncthreads();
    // 3. Rows below the block.
#pragma unroll
    for (int s = 0; s < NY; ++s) {
      const int j = s * BS_T + tid;
      if (j >= k1 && j < n) {
        constexpr int BQ = (P::L == 4 ? 2 : 8) / NY > 0 ? (P::L == 4 ? 2 : 8) / NY : 1;
        const double *rj = R + (size_t)j * ldr + k0;
#pragma unroll 1
        for (int c0 = 0; c0 < nb; c0 += BQ) {
          C rv[BQ];
#pragma unroll
          for (int t = 0; t < BQ; ++t) rv[t] = c0 + t < nb ? P::load(rj + c0 + t, planeR) : P::czero();
#pragma unroll
          for (int t = 0; t < BQ; ++t)
            if (c0 + t < nb) P::upd(gv[s], P::conj(rv[t]), P::load(xs + c0 + t, (size_t)BS_B));
        }
      }
    }
    __syncthreads();
  }
}

// gb = Q w and r = b - A x, split over column chunks of ADJ_CH columns so
// that the grid covers the device (rows x chunks x 2 products): each thread
// sums one row of one chunk in the fused accumulator (the chunk holding
// column 0 of r starts from b); adj_finish_kernel merges the chunk partials
// of a row in chunk order, so results are reproducible.
constexpr int ADJ_CH = 8;
constexpr int ADJ_T = 64;
template <class P>
__global__ __launch_bounds__(ADJ_T) void adj_partial_kernel(int m, int n, const double *Q, int ldq, size_t planeQ,
                                                             const double *A, int lda, size_t planeA,
                                                             const double *b, const double *x, const double *w,
                                                             typename P::Acc *partial) {
  using Acc = typename P::Acc;
  const int i = blockIdx.x * ADJ_T + threadIdx.x;
  const int cb = blockIdx.y, which = blockIdx.z;  // 0: Q w, 1: b - A x
  if (i >= m) return;
  const int nchunk = (n + ADJ_CH - 1) / ADJ_CH;
  const int j0 = cb * ADJ_CH, j1 = j0 + ADJ_CH < n ? j0 + ADJ_CH : n;
  Acc acc;
  if (which == 0) {
    P::acc_zero(acc);
#pragma unroll 4
    for (int k = j0; k < j1; ++k)
      P::acc_cmul(acc, P::load(Q + (size_t)k * ldq + i, planeQ), P::load(w + k, (size_t)n));
  } else {
    if (cb == 0)
      P::acc_set(acc, P::load(b + i, (size_t)m));
    else
      P::acc_zero(acc);
#pragma unroll 4
    for (int j = j0; j < j1; ++j)
      P::acc_cmul(acc, P::load(A + (size_t)j * lda + i, planeA), P::cneg(P::load(x + j, (size_t)n)));
  }
  partial[((size_t)which * nchunk + cb) * m + i] = acc;
}

template <class P>
__global__ __launch_bounds__(WG) void adj_finish_kernel(int m, int n, const typename P::Acc *partial, double *gb,
                                                         double *r) {
  using Acc = typename P::Acc;
  const int i = blockIdx.x * WG + threadIdx.x;
  const int which = blockIdx.y;
  if (i >= m) return;
  const int nchunk = (n + ADJ_CH - 1) / ADJ_CH;
  const Acc *p = partial + (size_t)which * nchunk * m + i;
  Acc acc = p[0];
  for (int c = 1; c < nchunk; ++c) P::acc_merge(acc, p[(size_t)c * m]);
  P::store((which == 0 ? gb : r) + i, (size_t)m, P::acc_value(acc));
}

// gA(i, j) = r_i conj(z_j) - gb_i conj(x_j): two fused updates from zero.
template <class P>
__global__ __launch_bounds__(WG) void adj_rank2_kernel(int m, int n, const double *r, const double *z,
                                                        const double *gb, const double *x, double *gA, int ldga,
                                                        size_t planeG) {
  using C = typename P::C;
  const int i = blockIdx.x * WG + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= m || j >= n) return;
  C a = P::czero();
  P::upd(a, P::cneg(P::load(r + i, (size_t)m)), P::conj(P::load(z + j, (size_t)n)));
  P::upd(a, P::load(gb + i, (size_t)m), P::conj(P::load(x + j, (size_t)n)));
  P::store(gA + (size_t)j * ldga + i, planeG, a);
}

}  // namespace mgsq
