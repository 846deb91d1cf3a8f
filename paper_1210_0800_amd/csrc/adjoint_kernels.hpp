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
// g_j -= conj(r_kj) w_k for j > k.  One block; thread tid keeps g_j for
// j = s*WG + tid; the row k+1 of R is fetched while step k is in progress.
template <class P, int NY>
__global__ __launch_bounds__(WG) void fwdsub_kernel(int n, const double *R, int ldr, size_t planeR,
                                                     const double *g, double *w, int *info) {
  using C = typename P::C;
  using Rl = typename P::R;
  __shared__ C ws[2];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0x7fffffff;
  __syncthreads();
  C gv[NY];
  Rl inv[NY];
#pragma unroll
  for (int s = 0; s < NY; ++s) {
    int j = s * WG + tid;
    if (j < n) {
      gv[s] = P::load(g + j, (size_t)n);
      C d = P::load(R + (size_t)j * ldr + j, planeR);
      if (!P::ok_norm(d.re)) atomicMin(&bad, j + 1);
      inv[s] = P::recip(d.re);
    } else {
      gv[s] = P::czero();
      inv[s] = P::rzero();
    }
  }
  __syncthreads();
  if (tid == 0) *info = (bad == 0x7fffffff) ? 0 : bad;
  // rk[s] = R(k, j) for the current k (row k of R, strided in memory)
  C rk[NY];
#pragma unroll
  for (int s = 0; s < NY; ++s) {
    int j = s * WG + tid;
    rk[s] = (j > 0 && j < n) ? P::load(R + (size_t)j * ldr + 0, planeR) : P::czero();
  }
#pragma unroll 1
  for (int k = 0; k < n; ++k) {
    const int sk = k / WG, owner = k - sk * WG;
    C rn[NY];
#pragma unroll
    for (int s = 0; s < NY; ++s) {
      int j = s * WG + tid;
      rn[s] = (j > k + 1 && j < n) ? P::load(R + (size_t)j * ldr + (k + 1), planeR) : P::czero();
    }
    if (tid == owner) {
#pragma unroll
      for (int s = 0; s < NY; ++s) {
        if (s == sk) {
          C wk = P::scale(gv[s], inv[s]);
          P::store(w + k, (size_t)n, wk);
          ws[k & 1] = wk;
        }
      }
    }
    __syncthreads();
    const C wk = ws[k & 1];
#pragma unroll
    for (int s = 0; s < NY; ++s) {
      int j = s * WG + tid;
      if (j > k && j < n) P::upd(gv[s], P::conj(rk[s]), wk);
      rk[s] = rn[s];
    }
  }
}

// gb = Q w and r = b - A x, one row per thread, sums over the columns in
// ascending order in the fused accumulators.
template <class P>
__global__ __launch_bounds__(WG) void adj_gemv_kernel(int m, int n, const double *Q, int ldq, size_t planeQ,
                                                       const double *A, int lda, size_t planeA, const double *b,
                                                       const double *x, const double *w, double *gb, double *r) {
  using Acc = typename P::Acc;
  const int i = blockIdx.x * WG + threadIdx.x;
  if (i >= m) return;
  Acc acc;
  P::acc_zero(acc);
#pragma unroll 4
  for (int k = 0; k < n; ++k) P::acc_cmul(acc, P::load(Q + (size_t)k * ldq + i, planeQ), P::load(w + k, (size_t)n));
  P::store(gb + i, (size_t)m, P::acc_value(acc));
  P::acc_set(acc, P::load(b + i, (size_t)m));
#pragma unroll 4
  for (int j = 0; j < n; ++j)
    P::acc_cmul(acc, P::load(A + (size_t)j * lda + i, planeA), P::cneg(P::load(x + j, (size_t)n)));
  P::store(r + i, (size_t)m, P::acc_value(acc));
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
