// Newton's method for a polynomial system, all on the card (Section 7: the
// corrector of a path tracker solves thousands of linear systems; the
// system is transferred once, the evaluated Jacobian and system never leave
// the card).  Equation e of the system is
//   f_e(x) = sum_m c_em prod_t x_{v_emt}^{d_emt}
// (the workload of the paper's Table 6: 32 equations, 32 variables, 32
// monomials of 5 variables each).  One Newton step for a batch of points:
//   1. poly_eval_kernel: -f(x) and the Jacobian J(x) of every point, in the
//      layout of mgs_lstsq_batched (J column j = d f / d x_j; the same kernel
//      gives f itself to mgs_poly_eval);
//   2. the batched MGS on [J -f] and back substitution (batched_kernels.hpp):
//      the correction d, least-squares solution of J d = -f;
//   3. newton_update_kernel: x += d, and the FP64 norm of d.
#pragma once
#include "../../include/mgsqr.h"
#include "batched_kernels.hpp"

namespace mgsq {

constexpr int NT_MAX_MON = 64;   // monomials per equation (one lane each)
constexpr int NT_MAX_VARS = 63;  // variables (columns of [J -f] <= 64)
constexpr int NT_MAX_VPM = 8;    // variables per monomial
constexpr int NT_MAX_DEG = 16;   // exponent bound

template <class P>
__device__ __forceinline__ typename P::C nt_mul(const typename P::C &a, const typename P::C &b) {
  typename P::Acc acc;
  P::acc_zero(acc);
  P::acc_cmul(acc, a, b);
  return P::acc_value(acc);
}
template <class P>
__device__ __forceinline__ typename P::C nt_pow(const typename P::C &b, int d) {
  typename P::C r = P::czero();
  r.re = P::rone();
  for (int k = 0; k < d; ++k) r = nt_mul<P>(r, b);
  return r;
}

// One wave per (equation e, point s); lane m holds monomial m.  Its value
// c prod_t x_t^{d_t} and its derivatives c d_t x_t^{d_t - 1} prod_{u != t}
// x_u^{d_u} (prefix and suffix products) are formed in the working
// precision; f_e is a wave sum (DPP, fixed tree), and each Jacobian entry
// J(e, j) the sum, in monomial order, of the derivatives by x_j: the
// derivative entries are listed by variable (stable, so each list is in
// monomial order: counts, their prefix sum over the lanes, then a fill),
// and the lane of variable j merges its list from LDS, all lanes at once,
// in as many rounds as the longest list.  f_e (-f_e when negate) goes to
// b, J to A, both in the batched least-squares layout.
template <class P>
__global__ __launch_bounds__(64) void poly_eval_kernel(int neq, int nvar, int nmon, int nvpm, const int *vars,
                                                       const int *exps, const double *coef, const double *x,
                                                       double *A, double *b, bool negate) {
  using C = typename P::C;
  using Acc = typename P::Acc;
  constexpr int NP = 2 * P::L;
  __shared__ double xs[NP][NT_MAX_VARS];                       // the point
  __shared__ double ds[NP][NT_MAX_MON * NT_MAX_VPM];           // derivatives [m * nvpm + t]
  __shared__ int vs[NT_MAX_MON * NT_MAX_VPM];                  // their variables
  __shared__ int by_var[NT_MAX_MON * NT_MAX_VPM];              // entries listed by variable
  const int lane = threadIdx.x;
  const int e = blockIdx.x, s = blockIdx.y;
  const double *xp = x + (size_t)s * NP * nvar;
  if (lane < nvar) {
#pragma unroll
    for (int q = 0; q < NP; ++q) xs[q][lane] = xp[lane + (size_t)q * nvar];
  }
  __syncthreads();
  C mono = P::czero();
  const bool live = lane < nmon;
  if (live) {
    const size_t base = ((size_t)e * nmon + lane) * nvpm;
    C c = P::load(coef + (size_t)e * nmon + lane, (size_t)neq * nmon);
    C pw[NT_MAX_VPM], pd[NT_MAX_VPM];  // x_t^{d_t}, x_t^{d_t - 1}
    int vt[NT_MAX_VPM], dt[NT_MAX_VPM];
#pragma unroll
    for (int t = 0; t < NT_MAX_VPM; ++t) {
      if (t < nvpm) {
        // indices and exponents outside their bounds are clamped into them
        const int v0 = vars[base + t], d0 = exps[base + t];
        vt[t] = v0 < 0 ? 0 : (v0 >= nvar ? nvar - 1 : v0);
        dt[t] = d0 < 0 ? 0 : (d0 > NT_MAX_DEG ? NT_MAX_DEG : d0);
        const C xv = P::load(&xs[0][vt[t]], (size_t)NT_MAX_VARS);
        pd[t] = nt_pow<P>(xv, dt[t] > 0 ? dt[t] - 1 : 0);
        pw[t] = dt[t] > 0 ? nt_mul<P>(pd[t], xv) : pd[t];
      } else {
        vt[t] = 0;
        dt[t] = 0;
        pw[t] = pd[t] = P::czero();
      }
    }
    // prefix products pre[t] = c prod_{u < t} pw[u]; suffix products
    C pre[NT_MAX_VPM + 1];
    pre[0] = c;
#pragma unroll
    for (int t = 0; t < NT_MAX_VPM; ++t) pre[t + 1] = t < nvpm ? nt_mul<P>(pre[t], pw[t]) : pre[t];
    mono = pre[NT_MAX_VPM];
    C suf = P::czero();
    suf.re = P::rone();
#pragma unroll
    for (int t = NT_MAX_VPM - 1; t >= 0; --t) {
      if (t < nvpm) {
        C dv = P::czero();
        if (dt[t] > 0) {
          C k = P::czero();
          k.re = P::rfrom((double)dt[t]);
          dv = nt_mul<P>(nt_mul<P>(nt_mul<P>(pre[t], k), pd[t]), suf);
        }
        P::store(&ds[0][lane * nvpm + t], (size_t)NT_MAX_MON * NT_MAX_VPM, dv);
        vs[lane * nvpm + t] = vt[t];
        suf = nt_mul<P>(pw[t], suf);
      }
    }
  }
  // -f_e: wave sum of the monomials (lanes past nmon hold zero)
  Acc acc;
  P::acc_set(acc, mono);
  wave_sum_any<P>(acc, false);
  const C fe = P::acc_value(acc_lane63<P>(acc));
  double *bp = b + (size_t)s * NP * neq;
  if (lane == 0) P::store(bp + e, (size_t)neq, negate ? P::cneg(fe) : fe);
  __syncthreads();
  // J(e, j) for j = lane.  The entries of variable `lane`, in ascending
  // order, go to by_var[off, off + cnt).
  const int nent = nmon * nvpm;
  int cnt = 0;
  for (int k = 0; k < nent; ++k) cnt += vs[k] == lane ? 1 : 0;
  int off = cnt;  // inclusive scan over the lanes, then exclusive
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_up(off, d);
    if (lane >= d) off += o;
  }
  off -= cnt;
  {
    int w = off;
    for (int k = 0; k < nent; ++k) {
      if (vs[k] == lane) by_var[w++] = k;
    }
  }
  int rounds = cnt;
#pragma unroll
  for (int mask = 32; mask >= 1; mask >>= 1) rounds = max(rounds, __shfl_xor(rounds, mask));
  __syncthreads();
  Acc aj;
  P::acc_zero(aj);
  for (int c = 0; c < rounds; ++c) {
    if (c < cnt) {
      Acc d1;
      P::acc_set(d1, P::load(&ds[0][by_var[off + c]], (size_t)NT_MAX_MON * NT_MAX_VPM));
      P::acc_merge(aj, d1);
    }
  }
  if (lane < nvar) {
    double *ap = A + (size_t)s * NP * neq * nvar;
    P::store(ap + (size_t)lane * neq + e, (size_t)neq * nvar, P::acc_value(aj));
  }
}

// x += d for every point (one wave per point, lane j = variable j), and the
// FP64 2-norm of d (leading limbs) into dnorm[s] when dnorm is given.  A
// point whose factorisation failed (info[s] != 0) keeps its x and gets a
// NaN norm.
template <class P>
__global__ __launch_bounds__(64) void newton_update_kernel(int nvar, double *x, const double *d, const int *info,
                                                           double *dnorm) {
  using C = typename P::C;
  constexpr int NP = 2 * P::L;
  const int lane = threadIdx.x, s = blockIdx.x;
  if (info[s] != 0) {
    if (dnorm != nullptr && lane == 0) dnorm[s] = __builtin_nan("");
    return;
  }
  double *xp = x + (size_t)s * NP * nvar;
  const double *dp = d + (size_t)s * NP * nvar;
  double sq = 0.0;
  if (lane < nvar) {
    C xv = P::load(xp + lane, (size_t)nvar);
    const C dv = P::load(dp + lane, (size_t)nvar);
    C m1 = P::czero();
    m1.re = P::rfrom(-1.0);
    P::upd(xv, m1, dv);  // x - (-1) d
    P::store(xp + lane, (size_t)nvar, xv);
    sq = dp[lane] * dp[lane] + dp[lane + nvar] * dp[lane + nvar];
  }
#pragma unroll
  for (int mask = 32; mask >= 1; mask >>= 1) sq += __shfl_xor(sq, mask);
  if (dnorm != nullptr && lane == 0) dnorm[s] = sqrt(sq);
}

}  // namespace mgsq
