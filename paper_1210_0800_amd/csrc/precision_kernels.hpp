// Precision form: FP64 blocked MGS factorisation with the trailing Gram and
// update products on FP64 MFMA, then iterative refinement with the residual
// and the solution accumulated in dd / qd.
//
// Factorisation of [A b] in FP64, panels of NB = 64 columns:
//   factor panel p by MGS (Figure 1 restricted to the panel, the step
//   kernel with plain complex doubles), then for the columns right of it,
//   W = Q_p^H A_t (written into R) and A_t -= Q_p W.  b rides along as the
//   last column, so its panel projections y_p = W(:, n) are those of the
//   factorisation (the augmented semantics of Equation (1)).
// Correction solve of A d = r: the same panel projections replayed on r
// (w_p = Q_p^H r, r -= Q_p w_p), then back substitution with R.
// Refinement: r = b - A x in dd / qd, d = FP64 solve of fl64(r),
// x += d in dd / qd, until ||d|| <= tol ||x||, stagnation, or max_iter.
#pragma once
#include "mgs_kernels.hpp"
#include "resident_kernels.hpp"

namespace mgsq {

typedef double v4d __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 operand layout on gfx950 (checked on the device):
// A[i][k] in lane i + 16k, B[k][j] in lane j + 16k, D[i][j] in lane
// j + 16 (i % 4), register i / 4.
__device__ __forceinline__ v4d mfma16x16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int NBP = 64;  // panel width of the blocked factorisation

// The reduction index of a 16x16x4 product may follow any order of the
// summed rows, as long as both operands use it.  The kernels below give
// lane i + 16 kk the rows (or panel columns) 4 kk + s of a block of 16 in
// product step s = 0..3: each lane then reads 4 consecutive entries of its
// column at once, and the 4 lanes that share a column cover 128
// contiguous bytes, one cache line per column instead of a quarter of one
// per load.

// Four consecutive doubles from p[0..3]; entries at or past `lim` (counted
// from p) read as zero.  Whole blocks take wide loads.
__device__ __forceinline__ void load4(const double *p, int lim, double (&v)[4]) {
  if (lim >= 4) {
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = p[s];
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = s < lim ? p[s] : 0.0;
  }
}

// W (NBP x N) = Q_p^H (NBP x m) A_t (m x N), complex, planar FP64.
// Q_p: the panel's first column (plane stride plane), A_t: the first
// trailing column, W: output with leading dimension ldw (R's block row).
// One workgroup per 16 x 16 tile of W (grid: trailing column tiles x panel
// column tiles, 4 x 124 = 496 workgroups for the first 2048 panel, enough
// to occupy every compute unit); its QHA_SLICES waves each reduce over one
// slice of the m rows (a multiple of 16), and the slice partials are then
// summed in slice order through LDS, so the result does not depend on
// timing.
constexpr int QHA_SLICES = 8;
__global__ __launch_bounds__(64 * QHA_SLICES) void zgemm_qha_kernel(int m, int N, int nbp, const double *Qp, int ldq,
                                                                     const double *At, int lda, size_t plane,
                                                                     double *W, int ldw, size_t planeW) {
  __shared__ double red[QHA_SLICES - 1][64][8];
  const int lane = threadIdx.x & 63, ks = threadIdx.x >> 6;
  const int i0 = blockIdx.y * 16;  // panel column tile
  const int j0 = blockIdx.x * 16;  // trailing column tile
  const int li = lane & 15, lk = lane >> 4;
  const int qc = i0 + li;  // panel column read by this lane (A operand)
  const int tc = j0 + li;  // trailing column read by this lane (B operand)
  const bool qok = qc < nbp, tok = tc < N;
  const int mq = ((m + 16 * QHA_SLICES - 1) / (16 * QHA_SLICES)) * 16;  // rows per slice, multiple of 16
  const int k0 = ks * mq, k1 = min(m, k0 + mq);
  v4d cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
  const double *qr = Qp + (size_t)(qok ? qc : 0) * ldq, *qi = qr + plane;
  const double *ar = At + (size_t)(tok ? tc : 0) * lda, *ai = ar + plane;
#pragma unroll 2
  for (int kb = k0; kb < k1; kb += 16) {
    const int row = kb + 4 * lk;  // rows row .. row + 3 of this lane
    const int lim = k1 - row;
    double a_r[4], a_i[4], b_r[4], b_i[4];
    load4(qr + row, qok ? lim : 0, a_r);
    load4(qi + row, qok ? lim : 0, a_i);
    load4(ar + row, tok ? lim : 0, b_r);
    load4(ai + row, tok ? lim : 0, b_i);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      // conj(q) a: re = qr ar + qi ai, im = qr ai - qi ar
      cr = mfma16x16x4(a_r[s], b_r[s], cr);
      cr = mfma16x16x4(a_i[s], b_i[s], cr);
      ci = mfma16x16x4(a_r[s], b_i[s], ci);
      ci = mfma16x16x4(-a_i[s], b_r[s], ci);
    }
  }
  if (ks > 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      red[ks - 1][lane][r] = cr[r];
      red[ks - 1][lane][4 + r] = ci[r];
    }
  }
  __syncthreads();
  if (ks != 0) return;
#pragma unroll
  for (int s = 0; s < QHA_SLICES - 1; ++s) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      cr[r] += red[s][lane][r];
      ci[r] += red[s][lane][4 + r];
    }
  }
  const int oc = j0 + li;
  if (oc < N) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int orow = i0 + lk + 4 * r;
      if (orow < nbp) {
        W[(size_t)oc * ldw + orow] = cr[r];
        W[(size_t)oc * ldw + orow + planeW] = ci[r];
      }
    }
  }
}

// A_t (m x N) -= Q_p (m x nbp) W (nbp x N).  One wave per 16 x 16 tile of
// A_t, K = nbp in blocks of 16 panel columns (the lane order above: W
// read 4 consecutive rows at a time, Q_p one column per product step,
// 16 consecutive rows across the lanes).
__global__ __launch_bounds__(256) void zgemm_update_kernel(int m, int N, int nbp, const double *Qp, int ldq,
                                                            double *At, int lda, size_t plane, const double *W,
                                                            int ldw, size_t planeW) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tiles_m = (m + 15) / 16;
  const int tile = blockIdx.x * 4 + wave;
  const int ti = tile % tiles_m, tj = tile / tiles_m;
  if (tj * 16 >= N) return;
  const int i0 = ti * 16, j0 = tj * 16;
  const int li = lane & 15, lk = lane >> 4;
  // output tile values (D layout): row i0 + lk + 4r, column j0 + li
  const int oc = j0 + li;
  const bool cok = oc < N;
  v4d cr, ci;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int orow = i0 + lk + 4 * r;
    const bool ok = cok && orow < m;
    cr[r] = ok ? At[(size_t)oc * lda + orow] : 0.0;
    ci[r] = ok ? At[(size_t)oc * lda + orow + plane] : 0.0;
  }
  const int arow = i0 + li;  // A operand row (Q_p)
  const bool aok = arow < m;
  const double *wr = W + (size_t)(cok ? oc : 0) * ldw, *wi = wr + planeW;
  for (int kb = 0; kb < nbp; kb += 16) {
    const int k = kb + 4 * lk;  // panel columns k .. k + 3 of this lane
    const int lim = nbp - k;
    double w_r[4], w_i[4];
    load4(wr + k, cok ? lim : 0, w_r);
    load4(wi + k, cok ? lim : 0, w_i);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool kok = aok && s < lim;
      const double q_r = kok ? Qp[(size_t)(k + s) * ldq + arow] : 0.0;
      const double q_i = kok ? Qp[(size_t)(k + s) * ldq + arow + plane] : 0.0;
      // a -= q w: re -= qr wr - qi wi, im -= qr wi + qi wr
      cr = mfma16x16x4(-q_r, w_r[s], cr);
      cr = mfma16x16x4(q_i, w_i[s], cr);
      ci = mfma16x16x4(-q_r, w_i[s], ci);
      ci = mfma16x16x4(-q_i, w_r[s], ci);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int orow = i0 + lk + 4 * r;
    if (cok && orow < m) {
      At[(size_t)oc * lda + orow] = cr[r];
      At[(size_t)oc * lda + orow + plane] = ci[r];
    }
  }
}

// ------------------------------------------------------- refinement ------
struct RefineCtl {
  int status;  // 0 running, 1 converged, 2 stagnated, 3 factorisation failed or a grid wait timed out
  int iters;
  double dprev;
  double err_est;
  unsigned int bar;    // arrivals at the grid barriers of proj_replay_kernel (zero at the start of a solve)
  unsigned int abort;  // set when one of its waits timed out
};

// Columns of Q64 (m x (n+1), ld m) from the leading limbs of A and b.
template <int L>
__global__ __launch_bounds__(256) void copy_hi_kernel(int m, int n, const double *A, int lda, const double *b,
                                                       double *Q64, RefineCtl *ctl, int *info) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (blockIdx.x == 0 && j == 0 && threadIdx.x == 0) {
    ctl->status = 0;
    ctl->iters = 0;
    ctl->dprev = INFINITY;
    ctl->err_est = INFINITY;
    ctl->bar = 0u;
    ctl->abort = 0u;
    *info = 0;
  }
  if (i >= m) return;
  const size_t plane64 = (size_t)m * (n + 1);
  if (j < n) {
    const size_t planeA = (size_t)lda * n;
    Q64[(size_t)j * m + i] = A[(size_t)j * lda + i];
    Q64[(size_t)j * m + i + plane64] = A[(size_t)j * lda + i + planeA];
  } else {
    Q64[(size_t)n * m + i] = b[i];
    Q64[(size_t)n * m + i + plane64] = b[i + m];
  }
}

// mgs_qr64: [A b] (FP64 complex planar, lda) into the working matrix
// Q64 (m x (n+1), column n = b or zero); clears info.
__global__ __launch_bounds__(256) void copy64_in_kernel(int m, int n, const double *A, int lda, const double *b,
                                                         double *Q64, int *info) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (blockIdx.x == 0 && j == 0 && threadIdx.x == 0) *info = 0;
  if (i >= m) return;
  const size_t plane64 = (size_t)m * (n + 1);
  if (j < n) {
    const size_t planeA = (size_t)lda * n;
    Q64[(size_t)j * m + i] = A[(size_t)j * lda + i];
    Q64[(size_t)j * m + i + plane64] = A[(size_t)j * lda + i + planeA];
  } else {
    Q64[(size_t)n * m + i] = b != nullptr ? b[i] : 0.0;
    Q64[(size_t)n * m + i + plane64] = b != nullptr ? b[i + m] : 0.0;
  }
}
// mgs_qr64: Q (m x n, ldq), R (n x n, ldr) and y (n) out of Q64 / R64.
// Block column j < n copies column j of Q and of R; j == n copies y.
__global__ __launch_bounds__(256) void copy64_out_kernel(int m, int n, const double *Q64, const double *R64,
                                                          double *Q, int ldq, double *R, int ldr, double *y) {
  const int j = blockIdx.y;
  const size_t plane64 = (size_t)m * (n + 1), planeR64 = (size_t)n * (n + 1);
  if (j < n) {
    const size_t planeQ = (size_t)ldq * n, planeR = (size_t)ldr * n;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256) {
      Q[(size_t)j * ldq + i] = Q64[(size_t)j * m + i];
      Q[(size_t)j * ldq + i + planeQ] = Q64[(size_t)j * m + i + plane64];
    }
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
      R[(size_t)j * ldr + i] = R64[(size_t)j * n + i];
      R[(size_t)j * ldr + i + planeR] = R64[(size_t)j * n + i + planeR64];
    }
  } else if (y != nullptr) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
      y[i] = R64[(size_t)n * n + i];
      y[i + n] = R64[(size_t)n * n + i + planeR64];
    }
  }
}

__global__ __launch_bounds__(256) void fill_zero_kernel(double *p, size_t count) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256) p[i] = 0.0;
}

// r = b - A x accumulated in quad-double whatever the working precision
// (A, b, x stored with LP limbs are widened exactly), split over column
// chunks: block (rb, cb) sums the columns [cb*CH, cb*CH + CH) of rows
// rb*256 .. into partial[cb][row].  Only the FP64 rounding of r feeds the
// correction; twice the working precision for dd keeps the residual's own
// error below the dd solution's.
template <int LP>
__device__ __forceinline__ cqd load_qd_from(const double *p, size_t plane) {
  cqd v;
  v.re.x0 = p[0];
  v.im.x0 = p[plane];
  v.re.x1 = LP > 1 ? p[2 * plane] : 0.0;
  v.im.x1 = LP > 1 ? p[3 * plane] : 0.0;
  v.re.x2 = LP > 2 ? p[4 * plane] : 0.0;
  v.im.x2 = LP > 2 ? p[5 * plane] : 0.0;
  v.re.x3 = LP > 2 ? p[6 * plane] : 0.0;
  v.im.x3 = LP > 2 ? p[7 * plane] : 0.0;
  return v;
}
template <int LP>
__global__ __launch_bounds__(256) void residual_partial_kernel(int m, int n, int chunk, const double *A, int lda,
                                                                const double *b, const double *x,
                                                                PrecQD::Acc *partial, const RefineCtl *ctl) {
  if (ctl->status != 0) return;
  using P = PrecQD;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int cb = blockIdx.y;
  if (i >= m) return;
  const size_t planeA = (size_t)lda * n;
  P::Acc acc;
  if (cb == 0)
    P::acc_set(acc, load_qd_from<LP>(b + i, (size_t)m));
  else
    P::acc_zero(acc);
  const int j1 = min(n, (cb + 1) * chunk);
  for (int j = cb * chunk; j < j1; ++j)
    P::acc_cmul(acc, load_qd_from<LP>(A + (size_t)j * lda + i, planeA), P::cneg(load_qd_from<LP>(x + j, (size_t)n)));
  partial[(size_t)cb * m + i] = acc;
}

// Sum the chunk partials in chunk order; r64 = FP64 rounding of r.
template <class P>
__global__ __launch_bounds__(256) void residual_finish_kernel(int m, int nchunk, const typename P::Acc *partial,
                                                               double *r64, const RefineCtl *ctl) {
  if (ctl->status != 0) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  typename P::Acc acc = partial[i];
  for (int c = 1; c < nchunk; ++c) P::acc_merge(acc, partial[(size_t)c * m + i]);
  typename P::C v = P::acc_value(acc);
  double tmp[2 * P::L];
  P::store(tmp, 1, v);  // tmp[0] = re hi, tmp[1] = im hi (planes 0 and 1)
  r64[i] = tmp[0];
  r64[i + m] = tmp[1];
}

// w = Q_p^H r: one block per panel column, rows summed in a fixed order.
__global__ __launch_bounds__(256) void proj_w_kernel(int m, const double *Qp, int ldq, size_t plane,
                                                      const double *r, double *w, size_t planew,
                                                      const RefineCtl *ctl) {
  if (ctl->status != 0) return;
  __shared__ double sr[4], si[4];
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double *qr = Qp + (size_t)c * ldq, *qi = qr + plane;
  double ar = 0.0, ai = 0.0;
  for (int i = tid; i < m; i += 256) {
    const double xr = r[i], xi = r[i + m];
    ar = __fma_rn(qr[i], xr, ar);
    ar = __fma_rn(qi[i], xi, ar);
    ai = __fma_rn(qr[i], xi, ai);
    ai = __fma_rn(-qi[i], xr, ai);
  }
#pragma unroll
  for (int mask = 32; mask >= 1; mask >>= 1) {
    ar += __shfl_xor(ar, mask);
    ai += __shfl_xor(ai, mask);
  }
  if (lane == 0) {
    sr[wave] = ar;
    si[wave] = ai;
  }
  __syncthreads();
  if (tid == 0) {
    w[c] = ((sr[0] + sr[1]) + sr[2]) + sr[3];
    w[c + planew] = ((si[0] + si[1]) + si[2]) + si[3];
  }
}

// r -= Q_p w, one row per thread.
__global__ __launch_bounds__(256) void proj_r_kernel(int m, int nbp, const double *Qp, int ldq, size_t plane,
                                                      const double *w, size_t planew, double *r,
                                                      const RefineCtl *ctl) {
  if (ctl->status != 0) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  double xr = r[i], xi = r[i + m];
  for (int c = 0; c < nbp; ++c) {
    const double qr = Qp[(size_t)c * ldq + i], qi = Qp[(size_t)c * ldq + i + plane];
    const double wr = w[c], wi = w[c + planew];
    xr = __fma_rn(-qr, wr, xr);
    xr = __fma_rn(qi, wi, xr);
    xi = __fma_rn(-qr, wi, xi);
    xi = __fma_rn(-qi, wr, xi);
  }
  r[i] = xr;
  r[i + m] = xi;
}

// The correction's projections of all panels in one cooperative launch (one
// per refinement step instead of two per panel): for each panel of NBP
// columns, w_p = Q_p^H r (workgroup g forms columns g, g + G, ... with the
// operations of proj_w_kernel), a grid barrier, r -= Q_p w_p (rows spread
// over the grid, the operations of proj_r_kernel), a grid barrier.  Every
// value is formed by one workgroup in a fixed order, so the results are
// those of the per-panel kernels, bit for bit.  r and w pass between
// workgroups with device-scope loads and stores (Q, written before the
// launch, with plain loads), so a barrier needs no cache maintenance: every
// wave waits for its stores to complete, then one thread per workgroup
// counts its arrival in ctl->bar (which grows by G per barrier from `base`,
// the arrivals of the earlier steps of this solve) and waits, bounded, for
// the others; on a time-out the step ends with status 3 and
// MGS_INFO_SYNC_TIMEOUT in info.  m <= PR_MAX_ROWS.
constexpr int PR_MAX_ROWS = 4096;
__global__ __launch_bounds__(256) void proj_replay_kernel(int m, int n, const double *Q, size_t planeQ, double *r,
                                                           double *w, size_t planew, RefineCtl *ctl, int *info,
                                                           unsigned int base, long long spin_ticks,
                                                           unsigned jitter) {
  if (ctl->status != 0) return;
  constexpr int NS = PR_MAX_ROWS / 256;
  __shared__ double sr[4], si[4];
  __shared__ double wl[2][NBP];
  __shared__ int ok;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int G = gridDim.x, g = blockIdx.x;
  unsigned int target = base;
  unsigned step = 0;
  auto grid_barrier = [&]() __attribute__((always_inline)) -> bool {
    res_jitter(jitter, step++);
    wait_vmem();  // this wave's device-scope stores of r and w have completed
    __syncthreads();
    target += (unsigned int)G;
    if (tid == 0) {
      atomicAdd(&ctl->bar, 1u);
      const long long t0 = wall_clock64();
      int good = 1;
      while (__hip_atomic_load(&ctl->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
            wall_clock64() - t0 > spin_ticks) {
          __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          good = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      ok = good;
    }
    __syncthreads();
    asm volatile("" ::: "memory");
    return ok != 0;
  };
  auto fail = [&]() __attribute__((always_inline)) {
    if (tid == 0) {
      ctl->status = 3;
      __hip_atomic_store(info, MGS_INFO_SYNC_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  for (int k0 = 0; k0 < n; k0 += NBP) {
    const int nb = n - k0 < NBP ? n - k0 : NBP;
    const double *Qp = Q + (size_t)k0 * m;
    double *wp = w + k0;
    if (g < nb) {
      // this thread's rows tid + 256 s of r, all loads in flight together
      double xr[NS], xi[NS];
#pragma unroll
      for (int s2 = 0; s2 < NS; ++s2) {
        const int i = tid + 256 * s2;
        xr[s2] = i < m ? coh_load(r + i) : 0.0;
        xi[s2] = i < m ? coh_load(r + i + m) : 0.0;
      }
      for (int c = g; c < nb; c += G) {
        const double *qr = Qp + (size_t)c * m, *qi = qr + planeQ;
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2) {
          const int i = tid + 256 * s2;
          if (i < m) {
            ar = __fma_rn(qr[i], xr[s2], ar);
            ar = __fma_rn(qi[i], xi[s2], ar);
            ai = __fma_rn(qr[i], xi[s2], ai);
            ai = __fma_rn(-qi[i], xr[s2], ai);
          }
        }
#pragma unroll
        for (int mask = 32; mask >= 1; mask >>= 1) {
          ar += __shfl_xor(ar, mask);
          ai += __shfl_xor(ai, mask);
        }
        if (lane == 0) {
          sr[wave] = ar;
          si[wave] = ai;
        }
        __syncthreads();
        if (tid == 0) {
          coh_store(wp + c, ((sr[0] + sr[1]) + sr[2]) + sr[3]);
          coh_store(wp + c + planew, ((si[0] + si[1]) + si[2]) + si[3]);
        }
        __syncthreads();
      }
    }
    if (!grid_barrier()) return fail();
    if (g * 256 < m) {
      if (tid < nb) {
        wl[0][tid] = coh_load(wp + tid);
        wl[1][tid] = coh_load(wp + tid + planew);
      }
      __syncthreads();
      for (int i = g * 256 + tid; i < m; i += G * 256) {
        double xr = coh_load(r + i), xi = coh_load(r + i + m);
        for (int c = 0; c < nb; ++c) {
          const double qr = Qp[(size_t)c * m + i], qi = Qp[(size_t)c * m + i + planeQ];
          const double wr = wl[0][c], wi = wl[1][c];
          xr = __fma_rn(-qr, wr, xr);
          xr = __fma_rn(qi, wi, xr);
          xi = __fma_rn(-qr, wi, xi);
          xi = __fma_rn(-qi, wr, xi);
        }
        coh_store(r + i, xr);
        coh_store(r + i + m, xi);
      }
    }
    if (!grid_barrier()) return fail();
  }
}

// The FP64 solution as the dd / qd starting x (first solve).
template <class P>
__global__ __launch_bounds__(256) void set_x_kernel(int n, const double *x64, double *x) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  for (int p = 0; p < 2 * P::L; ++p) x[i + (size_t)p * n] = (p < 2) ? x64[i + (size_t)p * n] : 0.0;
}

// x += d (d in FP64), with the stopping test on ||d|| and ||x||: stop when
// ||d|| <= tol ||x|| (converged) or ||d|| > ||d_prev|| / 2 (stalled).  One block.
template <class P>
__global__ __launch_bounds__(256) void refine_update_kernel(int n, const double *d64, double *x, double tol,
                                                             int iter, RefineCtl *ctl) {
  if (ctl->status != 0) return;
  __shared__ double red[2][4];
  __shared__ int stag;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double dn = 0.0, xn = 0.0;
  for (int i = tid; i < n; i += 256) {
    const double dr = d64[i], di = d64[i + n];
    dn = __fma_rn(dr, dr, __fma_rn(di, di, dn));
    const double xr = x[i], xi = x[i + n];
    xn = __fma_rn(xr, xr, __fma_rn(xi, xi, xn));
  }
#pragma unroll
  for (int mask = 32; mask >= 1; mask >>= 1) {
    dn += __shfl_xor(dn, mask);
    xn += __shfl_xor(xn, mask);
  }
  if (lane == 0) {
    red[0][wave] = dn;
    red[1][wave] = xn;
  }
  __syncthreads();
  dn = sqrt(((red[0][0] + red[0][1]) + red[0][2]) + red[0][3]);
  xn = sqrt(((red[1][0] + red[1][1]) + red[1][2]) + red[1][3]);
  if (tid == 0) stag = (iter > 1 && dn > 0.5 * ctl->dprev) ? 1 : 0;
  __syncthreads();
  if (stag) {
    // The corrections stopped shrinking: converged to the attainable
    // accuracy when the last applied one was already below sqrt(tol) of x,
    // a failure otherwise.  The stalled correction is not applied.
    if (tid == 0) ctl->status = (ctl->err_est <= sqrt(tol)) ? 1 : 2;
    return;
  }
  for (int i = tid; i < n; i += 256) {
    typename P::C v = P::load(x + i, (size_t)n);
    P::add_cd(v, d64[i], d64[i + n]);
    P::store(x + i, (size_t)n, v);
  }
  if (tid == 0) {
    ctl->iters = iter;
    ctl->err_est = xn > 0.0 ? dn / xn : dn;
    ctl->dprev = dn;
    if (dn <= tol * xn) ctl->status = 1;
  }
}

// Skip the refinement when the factorisation reported a bad column.
__global__ void refine_check_kernel(const int *info, RefineCtl *ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && *info != 0) ctl->status = 3;
}

__global__ void refine_finish_kernel(const RefineCtl *ctl, int *iters, double *err_est, int *info) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (iters) *iters = ctl->iters;
  if (err_est) *err_est = ctl->err_est;
  if (*info == 0) *info = ctl->status == 1 ? 0 : (ctl->status == 2 ? -1 : -2);
}

}  // namespace mgsq
