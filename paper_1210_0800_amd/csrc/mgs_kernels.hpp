// MGS QR, least-squares solve and back substitution kernels for gfx950.
//
// The factorisation follows Figure 1 of the paper (Section 3) on the matrix
// augmented with the right-hand side (Equation (1)): for every column k,
// r_kk = ||a_k||, q_k = a_k / r_kk, and for every later column j (b
// included) r_kj = q_k^H a_j, a_j -= r_kj q_k.  Every column j receives the
// projections in the order k = 1, 2, ..., j-1, exactly as in Figure 1; only
// the schedule differs from the paper's one launch per column (Section 5,
// Figure 2):
//
//   launch t (one per panel of `bw` columns, plus one for b):
//     block 0   ("panel")    applies the projections of panel t-1 to the
//               columns of panel t, then factors panel t (norms, square
//               roots, normalisation, projections inside the panel).  The
//               block's 4 waves spread the rows; reductions are wave
//               butterflies plus a 4-way exchange through LDS.
//     blocks 1+ ("trailing") apply the projections of panel t-1 to every
//               column beyond panel t: one column per team of `tw` waves,
//               the column held in registers (rpt rows per lane), q_k read
//               from L2, reductions by wave butterflies (plus LDS when tw>1).
//   So panel t is factored while the trailing matrix absorbs panel t-1
//   (one panel of look-ahead); the kernel boundary orders the panels.
//
// Reductions use a fixed butterfly order, so every lane of a team ends with
// the bitwise identical r_kj and results are reproducible run to run.
#pragma once
#include <utility>

#include "ddqd.hpp"

namespace mgsq {

constexpr int WG = 256;
constexpr int NWAVE = WG / 64;

// Compile-time loop: f(std::integral_constant<int, i>) for i = 0..N-1, so
// that register arrays indexed by i keep static indices however large the
// body is.
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Waits for this wave's LDS operations (through the builtin, so that the
// compiler knows they are done; the asm statements keep it from moving
// memory accesses across the wait).
__device__ __forceinline__ void lds_wait() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);
  asm volatile("" ::: "memory");
}

// Block barrier for LDS traffic only: waits for this wave's LDS operations
// (s_waitcnt lgkmcnt(0) through the builtin, so that the compiler knows
// they are done), then s_barrier.  Unlike __syncthreads() it does not wait
// for outstanding global loads, so register loads of a column can stay in
// flight across it.  The asm statements keep the compiler from moving
// memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);
  asm volatile("s_barrier" ::: "memory");
}

struct StepArgs {
  int m, n, ncols;  // ncols = n + 1 when b is augmented
  const double *A;
  int lda;
  size_t planeA;
  const double *b;  // original right-hand side (plane stride m) or null
  double *Q;
  int ldq;
  size_t planeQ;
  double *R;
  int ldr;
  size_t planeR;
  double *W;  // working copy of the augmented column (plane stride m)
  double *y;
  double *rho;
  int *info;
  int bw, t, npanel;
  int mpad;    // rows padded to the launch shape: LDS plane stride, multiple of WG
  int qstage;  // q vectors staged in LDS at a time
  int kbase;   // column offset of this matrix in the caller's, for info
  int init_info;  // the first launch clears *info
};

// Copy q_k0 .. q_{k0+cnt-1} from Q into LDS, layout [vector][plane][row]
// with plane stride mpad; rows m .. mpad-1 are zero.  Up to 16 loads per
// thread are in flight before the LDS stores.
template <class P>
__device__ __forceinline__ void stage_q(const StepArgs &a, int k0, int cnt, double *qs) {
  const int tid = threadIdx.x;
  const int chunks = a.mpad / WG;
  const int total = cnt * 2 * P::L * chunks;
  for (int base = 0; base < total; base += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = base + u;  // uniform across the block
      v[u] = 0.0;
      if (e < total) {
        const int cp = e / chunks, ch = e - cp * chunks;
        const int c = cp / (2 * P::L), p = cp - c * (2 * P::L);
        const int row = ch * WG + tid;
        if (row < a.m) v[u] = a.Q[(size_t)(k0 + c) * a.ldq + (size_t)p * a.planeQ + row];
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = base + u;
      if (e < total) {
        const int cp = e / chunks, ch = e - cp * chunks;
        qs[(size_t)cp * a.mpad + ch * WG + tid] = v[u];
      }
    }
  }
}

// Column j as read at launch t: on its first touch from A (or b), later
// from the working storage Q (or W).
__device__ __forceinline__ const double *col_src(const StepArgs &a, int j, bool first, size_t &plane) {
  if (j < a.n) {
    if (first) {
      plane = a.planeA;
      return a.A + (size_t)j * a.lda;
    }
    plane = a.planeQ;
    return a.Q + (size_t)j * a.ldq;
  }
  plane = (size_t)a.m;
  return first ? a.b : a.W;
}
__device__ __forceinline__ double *col_dst(const StepArgs &a, int j, size_t &plane) {
  if (j < a.n) {
    plane = a.planeQ;
    return a.Q + (size_t)j * a.ldq;
  }
  plane = (size_t)a.m;
  return a.W;
}
// r_kj goes to R(k, j), or to y(k) for the augmented column.
template <class P>
__device__ __forceinline__ void store_r(const StepArgs &a, int k, int j, const typename P::C &v) {
  if (j < a.n)
    P::store(a.R + (size_t)j * a.ldr + k, a.planeR, v);
  else
    P::store(a.y + k, (size_t)a.n, v);
}

template <class P>
__device__ __forceinline__ void wave_reduce(typename P::Acc &acc) {
#pragma unroll
  for (int mask = 32; mask >= 1; mask >>= 1) {
    typename P::Acc o = P::acc_shfl_xor(acc, mask);
    P::acc_merge(acc, o);
  }
}
template <class P>
__device__ __forceinline__ void wave_reduce_re(typename P::Acc &acc) {
#pragma unroll
  for (int mask = 32; mask >= 1; mask >>= 1) {
    typename P::Acc o = P::acc_shfl_xor_re(acc, mask);
    P::acc_merge_re(acc, o);
  }
}

// Batched block reduction of the accumulators c in [c_lo, c_hi): wave
// butterflies, then the partials of the first nwd waves combined in wave
// order through LDS (the waves past them hold only rows beyond m, whose
// partials are zero).
template <class P, int BWM>
__device__ __forceinline__ void block_reduce(typename P::Acc (&acc)[BWM], int c_lo, int c_hi,
                                             typename P::Acc *lds, int wave, int lane, int nwd) {
#pragma unroll
  for (int c = 0; c < BWM; ++c)
    if (c >= c_lo && c < c_hi) wave_reduce<P>(acc[c]);
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < BWM; ++c)
      if (c >= c_lo && c < c_hi) lds[wave * BWM + c] = acc[c];
  }
  lds_barrier();
#pragma unroll
  for (int c = 0; c < BWM; ++c) {
    if (c >= c_lo && c < c_hi) {
      acc[c] = lds[c];
#pragma unroll
      for (int w = 1; w < NWAVE; ++w)
        if (w < nwd) P::acc_merge(acc[c], lds[w * BWM + c]);
    }
  }
  lds_barrier();
}

// ------------------------------------------------------------ panel role --
// Thread tid holds rows i = r*WG + tid (r < RP) of the panel's columns;
// rows beyond m are zero, so the inner loops carry no bounds tests.
template <class P, int RP, int BWM>
__device__ __forceinline__ void panel_role(const StepArgs &a, typename P::Acc *lds, double *qs) {
  using C = typename P::C;
  using Acc = typename P::Acc;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int k0 = a.t * a.bw;
  const int nb = min(a.bw, a.n - k0);
  const bool first = a.t <= 1;
  // waves holding rows below m (rows r WG + tid): the others' partials are zero
  const int nwd = RP > 1 ? NWAVE : min(NWAVE, (a.m + 63) / 64);
  if (a.t == 0 && tid == 0 && a.init_info) *a.info = 0;

  C col[BWM][RP];
#pragma unroll
  for (int c = 0; c < BWM; ++c) {
    size_t ps;
    const double *src = col_src(a, k0 + c, first, ps);
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      int i = r * WG + tid;
      col[c][r] = (c < nb && i < a.m) ? P::load(src + i, ps) : P::czero();
    }
  }

  // Look-ahead: projections of panel t-1 onto panel t, k in order, the
  // q vectors read from LDS.
  if (a.t > 0) {
    const int kp0 = k0 - a.bw;
#pragma unroll 1
    for (int kc = kp0; kc < k0; kc += a.qstage) {
      const int cnt = min(a.qstage, k0 - kc);
      lds_barrier();
      stage_q<P>(a, kc, cnt, qs);
      lds_barrier();
#pragma unroll 1
      for (int cc = 0; cc < cnt; ++cc) {
        const int k = kc + cc;
        const double *qk = qs + (size_t)cc * 2 * P::L * a.mpad;
        C q[RP];
#pragma unroll
        for (int r = 0; r < RP; ++r) q[r] = P::load(qk + r * WG + tid, (size_t)a.mpad);
        Acc acc[BWM];
#pragma unroll
        for (int c = 0; c < BWM; ++c) {
          P::acc_zero(acc[c]);
          if (c < nb) {
#pragma unroll
            for (int r = 0; r < RP; ++r) P::acc_cmulc(acc[c], q[r], col[c][r]);
          }
        }
        block_reduce<P, BWM>(acc, 0, nb, lds, wave, lane, nwd);
#pragma unroll
        for (int c = 0; c < BWM; ++c) {
          if (c < nb) {
            C rk = P::acc_value(acc[c]);
            if (tid == 0) store_r<P>(a, k, k0 + c, rk);
#pragma unroll
            for (int r = 0; r < RP; ++r) P::upd(col[c][r], rk, q[r]);
          }
        }
      }
    }
  }

  // Factor the panel: Figure 1 restricted to columns k0 .. k0+nb-1.
  static_for<BWM>([&](auto cI) __attribute__((always_inline)) {
    constexpr int c = decltype(cI)::value;
    if (c < nb) {
      const int k = k0 + c;
      Acc nacc;
      P::acc_zero(nacc);
#pragma unroll
      for (int r = 0; r < RP; ++r) P::acc_abs2(nacc, col[c][r]);
      wave_reduce_re<P>(nacc);
      if (lane == 0) lds[wave * BWM + c] = nacc;
      lds_barrier();
      Acc s = lds[c];
#pragma unroll
      for (int w = 1; w < NWAVE; ++w)
        if (w < nwd) P::acc_merge_re(s, lds[w * BWM + c]);
      lds_barrier();
      typename P::R s2 = P::acc_value_re(s);
      if (!P::ok_norm(s2) && tid == 0 && *a.info == 0) *a.info = a.kbase + k + 1;
      typename P::R rkk, inv;
      root_and_inverse<P>(s2, rkk, inv);
      size_t pq;
      double *dst = col_dst(a, k, pq);
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        col[c][r] = P::scale(col[c][r], inv);
        int i = r * WG + tid;
        if (i < a.m) P::store(dst + i, pq, col[c][r]);
      }
      // R(k,k) = r_kk (imaginary +0); R(i,k) = 0 below the diagonal.
      if (tid == 0) {
        C d;
        d.re = rkk;
        d.im = P::rzero();
        P::store(a.R + (size_t)k * a.ldr + k, a.planeR, d);
      }
      for (int i = k + 1 + tid; i < a.n; i += WG) P::store(a.R + (size_t)k * a.ldr + i, a.planeR, P::czero());
      // projections of q_k on the rest of the panel
      Acc acc[BWM];
#pragma unroll
      for (int d = 0; d < BWM; ++d) {
        P::acc_zero(acc[d]);
        if (d > c && d < nb) {
#pragma unroll
          for (int r = 0; r < RP; ++r) P::acc_cmulc(acc[d], col[c][r], col[d][r]);
        }
      }
      if (c + 1 < nb) {
        block_reduce<P, BWM>(acc, c + 1, nb, lds, wave, lane, nwd);
#pragma unroll
        for (int d = 0; d < BWM; ++d) {
          if (d > c && d < nb) {
            C rk = P::acc_value(acc[d]);
            if (tid == 0) store_r<P>(a, k, k0 + d, rk);
#pragma unroll
            for (int r = 0; r < RP; ++r) P::upd(col[d][r], rk, col[c][r]);
          }
        }
      }
    }
  });
}

// --------------------------------------------------------- trailing role --
// A team of TW waves owns column j; lane holds rows
// i = (r*TW + tw_i)*64 + lane, r < RPT (rows beyond m zero).
template <class P, int RPT, int TW>
__device__ __forceinline__ void trailing_role(const StepArgs &a, int blk, typename P::Acc *lds, double *qs) {
  using C = typename P::C;
  using Acc = typename P::Acc;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  constexpr int TEAMS = NWAVE / TW;
  const int team = wave / TW, tw_i = wave % TW;
  const int kp0 = (a.t - 1) * a.bw;
  const int kp1 = min(kp0 + a.bw, a.n);
  const int jstart = min((a.t + 1) * a.bw, a.n);
  const int j = jstart + blk * TEAMS + team;
  const bool active = j < a.ncols;
  const bool first = a.t == 1;
  // team waves holding rows below m (rows (r TW + tw_i) 64 + lane)
  const int nwt = RPT > 1 ? TW : min(TW, (a.m + 63) / 64);

  C col[RPT];
  size_t ps = 0;
  const double *src = active ? col_src(a, j, first, ps) : nullptr;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    int i = (r * TW + tw_i) * 64 + lane;
    col[r] = (active && i < a.m) ? P::load(src + i, ps) : P::czero();
  }

#pragma unroll 1
  for (int kc = kp0; kc < kp1; kc += a.qstage) {
    const int cnt = min(a.qstage, kp1 - kc);
    lds_barrier();
    stage_q<P>(a, kc, cnt, qs);
    lds_barrier();
#pragma unroll 1
    for (int cc = 0; cc < cnt; ++cc) {
      const int k = kc + cc;
      const double *qk = qs + (size_t)cc * 2 * P::L * a.mpad;
      Acc acc;
      P::acc_zero(acc);
      if (active) {
#pragma unroll
        for (int r = 0; r < RPT; ++r)
          P::acc_cmulc(acc, P::load(qk + (r * TW + tw_i) * 64 + lane, (size_t)a.mpad), col[r]);
      }
      wave_reduce<P>(acc);
      if (TW > 1) {
        if (lane == 0) lds[wave] = acc;
        lds_barrier();
        acc = lds[team * TW];
#pragma unroll
        for (int w = 1; w < TW; ++w)
          if (w < nwt) P::acc_merge(acc, lds[team * TW + w]);
        lds_barrier();
      }
      if (active) {
        C rk = P::acc_value(acc);
        if (tw_i == 0 && lane == 0) store_r<P>(a, k, j, rk);
#pragma unroll
        for (int r = 0; r < RPT; ++r)
          P::upd(col[r], rk, P::load(qk + (r * TW + tw_i) * 64 + lane, (size_t)a.mpad));
      }
    }
  }

  if (active) {
    size_t pd;
    double *dst = col_dst(a, j, pd);
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      int i = (r * TW + tw_i) * 64 + lane;
      if (i < a.m) P::store(dst + i, pd, col[r]);
    }
  }
  // After the last panel: z of Equation (1), the norm of the projected b.
  if (a.t == a.npanel && a.rho != nullptr) {
    Acc acc;
    P::acc_zero(acc);
    if (active && j == a.n) {
#pragma unroll
      for (int r = 0; r < RPT; ++r) P::acc_abs2(acc, col[r]);
    }
    wave_reduce_re<P>(acc);
    if (TW > 1) {
      if (lane == 0) lds[wave] = acc;
      lds_barrier();
      acc = lds[team * TW];
#pragma unroll
      for (int w = 1; w < TW; ++w)
        if (w < nwt) P::acc_merge_re(acc, lds[team * TW + w]);
      lds_barrier();
    }
    if (active && j == a.n && tw_i == 0 && lane == 0) {
      typename P::R s = P::acc_value_re(acc);
      typename P::R z = P::ok_norm(s) ? P::sqrt_(s) : P::rzero();
      P::store_real(a.rho, 1, z);
    }
  }
}

template <class P, int RPT, int TW, int RP, int BWM>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(1, 1))) void mgs_step_kernel(StepArgs a) {
  __shared__ typename P::Acc lds[NWAVE * BWM];
  extern __shared__ double qs[];
  if (a.t < a.npanel) {
    if (blockIdx.x == 0)
      panel_role<P, RP, BWM>(a, lds, qs);
    else
      trailing_role<P, RPT, TW>(a, blockIdx.x - 1, lds, qs);
  } else {
    trailing_role<P, RPT, TW>(a, blockIdx.x, lds, qs);
  }
}

// ------------------------------------------------- back substitution -----
// Section 6, Figure 3: for k = n..1, x_k = y_k / r_kk, then y_j -= r_jk x_k
// for all j < k.  The reciprocals of the diagonal are formed in parallel up
// front.
// Blocked form of the same back substitution: one workgroup of BS_T
// threads, thread t holding y_j for j = s*BS_T + t.  The columns are taken
// in blocks [k0, k0 + B) from the bottom (B = 64, 32 in qd).  For each block:
//   1. its upper triangle of R is staged in LDS;
//   2. the one wave that holds rows k0 .. k0+B-1 solves the block:
//      x_k = y_k / r_kk (owner lane), x_k broadcast by readlane, then
//      y_j -= r_jk x_k for the block rows j < k;
//   3. every thread with a row j < k0 applies y_j -= r_jk x_k for the
//      block's k in descending order (R read from global, coalesced).
// Each y_j still receives r_jk x_k in the order k = n, n-1, ..., j+1 of
// Figure 3 with the same operations, so x is bitwise that of the
// column-oriented loop; the serial chain is B readlane steps per block
// instead of one block barrier per column.
constexpr int BS_T = 1024;
// Block width: 64 (one full wave; R block 128 KiB of LDS in dd), 32 in qd.
constexpr int bs_block(int L) { return L == 4 ? 32 : 64; }

template <class P>
__device__ __forceinline__ typename P::C bs_readlane(const typename P::C &v, int lane) {
  typename P::C r;
  double *pr = reinterpret_cast<double *>(&r);
  const double *pv = reinterpret_cast<const double *>(&v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(typename P::C) / sizeof(double)); ++i) {
    const long long b = __double_as_longlong(pv[i]);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    pr[i] = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
  return r;
}

template <class P, int NY>
__global__ __launch_bounds__(BS_T) void backsolve_blocked_kernel(int n, const double *R, int ldr, size_t planeR,
                                                                  const double *y, size_t planeY, double *x,
                                                                  int *info, const int *skip) {
  if (skip != nullptr && *skip != 0) return;
  using C = typename P::C;
  using Rl = typename P::R;
  constexpr int NP = 2 * P::L;  // planes of a complex element
  constexpr int BS_B = bs_block(P::L);
  __shared__ double rb[NP * BS_B * BS_B];  // block of R, planar [p][col][row]
  __shared__ double xs[NP * BS_B];         // x of the block, planar [p][k]
  __shared__ int bad;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (tid == 0) bad = 0x7fffffff;
  __syncthreads();
  C yv[NY];
  Rl inv[NY];
#pragma unroll
  for (int s = 0; s < NY; ++s) {
    const int j = s * BS_T + tid;
    if (j < n) {
      yv[s] = P::load(y + j, planeY);
      const C d = P::load(R + (size_t)j * ldr + j, planeR);
      if (!P::ok_norm(d.re)) atomicMin(&bad, j + 1);
      inv[s] = P::recip(d.re);
    } else {
      yv[s] = P::czero();
      inv[s] = P::rzero();
    }
  }
  __syncthreads();
  if (tid == 0 && info != nullptr) *info = (bad == 0x7fffffff) ? 0 : bad;
  const int nblk = (n + BS_B - 1) / BS_B;
#pragma unroll 1
  for (int kb = nblk - 1; kb >= 0; --kb) {
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
          for (int c = nb - 1; c >= 0; --c) {
            const C xl = P::scale(yv[s], inv[s]);
            const C xk = bs_readlane<P>(xl, l0 + c);
            if (i == c) {
              P::store(x + k0 + c, (size_t)n, xk);
              P::store(xs + c, (size_t)BS_B, xk);
            }
            if (i >= 0 && i < c) P::upd(yv[s], P::load(rb + c * BS_B + i, (size_t)BS_B * BS_B), xk);
          }
        }
      }
    }
    __syncthreads();
    // 3. Rows above the block, in the column order of Figure 3; the R
    // entries of BQ columns are loaded together (one memory latency per
    // BQ columns instead of per few).
#pragma unroll
    for (int s = 0; s < NY; ++s) {
      const int j = s * BS_T + tid;
      if (j < k0) {
        constexpr int BQ = (P::L == 4 ? 2 : 8) / NY > 0 ? (P::L == 4 ? 2 : 8) / NY : 1;
#pragma unroll 1
        for (int c0 = nb - 1; c0 >= 0; c0 -= BQ) {
          C rv[BQ];
#pragma unroll
          for (int t = 0; t < BQ; ++t)
            rv[t] = c0 - t >= 0 ? P::load(R + (size_t)(k0 + c0 - t) * ldr + j, planeR) : P::czero();
#pragma unroll
          for (int t = 0; t < BQ; ++t)
            if (c0 - t >= 0) P::upd(yv[s], rv[t], P::load(xs + c0 - t, (size_t)BS_B));
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------ projections y = Q^H b --------
// y_k = q_k^H b^(k-1), b^(k) = b^(k-1) - y_k q_k for k = 1..n: the same
// operations as the augmented column of Equation (1).  One block; b stays
// in registers (RB rows per thread).
template <class P, int RB>
__global__ __launch_bounds__(WG) void project_kernel(int m, int n, const double *Q, int ldq, size_t planeQ,
                                                      const double *b, double *y) {
  using C = typename P::C;
  using Acc = typename P::Acc;
  __shared__ Acc lds[NWAVE];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  C bv[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    int i = r * WG + tid;
    bv[r] = (i < m) ? P::load(b + i, (size_t)m) : P::czero();
  }
#pragma unroll 1
  for (int k = 0; k < n; ++k) {
    const double *qk = Q + (size_t)k * ldq;
    C q[RB];
    Acc acc;
    P::acc_zero(acc);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int i = r * WG + tid;
      q[r] = (i < m) ? P::load(qk + i, planeQ) : P::czero();
      P::acc_cmulc(acc, q[r], bv[r]);
    }
    wave_reduce<P>(acc);
    if (lane == 0) lds[wave] = acc;
    __syncthreads();
    acc = lds[0];
#pragma unroll
    for (int w = 1; w < NWAVE; ++w) P::acc_merge(acc, lds[w]);
    __syncthreads();
    C yk = P::acc_value(acc);
    if (tid == 0) P::store(y + k, (size_t)n, yk);
#pragma unroll
    for (int r = 0; r < RB; ++r) P::upd(bv[r], yk, q[r]);
  }
}

}  // namespace mgsq
