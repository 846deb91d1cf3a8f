// C ABI of the MGS least-squares library (declared in include/mgsqr.h):
// argument checks, launch-shape selection and kernel launches.  No
// allocation, no host<->device copies, no synchronisation.
#include "../../include/mgsqr.h"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <atomic>
#include <mutex>

#include "adjoint_kernels.hpp"
#include "backsolve_kernels.hpp"
#include "batched_kernels.hpp"
#include "mgs_kernels.hpp"
#include "newton_kernels.hpp"
#include "precision_kernels.hpp"
#include "resident_kernels.hpp"
#include "small_kernels.hpp"

using namespace mgsq;

// Workspace of mgs_qr_noalloc: a fixed device array, one copy per GPU the
// code object is loaded on, held until the process ends.  Host code never
// uses this name as an address (it denotes a host-side stand-in): the
// device address comes from hipGetSymbolAddress (scratch_address below).
static_assert(MGS_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
static __device__ __align__(256) unsigned char scratch[MGS_NOALLOC_SCRATCH_BYTES];

namespace {

bool aligned8(const void *p) { return p != nullptr && (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }
size_t round256(size_t b) { return (b + 255) & ~size_t(255); }
int max_rows(int prec) { return prec == 4 ? MGS_MAX_ROWS_QD : MGS_MAX_ROWS_DD; }
bool prec_ok(int prec) { return prec == 1 || prec == 2 || prec == 4; }
int pow2_at_least(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}
int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Launch shape of one factorisation (rows padded to the shape, zeros beyond m):
//   trailing role: a team of TW waves per column, RPT rows per lane
//     (RPT a power of two, at most 16 for dd and 8 for qd, so that the
//     column stays in registers);
//   panel role: RP = RPT*TW/4 rows per thread (at least 1) over the block's
//     256 threads, panel width BWM = elements-per-thread budget / RP.
struct Shape {
  int tw, rpt, rp;
};
Shape choose_shape(int m, int prec, int ncols = 0) {
  const int rpt_max = prec == 1 ? 32 : (prec == 2 ? 16 : 8);
  Shape s;
  s.tw = pow2_at_least(ceil_div(m, 64 * rpt_max));
  // qd with few columns: up to 4 waves per trailing column, so that the
  // trailing columns of a launch give about 1024 waves (4 per compute unit)
  // and each wave's share of a projection stays short.
  if (prec == 4)
    while (s.tw < 4 && ncols * s.tw < 1024) s.tw *= 2;
  s.rpt = pow2_at_least(ceil_div(m, 64 * s.tw));
  s.rp = s.rpt * s.tw / NWAVE > 1 ? s.rpt * s.tw / NWAVE : 1;
  return s;
}
constexpr int bw_for(int L, int RP) {
  // complex elements per thread held by the panel role: FP64 16, dd 8;
  // the panel width is capped (FP64 / dd 4) so that its loops unroll fully
  // and every register array keeps static indices.  qd: one column per
  // panel (the panel role's qd arithmetic is the serial part of each
  // launch, and its look-ahead work grows with the square of the width).
  return L == 1 ? (16 / RP >= 4 ? 4 : (16 / RP >= 1 ? 16 / RP : 1))
                : L == 2 ? (8 / RP >= 4 ? 4 : (8 / RP >= 1 ? 8 / RP : 1))
                         : 1;
}

// LDS budget for staged q vectors (gfx950: 160 KiB per CU).
constexpr size_t QSTAGE_BYTES = 128 * 1024;

template <class P, int RPT, int TW>
int launch_steps(StepArgs a, hipStream_t st) {
  constexpr int RP = RPT * TW / NWAVE > 1 ? RPT * TW / NWAVE : 1;
  constexpr int BWM = bw_for(P::L, RP);
  constexpr int TEAMS = NWAVE / TW;
  a.bw = BWM;
  a.npanel = ceil_div(a.n, a.bw);
  a.mpad = RPT * 64 * TW > RP * WG ? RPT * 64 * TW : RP * WG;
  const size_t qbytes = sizeof(double) * 2 * P::L * (size_t)a.mpad;
  a.qstage = (int)(QSTAGE_BYTES / qbytes);
  if (a.qstage > a.bw) a.qstage = a.bw;
  if (a.qstage < 1) return MGS_ERR_DIMS;
  const size_t shmem = qbytes * a.qstage;
  auto kern = mgs_step_kernel<P, RPT, TW, RP, BWM>;
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)shmem) != hipSuccess)
    return MGS_ERR_LAUNCH;
  const int last = a.ncols > a.n ? a.npanel : a.npanel - 1;
  for (int t = 0; t <= last; ++t) {
    a.t = t;
    const int jstart = (t + 1) * a.bw < a.n ? (t + 1) * a.bw : a.n;
    const int ntrail = t >= 1 ? a.ncols - jstart : 0;
    const int tblocks = ntrail > 0 ? ceil_div(ntrail, TEAMS) : 0;
    const int grid = (t < a.npanel ? 1 : 0) + tblocks;
    if (grid == 0) continue;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(WG), shmem, st, a);
    if (hipGetLastError() != hipSuccess) return MGS_ERR_LAUNCH;
  }
  return MGS_OK;
}

template <class P>
int dispatch_shape(const StepArgs &a, const Shape &sh, hipStream_t st) {
  if constexpr (P::L == 1) {
    if (sh.tw == 1) {
      switch (sh.rpt) {
        case 1: return launch_steps<P, 1, 1>(a, st);
        case 2: return launch_steps<P, 2, 1>(a, st);
        case 4: return launch_steps<P, 4, 1>(a, st);
        case 8: return launch_steps<P, 8, 1>(a, st);
        case 16: return launch_steps<P, 16, 1>(a, st);
        case 32: return launch_steps<P, 32, 1>(a, st);
      }
    } else if (sh.rpt == 32 && sh.tw == 2) {
      return launch_steps<P, 32, 2>(a, st);
    }
  } else if constexpr (P::L == 2) {
    if (sh.tw == 1) {
      switch (sh.rpt) {
        case 1: return launch_steps<P, 1, 1>(a, st);
        case 2: return launch_steps<P, 2, 1>(a, st);
        case 4: return launch_steps<P, 4, 1>(a, st);
        case 8: return launch_steps<P, 8, 1>(a, st);
        case 16: return launch_steps<P, 16, 1>(a, st);
      }
    } else if (sh.rpt == 16 && sh.tw == 2) {
      return launch_steps<P, 16, 2>(a, st);
    } else if (sh.rpt == 16 && sh.tw == 4) {
      return launch_steps<P, 16, 4>(a, st);
    }
  } else {
    if (sh.tw == 1) {
      switch (sh.rpt) {
        case 1: return launch_steps<P, 1, 1>(a, st);
        case 2: return launch_steps<P, 2, 1>(a, st);
        case 4: return launch_steps<P, 4, 1>(a, st);
        case 8: return launch_steps<P, 8, 1>(a, st);
      }
    } else if (sh.rpt == 8 && sh.tw == 2) {
      return launch_steps<P, 8, 2>(a, st);
    } else if (sh.tw == 4) {
      switch (sh.rpt) {
        case 1: return launch_steps<P, 1, 4>(a, st);
        case 2: return launch_steps<P, 2, 4>(a, st);
        case 4: return launch_steps<P, 4, 4>(a, st);
        case 8: return launch_steps<P, 8, 4>(a, st);
      }
    }
  }
  return MGS_ERR_DIMS;
}

#ifdef MGS_TRACE
// Diagnostic builds: stamps of the back substitution across workgroups
// (4 per workgroup), set by mgs_set_trace_backsolve.
long long *g_trace_bs = nullptr;
#endif

struct DevInfo {
  int cus;  // compute units when cooperative launches are supported, else 0
  long long wclk_khz;
};
bool dev_info(DevInfo &d);

// Race checks: the timing-jitter seed handed to the kernels that
// synchronise across waves or workgroups (mgs_set_jitter; 0: none).
std::atomic<unsigned> g_jitter{0};

// Back substitution across workgroups (one wave per 64 rows, cooperative);
// returns 1 when it does not apply (one block only, or the workgroups
// cannot all be resident), so that the caller takes the one-workgroup
// kernel.
template <class P, bool FWD = false>
int backsolve_pipe_launch(int n, const double *R, int ldr, size_t planeR, const double *y, size_t planeY, double *x,
                          int *info, const int *skip, hipStream_t st) {
  if (n <= BP_ROWS) return 1;
  DevInfo d;
  if (!dev_info(d) || d.cus <= 0) return 1;
  const int G = ceil_div(n, BP_ROWS);
  auto kern = trsv_pipe_kernel<P, FWD>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kern), BP_ROWS, 0) !=
          hipSuccess ||
      (long long)per_cu * d.cus < G)
    return 1;
  hipLaunchKernelGGL((bs_mark_kernel<P::L>), dim3(ceil_div(n, 256)), dim3(256), 0, st, n, x, info, skip);
  if (hipGetLastError() != hipSuccess) return MGS_ERR_LAUNCH;
  long long spin = d.wclk_khz * 2000;  // 2 s
#ifdef MGS_TRACE
  long long *trace = g_trace_bs;
#else
  long long *trace = nullptr;
#endif
  unsigned jitter = g_jitter.load(std::memory_order_relaxed);
  void *args[] = {&n, &R, &ldr, &planeR, &y, &planeY, &x, &info, &skip, &spin, &trace, &jitter};
  if (hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3(G), dim3(BP_ROWS), args, 0, st) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return MGS_OK;
}

template <class P>
int backsolve_launch(int n, const double *R, int ldr, const double *y, double *x, int *info, hipStream_t st,
                     size_t planeR = 0, const int *skip = nullptr, size_t planeY = 0) {
  const int ny = pow2_at_least(ceil_div(n, BS_T));
  if (planeR == 0) planeR = (size_t)ldr * n;
  if (planeY == 0) planeY = (size_t)n;
  const int rc = backsolve_pipe_launch<P>(n, R, ldr, planeR, y, planeY, x, info, skip, st);
  if (rc != 1) return rc;
#define MGS_NY_CASE(NYV)                                                                                    \
  case NYV:                                                                                                 \
    hipLaunchKernelGGL((backsolve_blocked_kernel<P, NYV>), dim3(1), dim3(BS_T), 0, st, n, R, ldr, planeR, y, \
                       planeY, x, info, skip);                                                              \
    break;
  switch (ny) {
    MGS_NY_CASE(1)
    MGS_NY_CASE(2)
    MGS_NY_CASE(4)
    default:
      return MGS_ERR_DIMS;
  }
#undef MGS_NY_CASE
  return hipGetLastError() == hipSuccess ? MGS_OK : MGS_ERR_LAUNCH;
}

template <class P>
int project_launch(int m, int n, const double *Q, int ldq, const double *b, double *y, hipStream_t st) {
  const int rb = pow2_at_least(ceil_div(m, WG));
  const size_t planeQ = (size_t)ldq * n;
#define MGS_RB_CASE(RBV)                                                                                     \
  case RBV:                                                                                                  \
    hipLaunchKernelGGL((project_kernel<P, RBV>), dim3(1), dim3(WG), 0, st, m, n, Q, ldq, planeQ, b, y);       \
    break;
  switch (rb) {
    MGS_RB_CASE(1)
    MGS_RB_CASE(2)
    MGS_RB_CASE(4)
    MGS_RB_CASE(8)
    MGS_RB_CASE(16)
    default:
      return MGS_ERR_DIMS;
  }
#undef MGS_RB_CASE
  return hipGetLastError() == hipSuccess ? MGS_OK : MGS_ERR_LAUNCH;
}

// QR: working copy of b (2Lm doubles), then the synchronisation words of
// the single-launch schedule, then (the shapes that can take it: dd with
// m <= 1024, FP64 with m <= 2048 and at most 32 MiB) its hand-off copy of
// the n columns (2Lmn doubles).
size_t qr_w_bytes(int m, int prec) { return round256(sizeof(double) * 2 * (size_t)prec * m); }
bool res_rows_ok(int m, int prec) { return (prec == 2 && m <= 1024) || (prec == 1 && m <= 2048); }
size_t qr_u_bytes(int m, int n, int prec) {
  const size_t u = round256(sizeof(double) * 2 * (size_t)prec * m * n);
  return (res_rows_ok(m, prec) && u <= ((size_t)32 << 20)) ? u : 0;
}
size_t qr_work_bytes(int m, int n, int prec) {
  return qr_w_bytes(m, prec) + sizeof(unsigned int) * RES_SYNC_WORDS + qr_u_bytes(m, n, prec);
}
size_t solve_work_bytes(int n, int prec) { return round256(sizeof(double) * 2 * (size_t)prec * n); }
// adjoint: w (n), z (n), r (m), then the chunk partials of Q w and b - A x
// (2 x chunks x m accumulators).
size_t adj_acc_bytes(int prec) { return prec == 1 ? sizeof(PrecD::Acc) : prec == 2 ? sizeof(PrecDD::Acc) : sizeof(PrecQD::Acc); }
size_t adjoint_work_bytes(int m, int n, int prec) {
  const size_t nchunk = (size_t)((n + ADJ_CH - 1) / ADJ_CH);
  return 2 * round256(sizeof(double) * 2 * (size_t)prec * n) + round256(sizeof(double) * 2 * (size_t)prec * m) +
         round256(adj_acc_bytes(prec) * 2 * nchunk * m);
}

template <class P>
int fwdsub_launch(int n, const double *R, int ldr, const double *g, double *w, int *info, hipStream_t st) {
  const int ny = pow2_at_least(ceil_div(n, BS_T));
  const size_t planeR = (size_t)ldr * n;
  const int rc = backsolve_pipe_launch<P, true>(n, R, ldr, planeR, g, (size_t)n, w, info, nullptr, st);
  if (rc != 1) return rc;
#define MGS_FS_CASE(NYV)                                                                                       \
  case NYV:                                                                                                    \
    hipLaunchKernelGGL((fwdsub_blocked_kernel<P, NYV>), dim3(1), dim3(BS_T), 0, st, n, R, ldr, planeR, g, w, info); \
    break;
  switch (ny) {
    MGS_FS_CASE(1)
    MGS_FS_CASE(2)
    MGS_FS_CASE(4)
    default:
      return MGS_ERR_DIMS;
  }
#undef MGS_FS_CASE
  return hipGetLastError() == hipSuccess ? MGS_OK : MGS_ERR_LAUNCH;
}

template <class P>
int adjoint_launch(int m, int n, const double *A, int lda, const double *b, const double *Q, int ldq,
                   const double *R, int ldr, const double *x, const double *gx, double *gA, int ldga, double *gb,
                   void *work, int *info, hipStream_t st) {
  double *w = static_cast<double *>(work);
  double *z = w + round256(sizeof(double) * 2 * P::L * (size_t)n) / sizeof(double);
  double *r = z + round256(sizeof(double) * 2 * P::L * (size_t)n) / sizeof(double);
  auto *part = reinterpret_cast<typename P::Acc *>(r + round256(sizeof(double) * 2 * P::L * (size_t)m) / sizeof(double));
  int rc = fwdsub_launch<P>(n, R, ldr, gx, w, info, st);
  if (rc != MGS_OK) return rc;
  rc = backsolve_launch<P>(n, R, ldr, w, z, info, st);
  if (rc != MGS_OK) return rc;
  hipLaunchKernelGGL((adj_partial_kernel<P>), dim3(ceil_div(m, ADJ_T), ceil_div(n, ADJ_CH), 2), dim3(ADJ_T), 0, st,
                     m, n, Q, ldq, (size_t)ldq * n, A, lda, (size_t)lda * n, b, x, w, part);
  if (hipGetLastError() != hipSuccess) return MGS_ERR_LAUNCH;
  hipLaunchKernelGGL((adj_finish_kernel<P>), dim3(ceil_div(m, WG), 2), dim3(WG), 0, st, m, n, part, gb, r);
  if (hipGetLastError() != hipSuccess) return MGS_ERR_LAUNCH;
  hipLaunchKernelGGL((adj_rank2_kernel<P>), dim3(ceil_div(m, WG), n), dim3(WG), 0, st, m, n, r, z, gb, x, gA, ldga,
                     (size_t)ldga * n);
  return hipGetLastError() == hipSuccess ? MGS_OK : MGS_ERR_LAUNCH;
}

// ------------------------------------------------------ precision form --
struct RefineWork {
  double *Q64, *R64, *y64, *d64, *r64;
  void *partial;
  RefineCtl *ctl;
  void *res;  // the FP64 panels' single launch: synchronisation words, then U (nullptr: none)
  size_t bytes;
};
// Synchronisation words and hand-off copy U of one FP64 panel (m x NBP)
// for the single-launch panel factorisation (m <= 2048), else nothing.
size_t panel_res_bytes(int m, int n) {
  if (m > 2048) return 0;
  const int nb = n < NBP ? n : NBP;
  return round256(sizeof(unsigned int) * RES_SYNC_WORDS) + round256(sizeof(double) * 2 * (size_t)m * nb);
}
RefineWork refine_layout(int m, int n, int prec, void *base) {
  const int nchunk = ceil_div(n, NBP);
  const size_t acc_bytes = sizeof(PrecQD::Acc);  // the residual accumulates in qd
  (void)prec;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off += round256(b);
    return static_cast<char *>(base) + o;
  };
  RefineWork w;
  w.Q64 = reinterpret_cast<double *>(take(sizeof(double) * 2 * (size_t)m * (n + 1)));
  w.R64 = reinterpret_cast<double *>(take(sizeof(double) * 2 * (size_t)n * (n + 1)));
  w.y64 = reinterpret_cast<double *>(take(sizeof(double) * 2 * (size_t)n));
  w.d64 = reinterpret_cast<double *>(take(sizeof(double) * 2 * (size_t)n));
  w.r64 = reinterpret_cast<double *>(take(sizeof(double) * 2 * (size_t)m));
  w.partial = take(acc_bytes * (size_t)nchunk * m);
  w.ctl = reinterpret_cast<RefineCtl *>(take(sizeof(RefineCtl)));
  w.res = panel_res_bytes(m, n) > 0 ? take(panel_res_bytes(m, n)) : nullptr;
  w.bytes = off;
  return w;
}

// mgs_qr64: Q64 (m x (n+1)) and R64 (n x (n+1)), FP64 complex, then the
// panel factorisation's single-launch area.
size_t qr64_work_bytes(int m, int n) {
  return round256(sizeof(double) * 2 * (size_t)m * (n + 1)) + round256(sizeof(double) * 2 * (size_t)n * (n + 1)) +
         panel_res_bytes(m, n);
}

template <class P>
int res_launch(const StepArgs &s, void *sync, double *u, hipStream_t st);

// FP64 blocked MGS of [A64 b64] held in Q64 (m x (n+1)); R64 (n x (n+1))
// receives R and, in its last column, y.
int factor64(int m, int n, const RefineWork &w, int *info, hipStream_t st) {
  const size_t planeQ = (size_t)m * (n + 1), planeR = (size_t)n * (n + 1);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(256), dim3(256), 0, st, w.R64, 2 * planeR);
  const Shape sh = choose_shape(m, 1);
  for (int k0 = 0; k0 < n; k0 += NBP) {
    const int nb = n - k0 < NBP ? n - k0 : NBP;
    StepArgs a;
    a.m = m;
    a.n = nb;
    a.ncols = nb;
    a.A = w.Q64 + (size_t)k0 * m;
    a.lda = m;
    a.planeA = planeQ;
    a.b = nullptr;
    a.Q = w.Q64 + (size_t)k0 * m;
    a.ldq = m;
    a.planeQ = planeQ;
    a.R = w.R64 + (size_t)k0 * n + k0;
    a.ldr = n;
    a.planeR = planeR;
    a.W = nullptr;
    a.y = nullptr;
    a.rho = nullptr;
    a.info = info;
    a.t = 0;
    a.kbase = k0;
    a.init_info = 0;
    // The panel in one cooperative launch when it fits, else one launch
    // per column pair.
    int rc = 1;
    if (w.res != nullptr) {
      double *u = reinterpret_cast<double *>(static_cast<char *>(w.res) +
                                             round256(sizeof(unsigned int) * RES_SYNC_WORDS));
      rc = res_launch<PrecD>(a, w.res, u, st);
    }
    if (rc == 1) rc = dispatch_shape<PrecD>(a, sh, st);
    if (rc != MGS_OK) return rc;
    const int N = n + 1 - (k0 + nb);  // trailing columns, b included
    if (N > 0) {
      const double *Qp = w.Q64 + (size_t)k0 * m;
      double *At = w.Q64 + (size_t)(k0 + nb) * m;
      double *Wb = w.R64 + (size_t)(k0 + nb) * n + k0;
      hipLaunchKernelGGL(zgemm_qha_kernel, dim3(ceil_div(N, 16), ceil_div(nb, 16)), dim3(64 * QHA_SLICES), 0, st, m, N,
                         nb, Qp, m, At, m, planeQ, Wb, n, planeR);
      const int tiles = ceil_div(m, 16) * ceil_div(N, 16);
      hipLaunchKernelGGL(zgemm_update_kernel, dim3(ceil_div(tiles, 4)), dim3(256), 0, st, m, N, nb, Qp, m, At, m,
                         planeQ, Wb, n, planeR);
    }
    if (hipGetLastError() != hipSuccess) return MGS_ERR_LAUNCH;
  }
  return MGS_OK;
}

template <class P>
int refine_solve(int m, int n, const double *A, int lda, const double *b, double *x, double tol, int max_iter,
                 int *iters, double *err_est, void *work, int *info, hipStream_t st) {
  RefineWork w = refine_layout(m, n, P::L, work);
  const size_t planeQ = (size_t)m * (n + 1), planeR = (size_t)n * (n + 1);
  hipLaunchKernelGGL((copy_hi_kernel<P::L>), dim3(ceil_div(m, 256), n + 1), dim3(256), 0, st, m, n, A, lda, b, w.Q64,
                     w.ctl, info);
  int rc = factor64(m, n, w, info, st);
  if (rc != MGS_OK) return rc;
  hipLaunchKernelGGL(refine_check_kernel, dim3(1), dim3(64), 0, st, info, w.ctl);
  const int *skip = &w.ctl->status;
  // x0: R x0 = y (the last column of R64)
  rc = backsolve_launch<PrecD>(n, w.R64, n, w.R64 + (size_t)n * n, w.d64, nullptr, st, planeR, skip, planeR);
  if (rc != MGS_OK) return rc;
  hipLaunchKernelGGL((set_x_kernel<P>), dim3(ceil_div(n, 256)), dim3(256), 0, st, n, w.d64, x);
  const int nchunk = ceil_div(n, NBP);
  // The correction's panel projections: one cooperative launch per step
  // (proj_replay_kernel) when it can run, else two launches per panel.  The
  // launches of a converged solve return at once, so the fixed max_iter
  // steps cost little past convergence.
  DevInfo d;
  // (the barrier count of all steps must fit the 32-bit counter)
  bool fused = m <= PR_MAX_ROWS && (long long)max_iter * 2 * nchunk * NBP < (1LL << 31) && dev_info(d) &&
               d.cus >= NBP;
  const long long spin = fused ? (long long)d.wclk_khz * 2000 : 0;  // 2 s
  const unsigned jitter = g_jitter.load(std::memory_order_relaxed);
  for (int it = 1; it <= max_iter; ++it) {
    hipLaunchKernelGGL((residual_partial_kernel<P::L>), dim3(ceil_div(m, 256), nchunk), dim3(256), 0, st, m, n, NBP,
                       A, lda, b, x, static_cast<PrecQD::Acc *>(w.partial), w.ctl);
    hipLaunchKernelGGL((residual_finish_kernel<PrecQD>), dim3(ceil_div(m, 256)), dim3(256), 0, st, m, nchunk,
                       static_cast<const PrecQD::Acc *>(w.partial), w.r64, w.ctl);
    if (fused) {
      // arrivals at the grid barriers of the earlier steps (2 per panel, G each)
      unsigned int base = (unsigned int)(it - 1) * 2u * (unsigned int)nchunk * (unsigned int)NBP;
      const double *Qa = w.Q64;
      size_t pq = planeQ, pw = (size_t)n;
      double *ra = w.r64, *wa = w.y64;
      RefineCtl *ctl = w.ctl;
      int mm = m, nn = n;
      long long sp = spin;
      unsigned jt = jitter;
      void *args[] = {&mm, &nn, &Qa, &pq, &ra, &wa, &pw, &ctl, &info, &base, &sp, &jt};
      if (hipLaunchCooperativeKernel(reinterpret_cast<const void *>(proj_replay_kernel), dim3(NBP), dim3(256), args, 0,
                                     st) != hipSuccess) {
        (void)hipGetLastError();
        fused = false;  // the barrier count is off from here: per-panel launches for the rest
      }
    }
    if (!fused) {
      for (int k0 = 0; k0 < n; k0 += NBP) {
        const int nb = n - k0 < NBP ? n - k0 : NBP;
        const double *Qp = w.Q64 + (size_t)k0 * m;
        hipLaunchKernelGGL(proj_w_kernel, dim3(nb), dim3(256), 0, st, m, Qp, m, planeQ, w.r64, w.y64 + k0, (size_t)n,
                           w.ctl);
        hipLaunchKernelGGL(proj_r_kernel, dim3(ceil_div(m, 256)), dim3(256), 0, st, m, nb, Qp, m, planeQ, w.y64 + k0,
                           (size_t)n, w.r64, w.ctl);
      }
    }
    rc = backsolve_launch<PrecD>(n, w.R64, n, w.y64, w.d64, nullptr, st, planeR, skip);
    if (rc != MGS_OK) return rc;
    hipLaunchKernelGGL((refine_update_kernel<P>), dim3(1), dim3(256), 0, st, n, w.d64, x, tol, it, w.ctl);
    if (hipGetLastError() != hipSuccess) return MGS_ERR_LAUNCH;
  }
  hipLaunchKernelGGL(refine_finish_kernel, dim3(1), dim3(64), 0, st, w.ctl, iters, err_est, info);
  return hipGetLastError() == hipSuccess ? MGS_OK : MGS_ERR_LAUNCH;
}

// ------------------------------------------- single-launch schedule --------
bool dev_info(DevInfo &d) {
  static DevInfo cache[64];
  static bool have[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
  if (!have[dev]) {
    int cus = 0, wclk = 0, coop = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&wclk, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess) return false;
    cache[dev].cus = coop ? cus : 0;
    cache[dev].wclk_khz = wclk > 0 ? wclk : 100000;
    have[dev] = true;
  }
  d = cache[dev];
  return true;
}

// Columns held by the workgroup holding the most, for panels of bw columns
// dealt in the reflected cyclic order of the resident kernel.
int res_max_cols(int ncols, int bw, int G) {
  const int np = ceil_div(ncols, bw);
  int best = 0;
  for (int g = 0; g < G; ++g) {
    int cnt = 0;
    for (int i = 0;; ++i) {
      const int qi = res_position(i, g, G);
      if (qi >= np) break;
      const int p = np - 1 - qi;
      cnt += (ncols - p * bw < bw) ? ncols - p * bw : bw;
    }
    if (cnt > best) best = cnt;
  }
  return best;
}

// Resident shapes (dd): workgroups of nw waves (up to 8, 2 per SIMD), RR
// rows per thread, CB column slots per workgroup (register budget 256 per
// lane).  Short columns take fewer waves (64 nw >= m), so that their block
// sums have fewer levels and their barriers fewer waves.
constexpr int RES_NW = 8;
// Column slots: 80 registers of columns per lane (dd: RR x CB <= 10 of 8
// registers; FP64: RR x CB <= 20 of 4), at most 8 slots.
constexpr int res_cb(int L, int rr) { return L == 2 ? (rr == 1 ? 8 : 5) : (rr <= 2 ? 8 : 5); }

struct ResPlan {
  int rr, nw, bw, np, G;
};
bool res_choose(int m, int ncols, int L, int cus, ResPlan &pl) {
  const int rr = pow2_at_least(ceil_div(m, 64 * RES_NW));
  if (rr > (L == 1 ? 4 : 2)) return false;
  int nw = RES_NW;
  if (rr == 1) {
    nw = pow2_at_least(ceil_div(m, 64));
    if (nw > RES_NW) nw = RES_NW;
  }
  const int cb = res_cb(L, rr);
  // Panels of one column: the look-ahead hand-off of the kernel assumes it.
  const int bws[1] = {1};
  for (int bw : bws) {
    const int np = ceil_div(ncols, bw);
    const int G = np < cus ? np : cus;
    if (res_max_cols(ncols, bw, G) <= cb) {
      pl.rr = rr;
      pl.nw = nw;
      pl.bw = bw;
      pl.np = np;
      pl.G = G;
      return true;
    }
  }
  return false;
}

#ifdef MGS_TRACE
// Diagnostic builds: device buffer of RES_TRACE_SLOTS stamps per column for
// the next single-launch factorisations (mgs_set_trace).
long long *g_trace = nullptr;
#endif

// Returns 1 when the single launch does not apply here (the caller then
// takes the per-panel schedule).
template <class P, int RR, int NW>
int res_launch_rr(ResArgs a, int cus, hipStream_t st) {
  constexpr int CB = res_cb(P::L, RR);
  auto kern = mgs_resident_kernel<P, RR, CB, NW>;
  // Only kernels that keep everything in registers and LDS take this
  // schedule: no private (scratch) memory in a cooperative launch.
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kern)) != hipSuccess || fa.localSizeBytes != 0)
    return 1;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kern), 64 * NW, 0) !=
      hipSuccess)
    return 1;
  if ((long long)per_cu * cus < a.G) return 1;
  hipLaunchKernelGGL(resident_init_kernel, dim3(1), dim3(RES_SYNC_WORDS), 0, st, a.sync, a.info, a.init_info);
  if (hipGetLastError() != hipSuccess) return MGS_ERR_LAUNCH;
  void *args[] = {&a};
  if (hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3(a.G), dim3(64 * NW), args, 0, st) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return MGS_OK;
}

// FP64 and dd only: the qd instantiations do not fit in registers.
template <class P>
int res_launch(const StepArgs &s, void *sync, double *u, hipStream_t st) {
  static_assert(P::L <= 2, "no qd instantiation of the single launch");
  DevInfo d;
  if (!dev_info(d) || d.cus <= 0) return 1;
  ResPlan pl;
  if (!res_choose(s.m, s.ncols, P::L, d.cus, pl)) return 1;
  ResArgs a;
  a.m = s.m;
  a.n = s.n;
  a.ncols = s.ncols;
  a.A = s.A;
  a.lda = s.lda;
  a.planeA = s.planeA;
  a.b = s.b;
  a.Q = s.Q;
  a.ldq = s.ldq;
  a.planeQ = s.planeQ;
  a.R = s.R;
  a.ldr = s.ldr;
  a.planeR = s.planeR;
  a.y = s.y;
  a.rho = s.rho;
  a.info = s.info;
  a.sync = static_cast<unsigned int *>(sync);
  a.U = u;
  a.ldu = s.m;
  a.planeU = (size_t)s.m * s.n;
  a.bw = pl.bw;
  a.np = pl.np;
  a.G = pl.G;
  a.xcd_group = pl.G % 8 == 0 ? pl.G / 8 : 0;
  a.defer = 12;
  a.spin_ticks = d.wclk_khz * 2000;  // 2 s
  a.kbase = s.kbase;
  a.init_info = s.init_info;
  a.jitter = g_jitter.load(std::memory_order_relaxed);
#ifdef MGS_TRACE
  a.trace = g_trace;
#endif
  if constexpr (P::L == 1) {
    if (pl.rr == 4) return res_launch_rr<P, 4, 8>(a, d.cus, st);
  }
  if (pl.rr == 2) return res_launch_rr<P, 2, 8>(a, d.cus, st);
  switch (pl.nw) {
    case 1: return res_launch_rr<P, 1, 1>(a, d.cus, st);
    case 2: return res_launch_rr<P, 1, 2>(a, d.cus, st);
    case 4: return res_launch_rr<P, 1, 4>(a, d.cus, st);
    case 8: return res_launch_rr<P, 1, 8>(a, d.cus, st);
  }
  return 1;
}

// dd systems of at most SMALL_MAX_ROWS rows and SMALL_MAX_COLS columns of
// [A b]: one workgroup (returns 1 when the shape does not apply).
int small_launch_dd(const StepArgs &s, hipStream_t st) {
  if (s.m > SMALL_MAX_ROWS || s.ncols > SMALL_MAX_COLS) return 1;
  DevInfo d;
  if (!dev_info(d)) return 1;
  SmallArgs a;
  a.m = s.m;
  a.n = s.n;
  a.ncols = s.ncols;
  a.A = s.A;
  a.lda = s.lda;
  a.planeA = s.planeA;
  a.b = s.b;
  a.Q = s.Q;
  a.ldq = s.ldq;
  a.planeQ = s.planeQ;
  a.R = s.R;
  a.ldr = s.ldr;
  a.planeR = s.planeR;
  a.y = s.y;
  a.rho = s.rho;
  a.info = s.info;
  a.spin_ticks = d.wclk_khz * 2000;  // 2 s
  a.jitter = g_jitter.load(std::memory_order_relaxed);
  hipLaunchKernelGGL(mgs_small_kernel, dim3(1), dim3(64 * SMALL_WAVES), 0, st, a);
  return hipGetLastError() == hipSuccess ? MGS_OK : MGS_ERR_LAUNCH;
}

// Batched systems: one workgroup per system (returns MGS_ERR_DIMS when one
// system's q vectors do not fit in LDS).  Waves per system: 4 (FP64), 8
// (dd), 16 (qd), so that a slot of every wave holds a column in registers
// and several systems share a compute unit.
template <class P, int NW, int CPW>
int batched_launch(const BatArgs &a, hipStream_t st) {
  static_assert(NW * CPW <= BAT_MAX_COLS, "slots beyond the flags");
  if (a.ncols > NW * CPW) return MGS_ERR_DIMS;  // every column of [A b] needs a slot
  const size_t shmem = sizeof(double) * 2 * P::L * (size_t)a.n * a.m;
  if (shmem > BAT_LDS_BYTES) return MGS_ERR_DIMS;
  if (a.batch == 0) return MGS_OK;
  auto kern = mgs_batched_kernel<P, NW, CPW>;
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)shmem) != hipSuccess)
    return MGS_ERR_LAUNCH;
  hipLaunchKernelGGL(kern, dim3(a.batch), dim3(64 * NW), shmem, st, a);
  return hipGetLastError() == hipSuccess ? MGS_OK : MGS_ERR_LAUNCH;
}
int batched_dispatch(int prec, const BatArgs &a, hipStream_t st) {
  if (prec == 1) {
    if (a.ncols <= 36) return batched_launch<PrecD, 12, 3>(a, st);
    return batched_launch<PrecD, 16, 4>(a, st);
  }
  if (prec == 2) {
    if (a.ncols <= 36) return batched_launch<PrecDD, 12, 3>(a, st);
    return batched_launch<PrecDD, 16, 4>(a, st);
  }
  // qd: 16 waves of 4 slots cap a wave at 128 registers (four waves per
  // SIMD), which spills; up to 36 columns, 12 waves of 3 slots (three
  // waves per SIMD, 168 registers)
  if (a.ncols <= 36) return batched_launch<PrecQD, 12, 3>(a, st);
  return batched_launch<PrecQD, 16, 4>(a, st);
}
bool batched_fits(int m, int n, int ncols, int prec) {
  return m <= BAT_MAX_ROWS && ncols <= BAT_MAX_COLS && sizeof(double) * 2 * prec * (size_t)n * m <= BAT_LDS_BYTES;
}

// ------------------------------------------------ allocation-free QR ----
// mgs_qr_noalloc keeps its workspace in `scratch` instead of a
// caller-supplied buffer; kernels get the device address from
// hipGetSymbolAddress, taken once per device with that device current.

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES];

// The current device's address of `scratch` (nullptr on failure).
void *scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Newton: J (batch systems of neq x nvar), b (batch x neq), R (batch x
// nvar x nvar), d (batch x nvar), each in the working precision; for one
// point in dd or qd also y (nvar), an int and the workspace of mgs_qr.
struct NewtonWork {
  double *A, *b, *R, *d, *y;
  int *info2;
  void *qrw;
  size_t qrw_bytes;
  size_t bytes;
};
NewtonWork newton_layout(int batch, int neq, int nvar, int prec, void *base) {
  size_t off = 0;
  auto take = [&](size_t nd) {
    const size_t o = off;
    off += round256(sizeof(double) * nd);
    return reinterpret_cast<double *>(static_cast<char *>(base) + o);
  };
  const size_t NP = 2 * (size_t)prec, B = (size_t)batch;
  NewtonWork w;
  w.A = take(B * NP * neq * nvar);
  w.b = take(B * NP * neq);
  w.R = take(B * NP * nvar * nvar);
  w.d = take(B * NP * nvar);
  w.y = nullptr;
  w.info2 = nullptr;
  w.qrw = nullptr;
  w.qrw_bytes = 0;
  if (batch == 1 && prec >= 2) {
    w.y = take(NP * nvar);
    w.info2 = reinterpret_cast<int *>(take(1));
    w.qrw_bytes = qr_work_bytes(neq, nvar, prec);
    w.qrw = take((w.qrw_bytes + sizeof(double) - 1) / sizeof(double));
  }
  w.bytes = off;
  return w;
}
bool newton_dims_ok(int batch, int neq, int nvar, int nmon, int nvpm, int prec) {
  return batch >= 0 && batch <= 65535 && nvar >= 1 && nvar <= NT_MAX_VARS && neq >= nvar && nmon >= 1 && nmon <= NT_MAX_MON &&
         nvpm >= 1 && nvpm <= NT_MAX_VPM && batched_fits(neq, nvar, nvar + 1, prec);
}
template <class P>
int newton_launch(int batch, int neq, int nvar, int nmon, int nvpm, const int *vars, const int *exps,
                  const double *coef, double *x, int iters, double *dnorm, const NewtonWork &w, int *info,
                  long long spin, hipStream_t st) {
  for (int k = 0; k < iters; ++k) {
    hipLaunchKernelGGL((poly_eval_kernel<P>), dim3(neq, batch), dim3(64), 0, st, neq, nvar, nmon, nvpm, vars, exps,
                       coef, x, w.A, w.b, true);
    if (hipGetLastError() != hipSuccess) return MGS_ERR_LAUNCH;
    if (w.qrw != nullptr) {
      // One point (dd, qd): the single-system schedules of mgs_qr (dd: one
      // workgroup of 16 waves; qd: one column per launch), quicker than a
      // batch of one, then the back substitution (its own status word: a
      // zero pivot is already reported by the factorisation).
      int rc = mgs_qr_schedule(neq, nvar, P::L, w.A, neq, w.A, neq, w.R, nvar, w.b, w.y, nullptr, w.qrw, w.qrw_bytes,
                               info, MGS_SCHED_AUTO, reinterpret_cast<mgs_stream_t>(st));
      if (rc != MGS_OK) return rc;
      rc = backsolve_launch<P>(nvar, w.R, nvar, w.y, w.d, w.info2, st);
      if (rc != MGS_OK) return rc;
      hipLaunchKernelGGL((newton_update_kernel<P>), dim3(batch), dim3(64), 0, st, nvar, x, w.d, info,
                         dnorm != nullptr ? dnorm + (size_t)k * batch : nullptr);
      if (hipGetLastError() != hipSuccess) return MGS_ERR_LAUNCH;
      continue;
    }
    BatArgs a;
    a.batch = batch;
    a.m = neq;
    a.n = nvar;
    a.ncols = nvar + 1;
    a.A = w.A;
    a.lda = neq;
    a.b = w.b;
    a.Q = w.A;  // in place
    a.ldq = neq;
    a.R = w.R;
    a.ldr = nvar;
    a.y = nullptr;
    a.x = w.d;
    a.rho = nullptr;
    a.info = info;
    a.spin_ticks = spin;
    a.jitter = g_jitter.load(std::memory_order_relaxed);
    const int rc = batched_dispatch(P::L, a, st);
    if (rc != MGS_OK) return rc;
    hipLaunchKernelGGL((newton_update_kernel<P>), dim3(batch), dim3(64), 0, st, nvar, x, w.d, info,
                       dnorm != nullptr ? dnorm + (size_t)k * batch : nullptr);
    if (hipGetLastError() != hipSuccess) return MGS_ERR_LAUNCH;
  }
  return MGS_OK;
}

}  // namespace

extern "C" {

void mgs_set_jitter(unsigned seed) { g_jitter.store(seed, std::memory_order_relaxed); }


#ifdef MGS_TRACE
// Diagnostic builds only (not declared in the public header).
void mgs_set_trace(long long *buf) { g_trace = buf; }
void mgs_set_trace_backsolve(long long *buf) { g_trace_bs = buf; }
#endif

int mgs_abi_version(void) { return MGS_ABI_VERSION; }

const char *mgs_status_string(int status) {
  switch (status) {
    case MGS_OK: return "success";
    case MGS_ERR_DIMS: return "invalid dimensions (need 1 <= n <= m <= max rows, ld >= rows)";
    case MGS_ERR_POINTER: return "null, misaligned or illegally aliased pointer";
    case MGS_ERR_PREC: return "unsupported precision or block size";
    case MGS_ERR_WORKSPACE: return "workspace too small";
    case MGS_ERR_LAUNCH: return "kernel launch failed";
    case MGS_ERR_UNSUPPORTED: return "unsupported operation or schedule";
  }
  return "unknown status";
}

int mgs_workspace_size(int m, int n, int prec, int op, size_t *bytes) {
  if (op == MGS_OP_QR64 ? prec != 1
                        : (op == MGS_OP_QR || op == MGS_OP_SOLVE ? !prec_ok(prec) : (prec != 2 && prec != 4)))
    return MGS_ERR_PREC;
  if (n < 1 || m < n || m > (op == MGS_OP_QR64 ? MGS_MAX_ROWS_DD : max_rows(prec))) return MGS_ERR_DIMS;
  if (!bytes) return MGS_ERR_POINTER;
  switch (op) {
    case MGS_OP_QR: *bytes = qr_work_bytes(m, n, prec); return MGS_OK;
    case MGS_OP_SOLVE: *bytes = solve_work_bytes(n, prec); return MGS_OK;
    case MGS_OP_ADJOINT: *bytes = adjoint_work_bytes(m, n, prec); return MGS_OK;
    case MGS_OP_REFINE: *bytes = refine_layout(m, n, prec, nullptr).bytes; return MGS_OK;
    case MGS_OP_QR64: *bytes = qr64_work_bytes(m, n); return MGS_OK;
  }
  return MGS_ERR_UNSUPPORTED;
}

int mgs_qr_schedule(int m, int n, int prec, const double *A, int lda, double *Q, int ldq, double *R, int ldr,
                    const double *b, double *y, double *rho, void *work, size_t work_bytes, int *info,
                    int schedule, mgs_stream_t stream) {
  if (!prec_ok(prec)) return MGS_ERR_PREC;
  if (schedule < MGS_SCHED_AUTO || schedule > MGS_SCHED_SMALL) return MGS_ERR_UNSUPPORTED;
  if (n < 1 || m < n || m > max_rows(prec) || lda < m || ldq < m || ldr < n) return MGS_ERR_DIMS;
  if (!aligned8(A) || !aligned8(Q) || !aligned8(R) || !aligned8(info)) return MGS_ERR_POINTER;
  if (Q == A && ldq != lda) return MGS_ERR_POINTER;
  if (rho && !aligned8(rho)) return MGS_ERR_POINTER;
  if (!aligned8(work)) return MGS_ERR_POINTER;
  if (b && (!aligned8(b) || !aligned8(y))) return MGS_ERR_POINTER;
  if (work_bytes < qr_work_bytes(m, n, prec)) return MGS_ERR_WORKSPACE;
  Shape sh = choose_shape(m, prec, n + (b ? 1 : 0));
  StepArgs a;
  a.m = m;
  a.n = n;
  a.ncols = n + (b ? 1 : 0);
  a.A = A;
  a.lda = lda;
  a.planeA = (size_t)lda * n;
  a.b = b;
  a.Q = Q;
  a.ldq = ldq;
  a.planeQ = (size_t)ldq * n;
  a.R = R;
  a.ldr = ldr;
  a.planeR = (size_t)ldr * n;
  a.W = b ? static_cast<double *>(work) : nullptr;
  a.y = b ? y : nullptr;
  a.rho = b ? rho : nullptr;
  a.info = info;
  a.t = 0;
  a.kbase = 0;
  a.init_info = 1;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int mode = schedule;
  if (mode == MGS_SCHED_AUTO || mode == MGS_SCHED_SMALL) {
    int rc = 1;
    if (prec == 2) {
      rc = small_launch_dd(a, st);
    } else if (batched_fits(m, n, a.ncols, prec) && (prec == 1 || mode == MGS_SCHED_SMALL)) {
      // FP64 (and qd when asked for): the batched kernel on a batch of
      // one.  A single qd system takes the per-panel schedule by default:
      // the batched kernel's qd instantiation holds 16 waves per system and
      // spills to scratch (0.94 ms for 32 x 32 against ~0.5 ms).
      DevInfo d;
      if (dev_info(d)) {
        BatArgs ba;
        ba.batch = 1;
        ba.m = m;
        ba.n = n;
        ba.ncols = a.ncols;
        ba.A = A;
        ba.lda = lda;
        ba.b = b;
        ba.Q = Q;
        ba.ldq = ldq;
        ba.R = R;
        ba.ldr = ldr;
        ba.y = a.y;
        ba.x = nullptr;
        ba.rho = a.rho;
        ba.info = info;
        ba.spin_ticks = d.wclk_khz * 2000;  // 2 s
        ba.jitter = g_jitter.load(std::memory_order_relaxed);
        rc = batched_dispatch(prec, ba, st);
      }
    }
    if (rc != 1) return rc;
    if (mode == MGS_SCHED_SMALL) return MGS_ERR_DIMS;
  }
  if (mode == MGS_SCHED_AUTO || mode == MGS_SCHED_RESIDENT) {
    void *sync = static_cast<char *>(work) + qr_w_bytes(m, prec);
    double *u = reinterpret_cast<double *>(static_cast<char *>(sync) + sizeof(unsigned int) * RES_SYNC_WORDS);
    int rc = 1;
    if (qr_u_bytes(m, n, prec) > 0) rc = prec == 2 ? res_launch<PrecDD>(a, sync, u, st) : res_launch<PrecD>(a, sync, u, st);
    if (rc != 1) return rc;
    if (mode == MGS_SCHED_RESIDENT) return MGS_ERR_DIMS;
  }
  if (prec == 1) return dispatch_shape<PrecD>(a, sh, st);
  if (prec == 2) return dispatch_shape<PrecDD>(a, sh, st);
  return dispatch_shape<PrecQD>(a, sh, st);
}

int mgs_qr(int m, int n, int prec, const double *A, int lda, double *Q, int ldq, double *R, int ldr,
           const double *b, double *y, double *rho, void *work, size_t work_bytes, int *info,
           mgs_stream_t stream) {
  return mgs_qr_schedule(m, n, prec, A, lda, Q, ldq, R, ldr, b, y, rho, work, work_bytes, info, MGS_SCHED_AUTO,
                         stream);
}

int mgs_qr_noalloc(int m, int n, int prec, const double *A, int lda, double *Q, int ldq, double *R, int ldr,
                   const double *b, double *y, double *rho, int *info, mgs_stream_t stream) {
  if (!prec_ok(prec)) return MGS_ERR_PREC;
  if (n < 1 || m < n || m > max_rows(prec) || lda < m || ldq < m || ldr < n) return MGS_ERR_DIMS;
  const size_t need = qr_work_bytes(m, n, prec);
  if (need > MGS_NOALLOC_SCRATCH_BYTES) return MGS_ERR_WORKSPACE;
  void *work = scratch_address();
  if (work == nullptr) return MGS_ERR_LAUNCH;
  return mgs_qr_schedule(m, n, prec, A, lda, Q, ldq, R, ldr, b, y, rho, work, MGS_NOALLOC_SCRATCH_BYTES, info,
                         MGS_SCHED_AUTO, stream);
}

int ls_backsolve(int n, int prec, const double *R, int ldr, const double *y, double *x, int *info,
                 mgs_stream_t stream) {
  if (!prec_ok(prec)) return MGS_ERR_PREC;
  if (n < 1 || n > max_rows(prec) || ldr < n) return MGS_ERR_DIMS;
  if (!aligned8(R) || !aligned8(y) || !aligned8(x) || !aligned8(info)) return MGS_ERR_POINTER;
  if (x == y) return MGS_ERR_POINTER;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (prec == 1) return backsolve_launch<PrecD>(n, R, ldr, y, x, info, st);
  if (prec == 2) return backsolve_launch<PrecDD>(n, R, ldr, y, x, info, st);
  return backsolve_launch<PrecQD>(n, R, ldr, y, x, info, st);
}

int ls_solve(int m, int n, int prec, const double *Q, int ldq, const double *R, int ldr,
             const double *b, double *x, void *work, size_t work_bytes, int *info,
             mgs_stream_t stream) {
  if (!prec_ok(prec)) return MGS_ERR_PREC;
  if (n < 1 || m < n || m > max_rows(prec) || ldq < m || ldr < n) return MGS_ERR_DIMS;
  if (!aligned8(Q) || !aligned8(R) || !aligned8(b) || !aligned8(x) || !aligned8(info) || !aligned8(work))
    return MGS_ERR_POINTER;
  if (work_bytes < solve_work_bytes(n, prec)) return MGS_ERR_WORKSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  double *y = static_cast<double *>(work);
  int rc = prec == 1   ? project_launch<PrecD>(m, n, Q, ldq, b, y, st)
           : prec == 2 ? project_launch<PrecDD>(m, n, Q, ldq, b, y, st)
                       : project_launch<PrecQD>(m, n, Q, ldq, b, y, st);
  if (rc != MGS_OK) return rc;
  if (prec == 1) return backsolve_launch<PrecD>(n, R, ldr, y, x, info, st);
  if (prec == 2) return backsolve_launch<PrecDD>(n, R, ldr, y, x, info, st);
  return backsolve_launch<PrecQD>(n, R, ldr, y, x, info, st);
}

int ls_adjoint(int m, int n, int prec, const double *A, int lda, const double *b, const double *Q, int ldq,
               const double *R, int ldr, const double *x, const double *gx, double *gA, int ldga, double *gb,
               void *work, size_t work_bytes, int *info, mgs_stream_t stream) {
  if (prec != 2 && prec != 4) return MGS_ERR_PREC;
  if (n < 1 || m < n || m > max_rows(prec) || lda < m || ldq < m || ldr < n || ldga < m) return MGS_ERR_DIMS;
  if (!aligned8(A) || !aligned8(b) || !aligned8(Q) || !aligned8(R) || !aligned8(x) || !aligned8(gx) ||
      !aligned8(gA) || !aligned8(gb) || !aligned8(work) || !aligned8(info))
    return MGS_ERR_POINTER;
  if (gA == A || gA == Q || gb == b) return MGS_ERR_POINTER;
  if (work_bytes < adjoint_work_bytes(m, n, prec)) return MGS_ERR_WORKSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (prec == 2) return adjoint_launch<PrecDD>(m, n, A, lda, b, Q, ldq, R, ldr, x, gx, gA, ldga, gb, work, info, st);
  return adjoint_launch<PrecQD>(m, n, A, lda, b, Q, ldq, R, ldr, x, gx, gA, ldga, gb, work, info, st);
}

int mgs_refine_solve(int m, int n, int prec, const double *A, int lda, const double *b, double *x, int block,
                     double tol, int max_iter, int *iters, double *err_est, void *work, size_t work_bytes, int *info,
                     mgs_stream_t stream) {
  if (prec != 2 && prec != 4) return MGS_ERR_PREC;
  if (n < 1 || m < n || m > max_rows(prec) || lda < m || max_iter < 0) return MGS_ERR_DIMS;
  if (block != NBP) return MGS_ERR_PREC;
  if (!aligned8(A) || !aligned8(b) || !aligned8(x) || !aligned8(work) || !aligned8(info)) return MGS_ERR_POINTER;
  if (x == b || x == A) return MGS_ERR_POINTER;
  if (work_bytes < refine_layout(m, n, prec, nullptr).bytes) return MGS_ERR_WORKSPACE;
  if (!(tol >= 0.0)) return MGS_ERR_DIMS;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (prec == 2) return refine_solve<PrecDD>(m, n, A, lda, b, x, tol, max_iter, iters, err_est, work, info, st);
  return refine_solve<PrecQD>(m, n, A, lda, b, x, tol, max_iter, iters, err_est, work, info, st);
}

int mgs_qr64(int m, int n, const double *A, int lda, const double *b, double *Q, int ldq, double *R, int ldr,
             double *y, int block, void *work, size_t work_bytes, int *info, mgs_stream_t stream) {
  if (block != NBP) return MGS_ERR_PREC;
  if (n < 1 || m < n || m > MGS_MAX_ROWS_DD || lda < m || ldq < m || ldr < n) return MGS_ERR_DIMS;
  if (!aligned8(A) || !aligned8(Q) || !aligned8(R) || !aligned8(info) || !aligned8(work)) return MGS_ERR_POINTER;
  if (b != nullptr && (!aligned8(b) || !aligned8(y))) return MGS_ERR_POINTER;
  if (work_bytes < qr64_work_bytes(m, n)) return MGS_ERR_WORKSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  RefineWork w;
  w.Q64 = static_cast<double *>(work);
  w.R64 = reinterpret_cast<double *>(static_cast<char *>(work) + round256(sizeof(double) * 2 * (size_t)m * (n + 1)));
  w.res = panel_res_bytes(m, n) > 0 ? static_cast<char *>(work) + round256(sizeof(double) * 2 * (size_t)m * (n + 1)) +
                                          round256(sizeof(double) * 2 * (size_t)n * (n + 1))
                                    : nullptr;
  hipLaunchKernelGGL(copy64_in_kernel, dim3(ceil_div(m, 256), n + 1), dim3(256), 0, st, m, n, A, lda, b, w.Q64, info);
  if (hipGetLastError() != hipSuccess) return MGS_ERR_LAUNCH;
  const int rc = factor64(m, n, w, info, st);
  if (rc != MGS_OK) return rc;
  const int gx = ceil_div(m, 256) < 4 ? ceil_div(m, 256) : 4;
  hipLaunchKernelGGL(copy64_out_kernel, dim3(gx, n + 1), dim3(256), 0, st, m, n, w.Q64, w.R64, Q, ldq, R, ldr,
                     b != nullptr ? y : nullptr);
  return hipGetLastError() == hipSuccess ? MGS_OK : MGS_ERR_LAUNCH;
}

int mgs_poly_eval(int batch, int neq, int nvar, int nmon, int nvpm, int prec, const int *vars, const int *exps,
                  const double *coef, const double *x, double *J, double *F, mgs_stream_t stream) {
  if (!prec_ok(prec)) return MGS_ERR_PREC;
  if (batch < 0 || neq < 1 || neq > 65535 || nvar < 1 || nvar > NT_MAX_VARS || nmon < 1 || nmon > NT_MAX_MON ||
      nvpm < 1 || nvpm > NT_MAX_VPM || batch > 65535)
    return MGS_ERR_DIMS;
  if (batch == 0) return MGS_OK;
  if (!aligned8(coef) || !aligned8(x) || !aligned8(J) || !aligned8(F)) return MGS_ERR_POINTER;
  if (vars == nullptr || exps == nullptr || (reinterpret_cast<uintptr_t>(vars) & 3u) ||
      (reinterpret_cast<uintptr_t>(exps) & 3u))
    return MGS_ERR_POINTER;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (prec == 1)
    hipLaunchKernelGGL((poly_eval_kernel<PrecD>), dim3(neq, batch), dim3(64), 0, st, neq, nvar, nmon, nvpm, vars,
                       exps, coef, x, J, F, false);
  else if (prec == 2)
    hipLaunchKernelGGL((poly_eval_kernel<PrecDD>), dim3(neq, batch), dim3(64), 0, st, neq, nvar, nmon, nvpm, vars,
                       exps, coef, x, J, F, false);
  else
    hipLaunchKernelGGL((poly_eval_kernel<PrecQD>), dim3(neq, batch), dim3(64), 0, st, neq, nvar, nmon, nvpm, vars,
                       exps, coef, x, J, F, false);
  return hipGetLastError() == hipSuccess ? MGS_OK : MGS_ERR_LAUNCH;
}

int mgs_newton_workspace_size(int batch, int neq, int nvar, int prec, size_t *bytes) {
  if (!prec_ok(prec)) return MGS_ERR_PREC;
  if (!newton_dims_ok(batch, neq, nvar, 1, 1, prec)) return MGS_ERR_DIMS;
  if (bytes == nullptr) return MGS_ERR_POINTER;
  *bytes = newton_layout(batch, neq, nvar, prec, nullptr).bytes;
  return MGS_OK;
}

int mgs_newton_batched(int batch, int neq, int nvar, int nmon, int nvpm, int prec, const int *vars, const int *exps,
                       const double *coef, double *x, int iters, double *dnorm, void *work, size_t work_bytes,
                       int *info, mgs_stream_t stream) {
  if (!prec_ok(prec)) return MGS_ERR_PREC;
  if (!newton_dims_ok(batch, neq, nvar, nmon, nvpm, prec) || iters < 0) return MGS_ERR_DIMS;
  if (batch == 0 || iters == 0) return MGS_OK;
  if (!aligned8(coef) || !aligned8(x) || !aligned8(work) || !aligned8(info)) return MGS_ERR_POINTER;
  if (vars == nullptr || exps == nullptr || (reinterpret_cast<uintptr_t>(vars) & 3u) ||
      (reinterpret_cast<uintptr_t>(exps) & 3u))
    return MGS_ERR_POINTER;
  if (dnorm != nullptr && !aligned8(dnorm)) return MGS_ERR_POINTER;
  const NewtonWork w = newton_layout(batch, neq, nvar, prec, work);
  if (work_bytes < w.bytes) return MGS_ERR_WORKSPACE;
  DevInfo d;
  if (!dev_info(d)) return MGS_ERR_LAUNCH;
  const long long spin = d.wclk_khz * 2000;  // 2 s
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (prec == 1)
    return newton_launch<PrecD>(batch, neq, nvar, nmon, nvpm, vars, exps, coef, x, iters, dnorm, w, info, spin, st);
  if (prec == 2)
    return newton_launch<PrecDD>(batch, neq, nvar, nmon, nvpm, vars, exps, coef, x, iters, dnorm, w, info, spin, st);
  return newton_launch<PrecQD>(batch, neq, nvar, nmon, nvpm, vars, exps, coef, x, iters, dnorm, w, info, spin, st);
}

int mgs_lstsq_batched(int batch, int m, int n, int prec, const double *A, int lda, const double *b, double *Q,
                      int ldq, double *R, int ldr, double *y, double *x, double *rho, int *info,
                      mgs_stream_t stream) {
  if (!prec_ok(prec)) return MGS_ERR_PREC;
  const int ncols = n + (b ? 1 : 0);
  if (batch < 0 || n < 1 || m < n || lda < m || ldq < m || ldr < n) return MGS_ERR_DIMS;
  if (!batched_fits(m, n, ncols, prec)) return MGS_ERR_DIMS;
  if (batch == 0) return MGS_OK;  // nothing is read or written (empty tensors may have null pointers)
  if (!aligned8(A) || !aligned8(Q) || !aligned8(R) || !aligned8(info)) return MGS_ERR_POINTER;
  if (Q == A && ldq != lda) return MGS_ERR_POINTER;
  if (b != nullptr) {
    if (!aligned8(b) || (y == nullptr && x == nullptr)) return MGS_ERR_POINTER;
    if ((y != nullptr && !aligned8(y)) || (x != nullptr && !aligned8(x)) || (x != nullptr && x == y))
      return MGS_ERR_POINTER;
    if (rho != nullptr && !aligned8(rho)) return MGS_ERR_POINTER;
  }
  DevInfo d;
  if (!dev_info(d)) return MGS_ERR_LAUNCH;
  BatArgs a;
  a.batch = batch;
  a.m = m;
  a.n = n;
  a.ncols = ncols;
  a.A = A;
  a.lda = lda;
  a.b = b;
  a.Q = Q;
  a.ldq = ldq;
  a.R = R;
  a.ldr = ldr;
  a.y = b ? y : nullptr;
  a.x = b ? x : nullptr;
  a.rho = b ? rho : nullptr;
  a.info = info;
  a.spin_ticks = d.wclk_khz * 2000;  // 2 s
  a.jitter = g_jitter.load(std::memory_order_relaxed);
  return batched_dispatch(prec, a, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
