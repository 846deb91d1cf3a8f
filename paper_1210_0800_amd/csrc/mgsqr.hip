// C ABI of the MGS least-squares library (declared in include/mgsqr.h):
// argument checks, launch-shape selection and kernel launches.  No
// allocation, no host<->device copies, no synchronisation.
#include "../../include/mgsqr.h"

#include <hip/hip_runtime.h>

#include <cstdint>

#include "adjoint_kernels.hpp"
#include "mgs_kernels.hpp"

using namespace mgsq;

namespace {

bool aligned8(const void *p) { return p != nullptr && (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }
size_t round256(size_t b) { return (b + 255) & ~size_t(255); }
int max_rows(int prec) { return prec == 2 ? MGS_MAX_ROWS_DD : MGS_MAX_ROWS_QD; }
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
Shape choose_shape(int m, int prec) {
  const int rpt_max = prec == 2 ? 16 : 8;
  Shape s;
  s.tw = pow2_at_least(ceil_div(m, 64 * rpt_max));
  s.rpt = pow2_at_least(ceil_div(m, 64 * s.tw));
  s.rp = s.rpt * s.tw / NWAVE > 1 ? s.rpt * s.tw / NWAVE : 1;
  return s;
}
constexpr int bw_for(int L, int RP) {
  // complex elements per thread held by the panel role: dd 8, qd 4; the
  // panel width is capped (dd 4, qd 2) so that its loops unroll fully and
  // every register array keeps static indices.
  return L == 2 ? (8 / RP >= 4 ? 4 : (8 / RP >= 1 ? 8 / RP : 1)) : (4 / RP >= 2 ? 2 : (4 / RP >= 1 ? 4 / RP : 1));
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
  if constexpr (P::L == 2) {
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
    } else if (sh.rpt == 8 && sh.tw == 4) {
      return launch_steps<P, 8, 4>(a, st);
    }
  }
  return MGS_ERR_DIMS;
}

template <class P>
int backsolve_launch(int n, const double *R, int ldr, const double *y, double *x, int *info, hipStream_t st) {
  const int ny = pow2_at_least(ceil_div(n, WG));
  const size_t planeR = (size_t)ldr * n;
#define MGS_NY_CASE(NYV)                                                                                  \
  case NYV:                                                                                               \
    hipLaunchKernelGGL((backsolve_kernel<P, NYV>), dim3(1), dim3(WG), 0, st, n, R, ldr, planeR, y, x, info); \
    break;
  switch (ny) {
    MGS_NY_CASE(1)
    MGS_NY_CASE(2)
    MGS_NY_CASE(4)
    MGS_NY_CASE(8)
    MGS_NY_CASE(16)
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

size_t qr_work_bytes(int m, int prec) { return round256(sizeof(double) * 2 * (size_t)prec * m); }
size_t solve_work_bytes(int n, int prec) { return round256(sizeof(double) * 2 * (size_t)prec * n); }
// adjoint: w (n), z (n), r (m)
size_t adjoint_work_bytes(int m, int n, int prec) {
  return 2 * round256(sizeof(double) * 2 * (size_t)prec * n) + round256(sizeof(double) * 2 * (size_t)prec * m);
}

template <class P>
int fwdsub_launch(int n, const double *R, int ldr, const double *g, double *w, int *info, hipStream_t st) {
  const int ny = pow2_at_least(ceil_div(n, WG));
  const size_t planeR = (size_t)ldr * n;
#define MGS_FS_CASE(NYV)                                                                                 \
  case NYV:                                                                                              \
    hipLaunchKernelGGL((fwdsub_kernel<P, NYV>), dim3(1), dim3(WG), 0, st, n, R, ldr, planeR, g, w, info); \
    break;
  switch (ny) {
    MGS_FS_CASE(1)
    MGS_FS_CASE(2)
    MGS_FS_CASE(4)
    MGS_FS_CASE(8)
    MGS_FS_CASE(16)
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
  int rc = fwdsub_launch<P>(n, R, ldr, gx, w, info, st);
  if (rc != MGS_OK) return rc;
  rc = backsolve_launch<P>(n, R, ldr, w, z, info, st);
  if (rc != MGS_OK) return rc;
  hipLaunchKernelGGL((adj_gemv_kernel<P>), dim3(ceil_div(m, WG)), dim3(WG), 0, st, m, n, Q, ldq, (size_t)ldq * n,
                     A, lda, (size_t)lda * n, b, x, w, gb, r);
  if (hipGetLastError() != hipSuccess) return MGS_ERR_LAUNCH;
  hipLaunchKernelGGL((adj_rank2_kernel<P>), dim3(ceil_div(m, WG), n), dim3(WG), 0, st, m, n, r, z, gb, x, gA, ldga,
                     (size_t)ldga * n);
  return hipGetLastError() == hipSuccess ? MGS_OK : MGS_ERR_LAUNCH;
}

}  // namespace

extern "C" {

int mgs_abi_version(void) { return MGS_ABI_VERSION; }

const char *mgs_status_string(int status) {
  switch (status) {
    case MGS_OK: return "success";
    case MGS_ERR_DIMS: return "invalid dimensions (need 1 <= n <= m <= max rows, ld >= rows)";
    case MGS_ERR_POINTER: return "null, misaligned or illegally aliased pointer";
    case MGS_ERR_PREC: return "unsupported precision (prec must be 2 or 4)";
    case MGS_ERR_WORKSPACE: return "workspace too small";
    case MGS_ERR_LAUNCH: return "kernel launch failed";
    case MGS_ERR_UNSUPPORTED: return "unsupported operation";
  }
  return "unknown status";
}

int mgs_workspace_size(int m, int n, int prec, int op, size_t *bytes) {
  if (prec != 2 && prec != 4) return MGS_ERR_PREC;
  if (n < 1 || m < n || m > max_rows(prec)) return MGS_ERR_DIMS;
  if (!bytes) return MGS_ERR_POINTER;
  switch (op) {
    case MGS_OP_QR: *bytes = qr_work_bytes(m, prec); return MGS_OK;
    case MGS_OP_SOLVE: *bytes = solve_work_bytes(n, prec); return MGS_OK;
    case MGS_OP_ADJOINT: *bytes = adjoint_work_bytes(m, n, prec); return MGS_OK;
  }
  return MGS_ERR_UNSUPPORTED;
}

int mgs_qr(int m, int n, int prec, const double *A, int lda, double *Q, int ldq, double *R, int ldr,
           const double *b, double *y, double *rho, void *work, size_t work_bytes, int *info,
           mgs_stream_t stream) {
  if (prec != 2 && prec != 4) return MGS_ERR_PREC;
  if (n < 1 || m < n || m > max_rows(prec) || lda < m || ldq < m || ldr < n) return MGS_ERR_DIMS;
  if (!aligned8(A) || !aligned8(Q) || !aligned8(R) || !aligned8(info)) return MGS_ERR_POINTER;
  if (Q == A && ldq != lda) return MGS_ERR_POINTER;
  if (rho && !aligned8(rho)) return MGS_ERR_POINTER;
  if (b) {
    if (!aligned8(b) || !aligned8(y) || !aligned8(work)) return MGS_ERR_POINTER;
    if (work_bytes < qr_work_bytes(m, prec)) return MGS_ERR_WORKSPACE;
  }
  Shape sh = choose_shape(m, prec);
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
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (prec == 2) return dispatch_shape<PrecDD>(a, sh, st);
  return dispatch_shape<PrecQD>(a, sh, st);
}

int ls_backsolve(int n, int prec, const double *R, int ldr, const double *y, double *x, int *info,
                 mgs_stream_t stream) {
  if (prec != 2 && prec != 4) return MGS_ERR_PREC;
  if (n < 1 || n > max_rows(prec) || ldr < n) return MGS_ERR_DIMS;
  if (!aligned8(R) || !aligned8(y) || !aligned8(x) || !aligned8(info)) return MGS_ERR_POINTER;
  if (x == y) return MGS_ERR_POINTER;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (prec == 2) return backsolve_launch<PrecDD>(n, R, ldr, y, x, info, st);
  return backsolve_launch<PrecQD>(n, R, ldr, y, x, info, st);
}

int ls_solve(int m, int n, int prec, const double *Q, int ldq, const double *R, int ldr,
             const double *b, double *x, void *work, size_t work_bytes, int *info,
             mgs_stream_t stream) {
  if (prec != 2 && prec != 4) return MGS_ERR_PREC;
  if (n < 1 || m < n || m > max_rows(prec) || ldq < m || ldr < n) return MGS_ERR_DIMS;
  if (!aligned8(Q) || !aligned8(R) || !aligned8(b) || !aligned8(x) || !aligned8(info) || !aligned8(work))
    return MGS_ERR_POINTER;
  if (work_bytes < solve_work_bytes(n, prec)) return MGS_ERR_WORKSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  double *y = static_cast<double *>(work);
  int rc = prec == 2 ? project_launch<PrecDD>(m, n, Q, ldq, b, y, st) : project_launch<PrecQD>(m, n, Q, ldq, b, y, st);
  if (rc != MGS_OK) return rc;
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

}  // extern "C"
