/*
 * mgsqr -- complex least squares by modified Gram-Schmidt (MGS) in
 * double-double (dd) and quad-double (qd) arithmetic on AMD MI355X (gfx950).
 *
 * Method: J. Verschelde and G. Yoffe, "Orthogonalization on a General
 * Purpose Graphics Processing Unit with Double Double and Quad Double
 * Arithmetic".  Section 3, Figure 1 defines MGS; Section 3, Equation (1)
 * defines the least-squares solve by MGS on the matrix augmented with the
 * right-hand side; Section 6, Figure 3 defines the column-oriented back
 * substitution.
 *
 * ------------------------------------------------------------------------
 * Number formats and layout ("planar", all device memory, float64):
 *   prec = number of FP64 limbs per real number: 1 (complex double, the
 *   paper's third precision), 2 (dd) or 4 (qd).  Entry points say which
 *   they accept.
 *   A complex matrix with `cols` columns, leading dimension ld >= rows, is
 *   2*prec planes of ld*cols doubles each; plane p = 2*limb + part holds
 *   limb `limb` of the real (part 0) or imaginary (part 1) parts,
 *   column-major: element (i, j) of plane p is at base[p*ld*cols + j*ld + i].
 *   A vector of length len is the same with ld = len, cols = 1.
 *   Inputs must be normalised: |x_{k+1}| <= ulp(x_k) / 2 limb by limb.
 *   A PyTorch view of a matrix is a contiguous float64 tensor of shape
 *   [prec, 2, cols, ld].
 *
 * Ownership: the caller allocates and frees every buffer, including the
 * workspace, and keeps them alive until the work enqueued on `stream` has
 * finished.  The library does not allocate, copy between host and device,
 * or synchronise; it enqueues kernels on `stream` (NULL = default stream).
 *
 * Errors: the return value reports argument errors synchronously:
 *   MGS_OK (0) success, MGS_ERR_DIMS, MGS_ERR_POINTER, MGS_ERR_PREC,
 *   MGS_ERR_WORKSPACE, MGS_ERR_LAUNCH, MGS_ERR_UNSUPPORTED (negative).
 * Numerical status goes to the device int *info (written by the kernels):
 *   0 = success; k > 0 = column k (1-based) had a zero or non-finite norm
 *   (MGS does not pivot, Section 4), outputs from column k on are then
 *   unspecified; MGS_INFO_SYNC_TIMEOUT = a wait between workgroups of the
 *   single-launch factorisation exceeded its time limit (outputs
 *   unspecified; not expected in normal operation).
 * ------------------------------------------------------------------------
 */
#ifndef MGSQR_H
#define MGSQR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

struct ihipStream_t; /* hipStream_t is `struct ihipStream_t *` */
typedef struct ihipStream_t *mgs_stream_t;

#define MGS_ABI_VERSION 1

enum {
  MGS_OK = 0,
  MGS_ERR_DIMS = -1,        /* n < 1, m < n, ld too small, size above the supported maximum */
  MGS_ERR_POINTER = -2,     /* required pointer NULL or not 8-byte aligned, forbidden aliasing */
  MGS_ERR_PREC = -3,        /* prec not supported by the entry point, or block not 64 */
  MGS_ERR_WORKSPACE = -4,   /* work_bytes below mgs_workspace_size() */
  MGS_ERR_LAUNCH = -5,      /* a kernel launch failed (HIP error) */
  MGS_ERR_UNSUPPORTED = -6  /* unknown operation code or schedule */
};

/* *info value of a factorisation whose inter-workgroup wait timed out. */
#define MGS_INFO_SYNC_TIMEOUT (-9)

enum { MGS_OP_QR = 0, MGS_OP_SOLVE = 1, MGS_OP_ADJOINT = 2, MGS_OP_REFINE = 3, MGS_OP_QR64 = 4 };

/* Largest supported row count m: double and dd 4096, qd 2048. */
#define MGS_MAX_ROWS_DD 4096
#define MGS_MAX_ROWS_QD 2048

int mgs_abi_version(void);
const char *mgs_status_string(int status);

/* Bytes of device workspace needed by operation `op` (MGS_OP_QR and
 * MGS_OP_SOLVE with prec 1, 2 or 4; MGS_OP_ADJOINT and MGS_OP_REFINE with
 * prec 2 or 4; MGS_OP_QR64 with prec 1) for an m x n problem;
 * written to *bytes.  A workspace may be reused by later calls on the same
 * stream; calls that may overlap need distinct workspaces. */
int mgs_workspace_size(int m, int n, int prec, int op, size_t *bytes);

/*
 * mgs_qr -- MGS QR of A (Section 3, Figure 1), optionally of [A b]
 * (Section 3, Equation (1)).
 *   A  [in]   m x n planar, lda >= m.  Not modified unless Q == A.
 *   Q  [out]  m x n planar, ldq >= m; Q == A (with ldq == lda) overwrites A
 *             in place as the paper's GPU algorithm does (Section 5).
 *   R  [out]  n x n planar, ldr >= n: upper triangular with a real
 *             positive diagonal (imaginary parts +0), lower triangle 0.
 *   b  [in]   m planar or NULL.  When given, MGS runs on [A b]:
 *   y  [out]  n planar, y = Q^H b as the projections of b (may be NULL
 *             only when b is NULL).
 *   rho[out]  prec doubles (the limbs of a real number) or NULL: the norm z
 *             of the projected right-hand side, ||b - A x|| of the
 *             least-squares solution x (Equation (1)).
 *   work      workspace of mgs_workspace_size(m, n, prec, MGS_OP_QR) bytes
 *             (always required: it holds the working copy of b, the
 *             publication counters of the single-launch factorisation and,
 *             in dd with m <= 1024 and in double with m <= 2048 and
 *             16 m n <= 32 MiB, its hand-off copy of the columns, 16 prec
 *             m n bytes).
 *   info      device int, see above.
 * prec 1, 2 or 4.  Requires 1 <= n <= m <= MGS_MAX_ROWS_{DD,QD}.
 * Schedule: in dd and double with m <= 64 and at most 64 columns of [A b],
 * one workgroup (a column per wave slot, q vectors through LDS; for double
 * the kernel of mgs_lstsq_batched on one system; qd takes it only when
 * mgs_qr_schedule asks for it, within 159 KiB of q vectors: 64 m n bytes);
 * in dd and double when
 * every column fits in the register file of the device (dd: m <= 1024 and
 * at most 5 columns per compute unit, 8 when m <= 512, e.g. 1024 x 1024
 * with b on 256 compute units; double: m <= 2048, 5 columns per compute
 * unit beyond 1024 rows, 8 below) one cooperative launch with the columns
 * held in registers; otherwise (and in qd) one launch per panel of
 * columns.
 * mgs_qr_schedule (below) forces one of them.
 * All schedules apply the projections of Figure 1 in the same order per
 * column; reduction trees differ, and in the single launch the last twelve
 * projections onto each column use r_kj = (a_k^H a_j) / r_kk with a_k
 * before its normalisation (equal to q_k^H a_j in exact arithmetic), so
 * results agree to rounding.
 */
int mgs_qr(int m, int n, int prec, const double *A, int lda, double *Q, int ldq, double *R, int ldr,
           const double *b, double *y, double *rho, void *work, size_t work_bytes, int *info,
           mgs_stream_t stream);

/*
 * mgs_qr_noalloc -- mgs_qr for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * allocation): no workspace argument; the workspace lives in a fixed
 * device array of MGS_NOALLOC_SCRATCH_BYTES that the library holds on each
 * GPU it runs on until the process ends.  Enough for every shape mgs_qr
 * accepts (the largest need is dd 1024 x 1024 with b: 32 MiB + 33 KiB);
 * a shape that would need more returns MGS_ERR_WORKSPACE.  Calls no
 * allocating routine.  Every call on one GPU shares that GPU's array, so
 * calls that may overlap in time on the same GPU (different streams or
 * threads) race: the caller serialises them.  Each call initialises what it
 * uses (counters, hand-off buffer) itself.  Arguments, results and status
 * otherwise as mgs_qr.
 */
#define MGS_NOALLOC_SCRATCH_BYTES (33u * 1024u * 1024u)
int mgs_qr_noalloc(int m, int n, int prec, const double *A, int lda, double *Q, int ldq, double *R, int ldr,
                   const double *b, double *y, double *rho, int *info, mgs_stream_t stream);

/* Schedules of mgs_qr_schedule. */
enum { MGS_SCHED_AUTO = 0, MGS_SCHED_PANEL = 1, MGS_SCHED_RESIDENT = 2, MGS_SCHED_SMALL = 3 };

/*
 * mgs_qr_schedule -- mgs_qr with the schedule named by the caller (for
 * tests and diagnostics; mgs_qr is this call with MGS_SCHED_AUTO):
 * MGS_SCHED_PANEL one launch per panel, MGS_SCHED_RESIDENT the single
 * cooperative launch, MGS_SCHED_SMALL the one-workgroup schedule.
 * Returns MGS_ERR_DIMS when the named schedule does not apply to the
 * shape and precision, MGS_ERR_UNSUPPORTED for an unknown schedule;
 * otherwise as mgs_qr.
 */
int mgs_qr_schedule(int m, int n, int prec, const double *A, int lda, double *Q, int ldq, double *R, int ldr,
                    const double *b, double *y, double *rho, void *work, size_t work_bytes, int *info,
                    int schedule, mgs_stream_t stream);

/*
 * ls_solve -- least-squares solution x of A x = b from the MGS factors of
 * A: y = Q^H b by n sequential MGS projections of b (the same operations as
 * the augmented column of Equation (1)), then the back substitution of
 * Section 6, Figure 3.
 *   Q  [in] m x n planar (ldq), R [in] n x n planar (ldr), b [in] m planar,
 *   x  [out] n planar.  prec 1, 2 or 4.
 *   work: mgs_workspace_size(m, n, prec, MGS_OP_SOLVE).
 */
int ls_solve(int m, int n, int prec, const double *Q, int ldq, const double *R, int ldr,
             const double *b, double *x, void *work, size_t work_bytes, int *info,
             mgs_stream_t stream);

/*
 * ls_backsolve -- x = R^{-1} y, column-oriented back substitution
 * (Section 6, Figure 3): for k = n..1, x_k = y_k / r_kk, then
 * y_j -= r_jk x_k for j < k.
 *   R [in] n x n planar (ldr >= n), upper triangle and real diagonal read;
 *   y [in] n planar (not modified); x [out] n planar.
 *   info: 0, or k > 0 when r_kk is zero or not finite (smallest such k).
 * prec 1, 2 or 4.  Requires 1 <= n <= MGS_MAX_ROWS_{DD,QD}.
 */
int ls_backsolve(int n, int prec, const double *R, int ldr, const double *y, double *x, int *info,
                 mgs_stream_t stream);

/*
 * ls_adjoint -- gradients of a loss L(x) through the least-squares solution
 * x = argmin ||b - A x|| (the differentiation form built around the solver
 * of Section 3; not itself in the paper).  Given gx = dL/dRe(x) + i dL/dIm(x)
 * and the MGS factors A = Q R of full column rank:
 *   w = R^{-H} gx, z = R^{-1} w (so z = (A^H A)^{-1} gx),
 *   gb = Q w (= A z),  r = b - A x,  gA = r z^H - gb x^H,
 * gA and gb in the same convention (dL/dRe + i dL/dIm).
 *   A [in] m x n (lda), b [in] m, Q [in] m x n (ldq), R [in] n x n (ldr),
 *   x [in] n (the solution from the same factors), gx [in] n.
 *   gA [out] m x n planar (ldga >= m), gb [out] m planar.
 *   work: mgs_workspace_size(m, n, prec, MGS_OP_ADJOINT) bytes.
 *   info: 0, or k > 0 when r_kk is zero or not finite.
 * gA may not alias A or Q, gb may not alias b.
 */
int ls_adjoint(int m, int n, int prec, const double *A, int lda, const double *b, const double *Q, int ldq,
               const double *R, int ldr, const double *x, const double *gx, double *gA, int ldga, double *gb,
               void *work, size_t work_bytes, int *info, mgs_stream_t stream);

/*
 * mgs_refine_solve -- the precision form (not in the paper; built around
 * the solver of Section 3): least squares A x = b with a factorisation in
 * plain FP64 and the solution refined in dd / qd.
 *   1. [fl64(A) fl64(b)] is factored by blocked MGS in FP64: panels of
 *      `block` = 64 columns, each factored by MGS (Figure 1), the trailing
 *      products W = Q_p^H A_t and A_t -= Q_p W on FP64 matrix cores; b is
 *      the last column, so y = Q^H b keeps the augmented semantics of
 *      Equation (1).  x0 = R^{-1} y in FP64.
 *   2. Repeat up to max_iter times: r = b - A x in dd / qd (A, b, x in the
 *      working precision), d = FP64 solve of fl64(r) (the same panel
 *      projections replayed on r, then R^{-1}), x += d in dd / qd; stop when
 *      ||d|| <= tol ||x||, or when ||d|| > ||d_prev|| / 2 (the corrections
 *      stalled; that d is not applied): converged to the attainable accuracy
 *      if the last applied ||d|| / ||x|| <= sqrt(tol), stagnation otherwise.
 *      All of it is enqueued at once (no host synchronisation): the steps
 *      after the stopping test return at once on the device, and the
 *      projections of one step run in one cooperative launch.
 *   A [in] m x n planar (lda), b [in] m planar, x [out] n planar, all in
 *   `prec` limbs.  block must be 64 (MGS_ERR_PREC otherwise).  tol >= 0 (e.g. 2^-104 dd, 2^-209 qd).
 *   iters [out, device int or NULL]: refinement steps applied.
 *   err_est [out, device double or NULL]: ||d|| / ||x|| of the last step.
 *   work: mgs_workspace_size(m, n, prec, MGS_OP_REFINE) bytes.
 *   info [device int]: 0 converged; k > 0 zero or non-finite norm at column
 *   k of the FP64 factorisation; -1 stagnated above sqrt(tol); -2 max_iter
 *   reached first; MGS_INFO_SYNC_TIMEOUT when a bounded wait between
 *   workgroups (the FP64 panels' single launch, the projections) ran out.
 * Convergence needs kappa(A) * 2^-53 well below 1 and a consistent or
 * nearly consistent system.
 */
int mgs_refine_solve(int m, int n, int prec, const double *A, int lda, const double *b, double *x, int block,
                     double tol, int max_iter, int *iters, double *err_est, void *work, size_t work_bytes, int *info,
                     mgs_stream_t stream);

/*
 * mgs_qr64 -- the factorisation of the precision form on its own: complex
 * FP64 blocked MGS of [A b] (not in the paper, whose Section 2 leaves
 * blocked versions aside).  For each panel of `block` columns, the MGS of
 * Figure 1 inside the panel (FP64 vector units), then W = Q_p^H A_t and
 * A_t -= Q_p W for the trailing columns A_t (b included) as complex
 * products on the FP64 matrix cores.  Every column receives the panels'
 * projections in panel order.
 *   A  [in]   m x n complex FP64 planar: 2 planes (re, im) of lda x n
 *             column-major doubles, lda >= m.
 *   b  [in]   m complex FP64 planar (2 planes of m) or NULL.
 *   Q  [out]  m x n planar (ldq >= m); R [out] n x n planar (ldr >= n),
 *             upper triangular, real positive diagonal, lower triangle 0.
 *   y  [out]  n planar: y = Q^H b as the projections of b (required when
 *             b != NULL, ignored otherwise).
 *   block     panel width; must be 64 (MGS_ERR_PREC otherwise).
 *   work      mgs_workspace_size(m, n, 1, MGS_OP_QR64, .) bytes (the FP64
 *             factors and, for m <= 2048, the hand-off area of the single
 *             launch that factors each panel).
 *   info      device int: 0, or k > 0 when column k had a zero or
 *             non-finite norm.
 * Requires 1 <= n <= m <= MGS_MAX_ROWS_DD.
 */
int mgs_qr64(int m, int n, const double *A, int lda, const double *b, double *Q, int ldq, double *R, int ldr,
             double *y, int block, void *work, size_t work_bytes, int *info, mgs_stream_t stream);

/*
 * mgs_lstsq_batched -- `batch` independent systems, each factored by the MGS
 * of Figure 1 (Section 3) on [A_s b_s] (Equation (1)) and, when b is given,
 * solved by the back substitution of Section 6, Figure 3: the many small
 * systems of many paths (Section 2), all resident on the card (Section 7).
 * One workgroup per system; systems are independent, so their order of
 * completion is unspecified and each system's results are the same as for a
 * batch of one.
 *   prec 1, 2 or 4.  Requires 1 <= n <= m <= 64, at most 64 columns of
 *   [A b], and 16 prec m n <= 162816 (the q vectors of a system in LDS;
 *   binding for qd only: e.g. m = n = 50).  batch >= 0 (0: nothing to do,
 *   pointers not examined).
 *   A  [in]  batch systems back to back: system s at A + s*2*prec*lda*n,
 *            each m x n planar with leading dimension lda >= m (a torch view
 *            [batch, prec, 2, n, lda]).
 *   b  [in]  batch vectors of m (system s at b + s*2*prec*m) or NULL (QR only).
 *   Q  [out] like A with ldq >= m; Q == A (ldq == lda) overwrites A.
 *   R  [out] batch n x n planar (ldr >= n), system s at R + s*2*prec*ldr*n:
 *            upper triangular, real positive diagonal, lower triangle 0.
 *   y  [out] batch vectors of n (system s at y + s*2*prec*n) or NULL: the
 *            projections Q^H b.
 *   x  [out] batch vectors of n or NULL: the least-squares solutions.
 *            With b given, at least one of y and x is required; x != y.
 *   rho[out] batch x prec doubles or NULL: ||b_s - A_s x_s|| (Equation (1)).
 *   info [out] batch device ints: 0, k > 0 when column k of that system had
 *            a zero or non-finite norm (its x is then not computed and its
 *            later columns are unspecified), or MGS_INFO_SYNC_TIMEOUT.
 * No workspace.
 */
int mgs_lstsq_batched(int batch, int m, int n, int prec, const double *A, int lda, const double *b, double *Q,
                      int ldq, double *R, int ldr, double *y, double *x, double *rho, int *info,
                      mgs_stream_t stream);

/*
 * Polynomial systems (Section 7: Newton's method as the corrector of a path
 * tracker, the system defined once on the card, its evaluated Jacobian and
 * values never leaving it; the workload of Table 6).  Equation e is
 *   f_e(x) = sum_m c_em prod_t x_{v_emt}^{d_emt},
 * m < nmon monomials of nvpm variables each.  Layouts:
 *   vars, exps [in] device int32 [neq][nmon][nvpm]: variable index
 *            (0 <= v < nvar) and exponent (0 <= d <= 16) of factor t of
 *            monomial m of equation e (values outside are clamped into
 *            those ranges).
 *   coef [in] planar (prec, 2, neq, nmon): c_em at e*nmon + m, plane
 *            stride neq*nmon.
 *   x    points: batch vectors of nvar planar (point s at x + s*2*prec*nvar),
 *            a torch view [batch, prec, 2, nvar].
 * Limits: 1 <= nvar <= 63, 1 <= nmon <= 64, 1 <= nvpm <= 8, batch <= 65535.
 */

/*
 * mgs_poly_eval -- F = f(x) and the Jacobian J = df/dx at batch points, in
 * the working precision: monomials and their derivatives by products of
 * powers, sums over the monomials in ascending order.
 *   J [out] batch neq x nvar planar with leading dimension neq (column j =
 *           d f / d x_j; point s at J + s*2*prec*neq*nvar), the A layout of
 *           mgs_lstsq_batched.
 *   F [out] batch vectors of neq (point s at F + s*2*prec*neq).
 *   neq <= 65535.  No workspace.
 */
int mgs_poly_eval(int batch, int neq, int nvar, int nmon, int nvpm, int prec, const int *vars, const int *exps,
                  const double *coef, const double *x, double *J, double *F, mgs_stream_t stream);

/*
 * mgs_newton_workspace_size -- bytes of device workspace mgs_newton_batched
 * needs (J, -f, R and the correction of every point; for a single point in
 * dd or qd also Q^H b, a status word and the workspace of mgs_qr's
 * single-system schedule).
 */
int mgs_newton_workspace_size(int batch, int neq, int nvar, int prec, size_t *bytes);

/*
 * mgs_newton_batched -- `iters` Newton steps at each of batch points, all on
 * the card: per step, f and J by mgs_poly_eval's kernel, the correction d
 * as the least-squares solution of J d = -f by the MGS of Figure 1 on
 * [J -f] (Equation (1)) and the back substitution of Figure 3 (the
 * mgs_lstsq_batched kernel, one workgroup per point; for a single point in
 * dd or qd the single-system schedules of mgs_qr and ls_backsolve), then
 * x += d.
 *   Requires nvar <= neq <= 64 and 16 prec neq nvar <= 162816 (the MGS
 *   limits of mgs_lstsq_batched), iters >= 0.
 *   x     [in/out] the points (updated in place).
 *   dnorm [out] iters x batch doubles or NULL: FP64 2-norm of the leading
 *         limbs of step k's correction of point s at dnorm[k*batch + s];
 *         NaN when that step's factorisation failed.
 *   work  mgs_newton_workspace_size(batch, neq, nvar, prec) bytes.
 *   info  [out] batch device ints: status of each point's last
 *         factorisation (0, k > 0 for a zero or non-finite norm of column
 *         k of J, MGS_INFO_SYNC_TIMEOUT); a failed point keeps its x for
 *         that step.
 * batch == 0 or iters == 0: nothing to do, pointers not examined.
 */
int mgs_newton_batched(int batch, int neq, int nvar, int nmon, int nvpm, int prec, const int *vars, const int *exps,
                       const double *coef, double *x, int iters, double *dnorm, void *work, size_t work_bytes,
                       int *info, mgs_stream_t stream);

/*
 * mgs_set_jitter -- race checks (diagnostics, not for production use):
 * with seed != 0, the kernels that synchronise across waves or workgroups
 * (the single-launch factorisation, the one-workgroup and batched kernels,
 * the triangular solves across workgroups) pause each wave for 0..15 x 64
 * clocks at every step, the length drawn from (seed, workgroup, wave,
 * step).  Every reduction order is fixed, so results must be bitwise those
 * of seed 0; a difference is a race.  Applies to launches made after the
 * call, process-wide, until called again with 0.
 */
void mgs_set_jitter(unsigned seed);

#ifdef __cplusplus
}
#endif

#endif /* MGSQR_H */
