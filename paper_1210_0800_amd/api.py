"""Torch-facing wrappers of the C ABI (include/mgsqr.h).

Tensors are float64, contiguous, on a HIP device, in the planar layout
[prec, 2, cols, ld] (matrices) or [prec, 2, len] (vectors): limb, real /
imaginary part, column, row.  prec = 1 (complex double), 2 (double-double)
or 4 (quad-double); the adjoint and the precision form take 2 and 4.
Batched calls put a leading batch axis in front: [batch, prec, 2, ...].
Work is enqueued on the current torch stream; nothing is synchronised.
"""
import torch

from . import _lib


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(t):
    return torch.cuda.current_stream(t.device).cuda_stream


def _check_planar(name, t, prec=None, ndim=None, shape=None, device=None):
    """t must be a contiguous float64 device tensor; shape (when given) is
    its full expected shape, so that no kernel reads or writes past it."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("%s must be a contiguous float64 tensor on a HIP device" % name)
    if device is not None and t.device != device:
        raise ValueError("%s must be on %s, got %s" % (name, device, t.device))
    if ndim is not None and t.dim() != ndim:
        raise ValueError("%s must have %d dimensions, got shape %s" % (name, ndim, tuple(t.shape)))
    if t.dim() < 2 or t.shape[1] != 2 or (prec is not None and t.shape[0] != prec):
        raise ValueError("%s must have shape [prec, 2, ...], got %s" % (name, tuple(t.shape)))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))


def _check_info(info, device):
    if not isinstance(info, torch.Tensor) or info.dtype != torch.int32 or info.numel() < 1 or \
            info.device != device or not info.is_contiguous():
        raise ValueError("info must be a contiguous int32 tensor on %s" % device)


def _check_work(work, nbytes, device):
    if not isinstance(work, torch.Tensor) or not work.is_contiguous() or work.device != device:
        raise ValueError("work must be a contiguous tensor on %s" % device)
    if work.numel() * work.element_size() < nbytes:
        raise ValueError("work holds %d bytes, %d needed" % (work.numel() * work.element_size(), nbytes))


def workspace(m, n, prec, op, device):
    nbytes = _lib.workspace_size(m, n, prec, op)
    return torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device=device)


def mgs_qr(A, b=None, *, Q=None, R=None, y=None, rho=None, info=None, work=None, with_rho=True,
           schedule=None):
    """MGS QR of A (Figure 1), of [A b] when b is given (Equation (1)).

    Returns dict(Q, R, y, rho, info) of device tensors; Q may be passed as A
    itself to factor in place.  schedule (None = automatic) names one of
    "panel", "resident", "small" (mgs_qr_schedule; for tests and timing).
    """
    _check_planar("A", A, ndim=4)
    prec, _, n, m = A.shape
    dev = A.device
    Q = torch.empty_like(A) if Q is None else Q
    _check_planar("Q", Q, prec, 4, shape=A.shape, device=dev)
    R = torch.empty((prec, 2, n, n), dtype=torch.float64, device=dev) if R is None else R
    _check_planar("R", R, prec, 4, shape=(prec, 2, n, n), device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev) if info is None else info
    _check_info(info, dev)
    if b is not None:
        _check_planar("b", b, prec, 3, shape=(prec, 2, m), device=dev)
        y = torch.empty((prec, 2, n), dtype=torch.float64, device=dev) if y is None else y
        _check_planar("y", y, prec, 3, shape=(prec, 2, n), device=dev)
        if with_rho and rho is None:
            rho = torch.empty(prec, dtype=torch.float64, device=dev)
        if rho is not None and (not isinstance(rho, torch.Tensor) or rho.dtype != torch.float64 or
                                rho.numel() != prec or rho.device != dev or not rho.is_contiguous()):
            raise ValueError("rho must be a contiguous float64 tensor of %d limbs on %s" % (prec, dev))
    else:
        y = rho = None
    nwork = _lib.workspace_size(m, n, prec, _lib.MGS_OP_QR)
    work = workspace(m, n, prec, _lib.MGS_OP_QR, dev) if work is None else work
    _check_work(work, nwork, dev)
    nwork = work.numel() * work.element_size()
    if schedule is None:
        st = _lib.lib().mgs_qr(m, n, prec, _ptr(A), m, _ptr(Q), m, _ptr(R), n, _ptr(b), _ptr(y),
                               _ptr(rho), _ptr(work), nwork, _ptr(info), _stream(A))
        _lib.check("mgs_qr", st)
    else:
        st = _lib.lib().mgs_qr_schedule(m, n, prec, _ptr(A), m, _ptr(Q), m, _ptr(R), n, _ptr(b), _ptr(y),
                                        _ptr(rho), _ptr(work), nwork, _ptr(info), _lib.SCHEDULES[schedule],
                                        _stream(A))
        _lib.check("mgs_qr_schedule", st)
    return dict(Q=Q, R=R, y=y, rho=rho, info=info)


def mgs_qr_noalloc(A, b=None, *, Q=None, R=None, y=None, rho=None, info=None, with_rho=True):
    """mgs_qr without a workspace argument (mgs_qr_noalloc): the library's
    fixed device array serves as workspace.  Calls that may overlap in time
    on one GPU race on that array; serialise them."""
    _check_planar("A", A, ndim=4)
    prec, _, n, m = A.shape
    dev = A.device
    Q = torch.empty_like(A) if Q is None else Q
    _check_planar("Q", Q, prec, 4, shape=A.shape, device=dev)
    R = torch.empty((prec, 2, n, n), dtype=torch.float64, device=dev) if R is None else R
    _check_planar("R", R, prec, 4, shape=(prec, 2, n, n), device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev) if info is None else info
    _check_info(info, dev)
    if b is not None:
        _check_planar("b", b, prec, 3, shape=(prec, 2, m), device=dev)
        y = torch.empty((prec, 2, n), dtype=torch.float64, device=dev) if y is None else y
        _check_planar("y", y, prec, 3, shape=(prec, 2, n), device=dev)
        if with_rho and rho is None:
            rho = torch.empty(prec, dtype=torch.float64, device=dev)
        if rho is not None and (not isinstance(rho, torch.Tensor) or rho.dtype != torch.float64 or
                                rho.numel() != prec or rho.device != dev or not rho.is_contiguous()):
            raise ValueError("rho must be a contiguous float64 tensor of %d limbs on %s" % (prec, dev))
    else:
        y = rho = None
    st = _lib.lib().mgs_qr_noalloc(m, n, prec, _ptr(A), m, _ptr(Q), m, _ptr(R), n, _ptr(b), _ptr(y), _ptr(rho),
                                   _ptr(info), _stream(A))
    _lib.check("mgs_qr_noalloc", st)
    return dict(Q=Q, R=R, y=y, rho=rho, info=info)


def ls_backsolve(R, y, *, x=None, info=None):
    """x = R^-1 y by the column-oriented back substitution of Figure 3."""
    _check_planar("R", R, ndim=4)
    prec, _, n, ldr = R.shape
    dev = R.device
    if ldr != n:
        raise ValueError("R must be square, got %s" % (tuple(R.shape),))
    _check_planar("y", y, prec, 3, shape=(prec, 2, n), device=dev)
    x = torch.empty_like(y) if x is None else x
    _check_planar("x", x, prec, 3, shape=(prec, 2, n), device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev) if info is None else info
    _check_info(info, dev)
    st = _lib.lib().ls_backsolve(n, prec, _ptr(R), ldr, _ptr(y), _ptr(x), _ptr(info), _stream(R))
    _lib.check("ls_backsolve", st)
    return x, info


def ls_solve(Q, R, b, *, x=None, info=None, work=None):
    """x = R^-1 (Q^H b), Q^H b by sequential MGS projections of b."""
    _check_planar("Q", Q, ndim=4)
    prec, _, n, m = Q.shape
    dev = Q.device
    _check_planar("R", R, prec, 4, shape=(prec, 2, n, n), device=dev)
    _check_planar("b", b, prec, 3, shape=(prec, 2, m), device=dev)
    x = torch.empty((prec, 2, n), dtype=torch.float64, device=dev) if x is None else x
    _check_planar("x", x, prec, 3, shape=(prec, 2, n), device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev) if info is None else info
    _check_info(info, dev)
    nwork = _lib.workspace_size(m, n, prec, _lib.MGS_OP_SOLVE)
    work = workspace(m, n, prec, _lib.MGS_OP_SOLVE, dev) if work is None else work
    _check_work(work, nwork, dev)
    st = _lib.lib().ls_solve(m, n, prec, _ptr(Q), m, _ptr(R), n, _ptr(b), _ptr(x), _ptr(work),
                             work.numel() * work.element_size(), _ptr(info), _stream(Q))
    _lib.check("ls_solve", st)
    return x, info


def lstsq(A, b, *, schedule=None):
    """Least-squares solution of A x = b: MGS on [A b], then back substitution."""
    f = mgs_qr(A, b, schedule=schedule)
    x, info2 = ls_backsolve(f["R"], f["y"])
    f["x"] = x
    f["info_backsolve"] = info2
    return f


def ls_adjoint(A, b, Q, R, x, gx, *, gA=None, gb=None, info=None, work=None):
    """Gradients (gA, gb) of a loss through x = argmin ||b - A x||.

    gx = dL/dRe(x) + i dL/dIm(x) (planar [prec, 2, n]); returns gA, gb in the
    same convention, from the saved MGS factors Q, R (full column rank).
    """
    _check_planar("A", A, ndim=4)
    prec, _, n, m = A.shape
    dev = A.device
    for name, t, shp in (("b", b, (prec, 2, m)), ("Q", Q, (prec, 2, n, m)), ("R", R, (prec, 2, n, n)),
                         ("x", x, (prec, 2, n)), ("gx", gx, (prec, 2, n))):
        _check_planar(name, t, prec, len(shp), shape=shp, device=dev)
    gA = torch.empty_like(A) if gA is None else gA
    gb = torch.empty_like(b) if gb is None else gb
    _check_planar("gA", gA, prec, 4, shape=A.shape, device=dev)
    _check_planar("gb", gb, prec, 3, shape=(prec, 2, m), device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev) if info is None else info
    _check_info(info, dev)
    nwork = _lib.workspace_size(m, n, prec, _lib.MGS_OP_ADJOINT)
    work = workspace(m, n, prec, _lib.MGS_OP_ADJOINT, dev) if work is None else work
    _check_work(work, nwork, dev)
    st = _lib.lib().ls_adjoint(m, n, prec, _ptr(A), m, _ptr(b), _ptr(Q), m, _ptr(R), n, _ptr(x),
                               _ptr(gx), _ptr(gA), m, _ptr(gb), _ptr(work), work.numel() * work.element_size(),
                               _ptr(info), _stream(A))
    _lib.check("ls_adjoint", st)
    return gA, gb, info


def mgs_qr64(A, b=None, *, block=64):
    """FP64 complex blocked MGS of [A b] (the precision form's factorisation).

    A: float64 [2, n, m] planar (re, im) on a HIP device, b: [2, m] or None.
    Returns dict(Q, R, y, info).
    """
    if not isinstance(A, torch.Tensor) or A.dtype != torch.float64 or not A.is_contiguous() or not A.is_cuda:
        raise ValueError("A must be a contiguous float64 tensor on a HIP device")
    if A.dim() != 3 or A.shape[0] != 2:
        raise ValueError("A must have shape [2, n, m], got %s" % (tuple(A.shape),))
    _, n, m = A.shape
    dev = A.device
    if b is not None:
        if not isinstance(b, torch.Tensor) or b.dtype != torch.float64 or not b.is_contiguous() or not b.is_cuda \
                or tuple(b.shape) != (2, m):
            raise ValueError("b must be a contiguous float64 [2, m] tensor on the device of A")
    Q = torch.empty_like(A)
    R = torch.empty((2, n, n), dtype=torch.float64, device=dev)
    y = torch.empty((2, n), dtype=torch.float64, device=dev) if b is not None else None
    info = torch.empty(1, dtype=torch.int32, device=dev)
    work = workspace(m, n, 1, _lib.MGS_OP_QR64, dev)
    st = _lib.lib().mgs_qr64(m, n, _ptr(A), m, _ptr(b), _ptr(Q), m, _ptr(R), n, _ptr(y), block, _ptr(work),
                             work.numel() * 8, _ptr(info), _stream(A))
    _lib.check("mgs_qr64", st)
    return dict(Q=Q, R=R, y=y, info=info)


def refine_lstsq(A, b, *, tol=None, max_iter=20, x=None, work=None):
    """Precision form: FP64 blocked-MGS factorisation (panels of 64, trailing
    products on matrix cores) and dd / qd iterative refinement of x.

    Returns dict(x, iters, err_est, info) of device tensors; info 0 converged,
    k > 0 bad column k, -1 stagnated, -2 max_iter reached.
    """
    _check_planar("A", A, ndim=4)
    prec, _, n, m = A.shape
    dev = A.device
    _check_planar("b", b, prec, 3, shape=(prec, 2, m), device=dev)
    if tol is None:
        tol = 2.0 ** -104 if prec == 2 else 2.0 ** -209
    x = torch.empty((prec, 2, n), dtype=torch.float64, device=dev) if x is None else x
    _check_planar("x", x, prec, 3, shape=(prec, 2, n), device=dev)
    iters = torch.zeros(1, dtype=torch.int32, device=dev)
    err = torch.zeros(1, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    nwork = _lib.workspace_size(m, n, prec, _lib.MGS_OP_REFINE)
    work = workspace(m, n, prec, _lib.MGS_OP_REFINE, dev) if work is None else work
    _check_work(work, nwork, dev)
    st = _lib.lib().mgs_refine_solve(m, n, prec, _ptr(A), m, _ptr(b), _ptr(x), 64, float(tol), int(max_iter),
                                     _ptr(iters), _ptr(err), _ptr(work), work.numel() * work.element_size(),
                                     _ptr(info), _stream(A))
    _lib.check("mgs_refine_solve", st)
    return dict(x=x, iters=iters, err_est=err, info=info)


def lstsq_batched(A, b=None, *, Q=None, R=None, y=None, x=None, rho=None, info=None, with_y=False,
                  with_rho=False):
    """`batch` independent systems: MGS of each [A_s b_s] (Figure 1, Equation
    (1)) and, when b is given, the back substitution (Figure 3), one
    workgroup per system (mgs_lstsq_batched).

    A: [batch, prec, 2, n, m], b: [batch, prec, 2, m] or None.  Returns
    dict(Q, R, y, x, rho, info) (info: one int32 per system); Q may be A
    itself to factor in place.
    """
    if not isinstance(A, torch.Tensor) or A.dim() != 5:
        raise ValueError("A must be a [batch, prec, 2, n, m] tensor")
    batch, prec, two, n, m = A.shape
    dev = A.device
    if not A.is_contiguous() or A.dtype != torch.float64 or not A.is_cuda or two != 2:
        raise ValueError("A must be a contiguous float64 [batch, prec, 2, n, m] tensor on a HIP device")

    def out(name, t, shape):
        t = torch.empty(shape, dtype=torch.float64, device=dev) if t is None else t
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_contiguous() or \
                t.device != dev or tuple(t.shape) != tuple(shape):
            raise ValueError("%s must be a contiguous float64 tensor of shape %s on %s" % (name, tuple(shape), dev))
        return t

    Q = out("Q", Q, A.shape)
    R = out("R", R, (batch, prec, 2, n, n))
    info = torch.empty(batch, dtype=torch.int32, device=dev) if info is None else info
    if not isinstance(info, torch.Tensor) or info.dtype != torch.int32 or info.numel() != batch or \
            info.device != dev or not info.is_contiguous():
        raise ValueError("info must be a contiguous int32 tensor of %d entries on %s" % (batch, dev))
    if b is not None:
        b = out("b", b, (batch, prec, 2, m))
        x = out("x", x, (batch, prec, 2, n))
        y = out("y", y, (batch, prec, 2, n)) if (with_y or y is not None) else None
        rho = out("rho", rho, (batch, prec)) if (with_rho or rho is not None) else None
    else:
        x = y = rho = None
    st = _lib.lib().mgs_lstsq_batched(batch, m, n, prec, _ptr(A), m, _ptr(b), _ptr(Q), m, _ptr(R), n, _ptr(y),
                                      _ptr(x), _ptr(rho), _ptr(info), _stream(A))
    _lib.check("mgs_lstsq_batched", st)
    return dict(Q=Q, R=R, y=y, x=x, rho=rho, info=info)


def set_jitter(seed):
    """Race checks (mgs_set_jitter): seed != 0 adds pseudo-random pauses to
    the kernels that synchronise across waves or workgroups; results must
    stay bitwise the same.  0 switches it off."""
    _lib.lib().mgs_set_jitter(int(seed) & 0xFFFFFFFF)


class PolySystem:
    """A polynomial system on the card (Section 7: transferred once):
    vars, exps int32 [neq, nmon, nvpm], coef float64 [prec, 2, neq, nmon]
    (f_e = sum_m c_em prod_t x_{v_emt}^{d_emt}); nvar variables."""

    def __init__(self, vars, exps, coef, nvar, device):
        self.vars = torch.as_tensor(vars, dtype=torch.int32).contiguous().to(device)
        self.exps = torch.as_tensor(exps, dtype=torch.int32).contiguous().to(device)
        self.coef = torch.as_tensor(coef, dtype=torch.float64).contiguous().to(device)
        if self.vars.dim() != 3 or self.exps.shape != self.vars.shape:
            raise ValueError("vars and exps must both be [neq, nmon, nvpm]")
        self.neq, self.nmon, self.nvpm = self.vars.shape
        self.prec = self.coef.shape[0]
        if tuple(self.coef.shape) != (self.prec, 2, self.neq, self.nmon):
            raise ValueError("coef must be [prec, 2, neq, nmon], got %s" % (tuple(self.coef.shape),))
        self.nvar = int(nvar)
        self.device = self.coef.device

    def _points(self, x):
        if not isinstance(x, torch.Tensor) or x.dim() != 4 or x.dtype != torch.float64 or \
                not x.is_contiguous() or x.device != self.device or \
                tuple(x.shape[1:]) != (self.prec, 2, self.nvar):
            raise ValueError("x must be a contiguous float64 [batch, %d, 2, %d] tensor on %s"
                             % (self.prec, self.nvar, self.device))
        return x.shape[0]


def poly_eval(system, x, *, J=None, F=None):
    """f(x) and the Jacobian at batch points x [batch, prec, 2, nvar]
    (mgs_poly_eval).  Returns (J [batch, prec, 2, nvar, neq], F [batch,
    prec, 2, neq])."""
    batch = system._points(x)
    shapeJ = (batch, system.prec, 2, system.nvar, system.neq)
    shapeF = (batch, system.prec, 2, system.neq)
    J = torch.empty(shapeJ, dtype=torch.float64, device=x.device) if J is None else J
    F = torch.empty(shapeF, dtype=torch.float64, device=x.device) if F is None else F
    for name, t, shp in (("J", J, shapeJ), ("F", F, shapeF)):
        if t.dtype != torch.float64 or not t.is_contiguous() or t.device != x.device or tuple(t.shape) != shp:
            raise ValueError("%s must be a contiguous float64 tensor of shape %s on %s" % (name, shp, x.device))
    st = _lib.lib().mgs_poly_eval(batch, system.neq, system.nvar, system.nmon, system.nvpm, system.prec,
                                  _ptr(system.vars), _ptr(system.exps), _ptr(system.coef), _ptr(x), _ptr(J),
                                  _ptr(F), _stream(x))
    _lib.check("mgs_poly_eval", st)
    return J, F


def newton_batched(system, x, iters, *, dnorm=True, info=None, work=None):
    """`iters` Newton steps at each point of x [batch, prec, 2, nvar],
    updated in place (mgs_newton_batched: evaluation, MGS on [J -f], back
    substitution, update, all on the card).  Returns dict(x, dnorm [iters,
    batch] or None, info [batch])."""
    batch = system._points(x)
    dev = x.device
    nbytes = _lib.newton_workspace_size(batch, system.neq, system.nvar, system.prec)
    work = torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device=dev) if work is None else work
    _check_work(work, nbytes, dev)
    info = torch.empty(max(batch, 1), dtype=torch.int32, device=dev) if info is None else info
    if not isinstance(info, torch.Tensor) or info.dtype != torch.int32 or info.numel() < batch or \
            info.device != dev or not info.is_contiguous():
        raise ValueError("info must be a contiguous int32 tensor of >= %d entries on %s" % (batch, dev))
    dn = torch.empty((max(iters, 1), max(batch, 1)), dtype=torch.float64, device=dev) if dnorm else None
    st = _lib.lib().mgs_newton_batched(batch, system.neq, system.nvar, system.nmon, system.nvpm, system.prec,
                                       _ptr(system.vars), _ptr(system.exps), _ptr(system.coef), _ptr(x),
                                       int(iters), _ptr(dn), _ptr(work), work.numel() * work.element_size(),
                                       _ptr(info), _stream(x))
    _lib.check("mgs_newton_batched", st)
    return dict(x=x, dnorm=None if dn is None else dn[:iters, :batch], info=info[:batch])


class LstsqFn(torch.autograd.Function):
    """x = argmin ||b - A x|| by MGS on [A b] and back substitution, with the
    hand-written adjoint as its backward.

    Tensors are planar dd / qd ([prec, 2, ...] float64 on the GPU); the
    gradients returned are extended-precision VALUES in the same layout (the
    limb planes encode one number per entry, they are not per-limb partial
    derivatives), in the convention dL/dRe + i dL/dIm.
    """

    @staticmethod
    def forward(ctx, A, b):
        f = mgs_qr(A.detach(), b.detach())
        x, _ = ls_backsolve(f["R"], f["y"])
        ctx.save_for_backward(A.detach(), b.detach(), f["Q"], f["R"], x)
        ctx.info = (f["info"],)
        return x

    @staticmethod
    def backward(ctx, gx):
        A, b, Q, R, x = ctx.saved_tensors
        gA, gb, _ = ls_adjoint(A, b, Q, R, x, gx.contiguous())
        return gA, gb
