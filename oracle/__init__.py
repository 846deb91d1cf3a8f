"""TEST INFRASTRUCTURE -- the CPU oracle of the complex MGS least-squares solver.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never calls it and shares no code with it.

The oracle is a plain, sequential implementation, in its own double-double
and quad-double arithmetic, of what the paper defines:

* modified Gram-Schmidt QR (Section 3, Figure 1) on the matrix augmented with
  the right-hand side (Section 3, Equation (1)),
* column-oriented back substitution (Section 6, Figure 3),
* least squares by sequential projections of b followed by back substitution,
* the accuracy measure e of Section 4, Equation (2),
* the closed-form adjoint (dL/dA, dL/db) of the least-squares solution for
  L = Re(g^H x) (the differentiation form; not in the paper),
* the precision form (not in the paper): FP64 blocked MGS, then iterative
  refinement with the residual in quad-double,
* a polynomial system's values and Jacobian, and Newton's method with the
  MGS least-squares solve (Section 7: the corrector of a path tracker).

Array layout ("planar"): a complex matrix with ``cols`` columns and leading
dimension ``ld`` in L-limb precision is a float64 array of shape
``(L, 2, cols, ld)``: ``X[l, 0]`` holds limb ``l`` of the real parts and
``X[l, 1]`` limb ``l`` of the imaginary parts, column-major.  A vector is
``(L, 2, len)``.  ``prec`` is the number of limbs: 1 (double), 2 (dd), 4 (qd).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORC_MGS_LIB names another build of the same source (the sanitizer build
# of the tests); the default is the in-tree library.
_SO = os.environ.get("ORC_MGS_LIB") or os.path.join(_HERE, "liborc_mgs.so")
_SRC = [os.path.join(_HERE, "orc_mgs.cpp"), os.path.join(_HERE, "orc_arith.hpp")]

CXXFLAGS = ["-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-march=x86-64-v3",
            "-fopenmp", "-fPIC", "-shared", "-Wall"]


SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def build(force=True, out=None, sanitize=False):
    """Compile the oracle library with g++ (in place unless ``out`` names
    another file; ``sanitize`` adds AddressSanitizer and UBSan)."""
    so = out or _SO
    if not force and os.path.exists(so):
        return so
    tmp = so + ".tmp%d" % os.getpid()
    cmd = ["g++"] + CXXFLAGS + (SANITIZE if sanitize else []) + ["-o", tmp, _SRC[0]]
    subprocess.run(cmd, check=True)
    os.replace(tmp, so)
    return so


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I = ctypes.c_int
        L.orc_mgs.argtypes = [I, I, I, P, I, P, P, I, P, I, P, P, I]
        L.orc_backsolve.argtypes = [I, I, P, I, P, P]
        L.orc_ls_solve.argtypes = [I, I, I, P, I, P, I, P, P]
        L.orc_arith.argtypes = [I, I, I, P, P, P]
        L.orc_errors.argtypes = [I, I, I, P, I, P, I, P, I, P, I, P, I]
        L.orc_adjoint.argtypes = [I, I, I, P, I, P, P, P, P, P, I]
        L.orc_emax_batch.argtypes = [I, I, I, I, P, I, P, I, P, I, P, I]
        L.orc_refine.argtypes = [I, I, I, P, I, P, P, P, I, ctypes.c_double, I, P, P, I]
        L.orc_poly_eval.argtypes = [I, I, I, I, I, P, P, P, P, P, P]
        L.orc_newton.argtypes = [I, I, I, I, I, P, P, P, P, I, P]
        for f in (L.orc_mgs, L.orc_backsolve, L.orc_ls_solve, L.orc_arith, L.orc_errors, L.orc_adjoint,
                  L.orc_emax_batch, L.orc_refine, L.orc_poly_eval, L.orc_newton):
            f.restype = I
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def mgs(A, b=None, nthreads=0):
    """MGS QR of A (planar (L,2,n,m)), augmented with b (planar (L,2,m)) if given.

    Returns dict(Q, R, y, rho, info): Q (L,2,n,m), R (L,2,n,n) with zero lower
    triangle, y (L,2,n) = Q^H b and rho (L,) = norm of the projected b
    (the z of Equation (1)) when b is given.
    """
    A = _c(A)
    L, two, n, m = A.shape
    assert two == 2
    Q = np.zeros_like(A)
    R = np.zeros((L, 2, n, n))
    y = rho = None
    if b is not None:
        b = _c(b)
        assert b.shape == (L, 2, m)
        y = np.zeros((L, 2, n))
        rho = np.zeros(L)
    info = lib().orc_mgs(L, m, n, _p(A), m, _p(b), _p(Q), m, _p(R), n, _p(y), _p(rho), int(nthreads))
    if info < 0:
        raise ValueError("orc_mgs argument error %d" % info)
    return dict(Q=Q, R=R, y=y, rho=rho, info=info)


def backsolve(R, y):
    """Solve R x = y (Figure 3); R planar (L,2,n,n), y planar (L,2,n)."""
    R = _c(R)
    y = _c(y)
    L, _, n, _ = R.shape
    x = np.zeros((L, 2, n))
    info = lib().orc_backsolve(L, n, _p(R), n, _p(y), _p(x))
    if info < 0:
        raise ValueError("orc_backsolve argument error %d" % info)
    return x, info


def ls_solve(Q, R, b):
    """x = R^{-1} (Q^H b), Q^H b by sequential MGS projections of b."""
    Q = _c(Q)
    R = _c(R)
    b = _c(b)
    L, _, n, m = Q.shape
    x = np.zeros((L, 2, n))
    info = lib().orc_ls_solve(L, m, n, _p(Q), m, _p(R), n, _p(b), _p(x))
    if info < 0:
        raise ValueError("orc_ls_solve argument error %d" % info)
    return x, info


OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3, "sqrt": 4}


def arith(prec, op, a, b=None):
    """Elementwise real dd/qd arithmetic: a, b of shape (count, prec) limbs."""
    a = _c(a).reshape(-1, prec)
    b = a if b is None else _c(b).reshape(-1, prec)
    out = np.zeros_like(a)
    rc = lib().orc_arith(prec, OPS[op], a.shape[0], _p(a), _p(b), _p(out))
    if rc != 0:
        raise ValueError("orc_arith error %d" % rc)
    return out


def errors(A, Q, R, cols=None, nthreads=0):
    """(e_max of Equation (2), max_j ||a_j - Q r_j||/||a_j||, max |Q^H Q - I|).

    Every difference is formed exactly (expansion arithmetic) and rounded once.
    ``cols`` restricts the measures to the listed columns j.
    """
    A, Q, R = _c(A), _c(Q), _c(R)
    L, _, n, m = A.shape
    out = np.zeros(3)
    cj = None if cols is None else np.ascontiguousarray(cols, dtype=np.int32)
    lib().orc_errors(L, m, n, _p(A), m, _p(Q), m, _p(R), n, _p(cj), 0 if cj is None else len(cj),
                     _p(out), int(nthreads))
    return out


def emax_batch(A, Q, R, nthreads=0):
    """e_max of Equation (2) for each system of a batch: A, Q (count,L,2,n,m),
    R (count,L,2,n,n); evaluated exactly as by ``errors``, one system per
    thread.  Returns a float64 array of count values."""
    A, Q, R = _c(A), _c(Q), _c(R)
    count, L, _, n, m = A.shape
    out = np.zeros(count)
    rc = lib().orc_emax_batch(L, count, m, n, _p(A), m, _p(Q), m, _p(R), n, _p(out), int(nthreads))
    if rc != 0:
        raise ValueError("orc_emax_batch error %d" % rc)
    return out


def refine(A, b, block=64, tol=None, max_iter=30, nthreads=0):
    """The precision form: FP64 blocked MGS of [fl64(A) fl64(b)] (panels of
    ``block``), x0 = R^-1 y, then refinement with the residual in qd and the
    FP64 correction solve replaying the panels' projections.

    Returns dict(x, x0, iters, err_est, info): info 0 converged, -1
    stagnated, -2 max_iter reached, k > 0 bad column k.
    """
    A, b = _c(A), _c(b)
    L, _, n, m = A.shape
    if tol is None:
        tol = 2.0 ** -104 if L == 2 else 2.0 ** -209
    x = np.zeros((L, 2, n))
    x0 = np.zeros((L, 2, n))
    it = ctypes.c_int(0)
    est = ctypes.c_double(0.0)
    info = lib().orc_refine(L, m, n, _p(A), m, _p(b), _p(x), _p(x0), int(block), float(tol), int(max_iter),
                            ctypes.byref(it), ctypes.byref(est), int(nthreads))
    if info < -2:
        raise ValueError("orc_refine argument error %d" % info)
    return dict(x=x, x0=x0, iters=it.value, err_est=est.value, info=info)


def _sys(system):
    v = np.ascontiguousarray(system["vars"], dtype=np.int32)
    d = np.ascontiguousarray(system["exps"], dtype=np.int32)
    c = _c(system["coef"])
    neq, nmon, nvpm = v.shape
    return v, d, c, neq, nmon, nvpm, int(system["nvar"])


def poly_eval(system, x):
    """F = f(x) (L,2,neq) and the Jacobian J (L,2,nvar,neq) of a polynomial
    system: dict(vars, exps [neq,nmon,nvpm], coef (L,2,neq,nmon), nvar)."""
    v, d, c, neq, nmon, nvpm, nvar = _sys(system)
    x = _c(x)
    L = x.shape[0]
    F = np.zeros((L, 2, neq))
    J = np.zeros((L, 2, nvar, neq))
    rc = lib().orc_poly_eval(L, neq, nvar, nmon, nvpm, _p(v), _p(d), _p(c), _p(x), _p(F), _p(J))
    if rc != 0:
        raise ValueError("orc_poly_eval error %d" % rc)
    return F, J


def newton(system, x0, iters):
    """`iters` Newton steps from x0 with the MGS least-squares solve of
    J d = -F; returns (x, correction norms)."""
    v, d, c, neq, nmon, nvpm, nvar = _sys(system)
    x = _c(x0).copy()
    L = x.shape[0]
    dn = np.zeros(max(iters, 1))
    rc = lib().orc_newton(L, neq, nvar, nmon, nvpm, _p(v), _p(d), _p(c), _p(x), int(iters), _p(dn))
    if rc != 0:
        raise ValueError("orc_newton error %d" % rc)
    return x, dn[:iters]


def adjoint(A, b, g, nthreads=0):
    """Closed-form adjoint of x = argmin ||b - A x|| for L = Re(g^H x).

    Returns (gA (L,2,n,m), gb (L,2,m), x (L,2,n)), gradients in the
    convention dL/dRe + i dL/dIm.
    """
    A, b, g = _c(A), _c(b), _c(g)
    L, _, n, m = A.shape
    gA = np.zeros_like(A)
    gb = np.zeros((L, 2, m))
    x = np.zeros((L, 2, n))
    info = lib().orc_adjoint(L, m, n, _p(A), m, _p(b), _p(g), _p(gA), _p(gb), _p(x), int(nthreads))
    if info != 0:
        raise ValueError("orc_adjoint failed with %d" % info)
    return gA, gb, x
