"""Parity helpers: differences of dd / qd arrays and the error measures.

Differences are formed from the limbs with error-free TwoSum distillation
(SumK, Ogita-Rump-Oishi), so that two extended-precision arrays that agree
to 60 digits still give an accurate difference; norms are then FP64.
"""
import numpy as np


def _two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def diff(X, Y):
    """FP64 value of X - Y for planar arrays with the limb axis first."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    L = X.shape[0]
    t = []
    for l in range(L - 1, -1, -1):  # smallest limbs first
        t.append(X[l].copy())
        t.append(-Y[l])
    for _ in range(8):
        for i in range(len(t) - 1):
            t[i + 1], t[i] = _two_sum(t[i + 1], t[i])
    return t[-1] + sum(t[:-1])


def value(X):
    """FP64 rounding of a planar array (sum of limbs)."""
    return diff(X, np.zeros_like(X))


def col_norms(A):
    """||a_j||_2 from the hi limbs of planar A (L, 2, n, m)."""
    return np.sqrt(np.sum(A[0, 0] ** 2 + A[0, 1] ** 2, axis=1))


def kappa_eff(A):
    """kappa_2(A D^-1), D the column norms, from the hi limbs."""
    M = (A[0, 0] + 1j * A[0, 1]).T
    M = M / np.linalg.norm(M, axis=0)
    s = np.linalg.svd(M, compute_uv=False)
    return float(s[0] / s[-1]), M


def errors(A, Qg, Rg, Qo, Ro, xg=None, xo=None, rho=None):
    """err_Q, err_R (column relative), err_x (equilibrated), kappa, kappa_LS."""
    dQ = diff(Qg, Qo)  # (2, n, m)
    err_q = float(np.max(np.sqrt(np.sum(dQ[0] ** 2 + dQ[1] ** 2, axis=1))))
    dR = diff(Rg, Ro)
    nA = col_norms(A)
    err_r = float(np.max(np.sqrt(np.sum(dR[0] ** 2 + dR[1] ** 2, axis=1)) / nA))
    kap, Ms = kappa_eff(A)
    out = dict(err_q=err_q, err_r=err_r, kappa=kap)
    if xg is not None:
        dx = diff(xg, xo)
        xv = value(xo)
        num = np.sqrt(np.sum((nA * dx[0]) ** 2 + (nA * dx[1]) ** 2))
        den = np.sqrt(np.sum((nA * xv[0]) ** 2 + (nA * xv[1]) ** 2))
        out["err_x"] = float(num / den)
        r = 0.0 if rho is None else abs(float(value(rho[:, None])[0]))
        nAs = np.linalg.norm(Ms, 2)
        out["kappa_ls"] = kap + kap * kap * r / (nAs * den)
    return out


# Parity bars per precision: about 2^12 units of the working precision
# (FP64 2^-53, dd 2^-104, qd 2^-209), times max(1, kappa / 100) at use.
TAU = {1: 5e-13, 2: 1e-28, 4: 1e-58}


def assert_parity(e, prec, what=("err_q", "err_r", "err_x")):
    tau = TAU[prec]
    for k in what:
        if k not in e:
            continue
        kap = e["kappa_ls"] if k == "err_x" else e["kappa"]
        tol = tau * max(1.0, kap / 100.0)
        assert e[k] <= tol, "%s = %.3e exceeds %.3e (kappa %.3e)" % (k, e[k], tol, kap)
