"""Exact rational helpers for pinning the oracle (fractions.Fraction)."""
import math
from fractions import Fraction as F

import numpy as np

# Conservative unit roundoffs per precision (limbs): FP64, dd, qd.
EPS = {1: 2.0 ** -53, 2: 2.0 ** -104, 4: 2.0 ** -209}


def fval(limbs):
    """Exact value of a number given by its limbs."""
    return sum((F(float(v)) for v in limbs), F(0))


def cmat(X):
    """Planar (L,2,n,m) -> list of columns of exact complex pairs (re, im)."""
    L, _, n, m = X.shape
    return [[(fval(X[:, 0, j, i]), fval(X[:, 1, j, i])) for i in range(m)] for j in range(n)]


def cvec(x):
    L, _, m = x.shape
    return [(fval(x[:, 0, i]), fval(x[:, 1, i])) for i in range(m)]


def cmul(a, b):
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def cmulc(a, b):
    """conj(a) * b."""
    return (a[0] * b[0] + a[1] * b[1], a[0] * b[1] - a[1] * b[0])


def cadd(a, b):
    return (a[0] + b[0], a[1] + b[1])


def csub(a, b):
    return (a[0] - b[0], a[1] - b[1])


def cabs(a):
    return math.sqrt(float(a[0] * a[0] + a[1] * a[1]))


def vnorm(v):
    return math.sqrt(float(sum(a[0] * a[0] + a[1] * a[1] for a in v)))


def matvec(cols, x):
    """sum_j cols[j] * x[j]."""
    m = len(cols[0])
    out = [(F(0), F(0))] * m
    for j, c in enumerate(cols):
        out = [cadd(o, cmul(c[i], x[j])) for i, o in enumerate(out)]
    return out


def inner(x, y):
    s = (F(0), F(0))
    for a, b in zip(x, y):
        s = cadd(s, cmulc(a, b))
    return s


def planar_from_exact(cols, L):
    """List of columns of exact complex values -> planar float64 limbs (rounded)."""
    n, m = len(cols), len(cols[0])
    X = np.zeros((L, 2, n, m))
    for j in range(n):
        for i in range(m):
            for p in range(2):
                v = cols[j][i][p]
                for l in range(L):
                    f = float(v)
                    X[l, p, j, i] = f
                    v -= F(f)
    return X


def kappa_eq(A):
    """kappa_2(A D^-1) from the hi limbs, D = column norms."""
    M = (A[0, 0] + 1j * A[0, 1]).T
    M = M / np.linalg.norm(M, axis=0)
    s = np.linalg.svd(M, compute_uv=False)
    return s[0] / s[-1]
