"""Pins of the oracle's closed-form least-squares adjoint.

For L = Re(g^H x), x = argmin ||b - A x||, the gradient (dL/dRe + i dL/dIm)
is pinned against
* central finite differences of L computed from qd least-squares solves,
  with L and the difference quotient evaluated in exact rational
  arithmetic (step h = 2^-70: truncation and rounding error near 1e-40);
* the exact identities Re<dL/dA, A> = -L (x(tA) = x/t) and
  Re<dL/db, b> = L (x is linear in b);
* the square case, where the residual vanishes and dL/dA = -(dL/db) x^H.
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from paper_1210_0800_amd import inputs
from tests._exact import EPS, cvec, fval, kappa_eq


def _problem(m, n, seed, L=4):
    g0 = inputs.rng(61, seed, 0)
    A = np.zeros((L, 2, n, m))
    A[0] = g0.uniform(0.1, 1.0, (2, n, m)) * g0.choice([-1.0, 1.0], (2, n, m))
    b = np.zeros((L, 2, m))
    b[0] = g0.uniform(-1, 1, (2, m))
    g = np.zeros((L, 2, n))
    g[0] = g0.uniform(-1, 1, (2, n))
    return A, b, g


def _loss(A, b, g):
    """Exact L = Re(g^H x) of the qd least-squares solution."""
    o = oracle.mgs(A, b)
    assert o["info"] == 0
    x, _ = oracle.backsolve(o["R"], o["y"])
    xs, gs = cvec(x), cvec(g)
    return sum(gv[0] * xv[0] + gv[1] * xv[1] for gv, xv in zip(gs, xs))


def _perturb(X, idx, part, h):
    Y = X.copy()
    sl = (slice(None), part) + idx
    limbs = inputs.normalize([Y[(l, part) + idx] * np.ones(1) for l in range(Y.shape[0])] + [np.array([h])])
    for l in range(Y.shape[0]):
        Y[(l, part) + idx] = limbs[l][0]
    assert fval(Y[sl]) == fval(X[sl]) + F(h)
    return Y


@pytest.mark.parametrize("m,n,seed", [(10, 6, 0), (7, 7, 1), (12, 4, 2)])
def test_adjoint_matches_qd_central_differences(m, n, seed):
    A, b, g = _problem(m, n, seed)
    gA, gb, x = oracle.adjoint(A, b, g)
    h = 2.0 ** -70
    rng = np.random.default_rng([1210, m, n, seed])
    scale = max(np.max(np.abs(gA[0])), np.max(np.abs(gb[0])))
    for _ in range(10):
        i, j, part = int(rng.integers(0, m)), int(rng.integers(0, n)), int(rng.integers(0, 2))
        Lp = _loss(_perturb(A, (j, i), part, h), b, g)
        Lm = _loss(_perturb(A, (j, i), part, -h), b, g)
        fd = (Lp - Lm) / (2 * F(h))
        ex = fval(gA[:, part, j, i])
        assert abs(float(fd - ex)) <= 1e-35 * scale, (i, j, part, float(fd), float(ex))
    for _ in range(6):
        i, part = int(rng.integers(0, m)), int(rng.integers(0, 2))
        Lp = _loss(A, _perturb(b, (i,), part, h), g)
        Lm = _loss(A, _perturb(b, (i,), part, -h), g)
        fd = (Lp - Lm) / (2 * F(h))
        ex = fval(gb[:, part, i])
        assert abs(float(fd - ex)) <= 1e-35 * scale, (i, part, float(fd), float(ex))


@pytest.mark.parametrize("L", [2, 4])
@pytest.mark.parametrize("m,n", [(9, 5), (6, 6), (20, 3)])
def test_adjoint_identities(L, m, n):
    p = inputs.random_problem(L, m, n, seed=m + n, config=62)
    A, b = p["A"], p["b"]
    g = inputs.random_complex(inputs.rng(62, m + n, 3), (n,), L)
    gA, gb, x = oracle.adjoint(A, b, g)
    xs, gs = cvec(x), cvec(g)
    Lval = sum(gv[0] * xv[0] + gv[1] * xv[1] for gv, xv in zip(gs, xs))
    # Re <gA, A> = sum Re(conj(gA_ij) A_ij)
    ip = F(0)
    for j in range(n):
        for i in range(m):
            ip += fval(gA[:, 0, j, i]) * fval(A[:, 0, j, i]) + fval(gA[:, 1, j, i]) * fval(A[:, 1, j, i])
    ipb = sum(fval(gb[:, 0, i]) * fval(b[:, 0, i]) + fval(gb[:, 1, i]) * fval(b[:, 1, i]) for i in range(m))
    kap = kappa_eq(A)
    nA = math.sqrt(float(sum(fval(A[:, p, j, i]) ** 2 for p in range(2) for j in range(n) for i in range(m))))
    ngA = math.sqrt(float(sum(fval(gA[:, p, j, i]) ** 2 for p in range(2) for j in range(n) for i in range(m))))
    tol = 100 * kap * kap * m * EPS[L]
    assert abs(float(ip + Lval)) <= tol * nA * ngA
    ngb = math.sqrt(float(sum(fval(gb[:, p, i]) ** 2 for p in range(2) for i in range(m))))
    nb = math.sqrt(float(sum(fval(b[:, p, i]) ** 2 for p in range(2) for i in range(m))))
    assert abs(float(ipb - Lval)) <= tol * nb * ngb


@pytest.mark.parametrize("L", [2, 4])
def test_square_case_has_no_residual_term(L):
    p = inputs.random_problem(L, 8, 8, seed=3, config=63)
    g = inputs.random_complex(inputs.rng(63, 3, 3), (8,), L)
    gA, gb, x = oracle.adjoint(p["A"], p["b"], g)
    xs, bs = cvec(x), cvec(gb)
    kap = kappa_eq(p["A"])
    worst = 0.0
    scale = 0.0
    for j in range(8):
        for i in range(8):
            # gA_ij + gb_i conj(x_j) = 0
            re = fval(gA[:, 0, j, i]) + bs[i][0] * xs[j][0] + bs[i][1] * xs[j][1]
            im = fval(gA[:, 1, j, i]) + bs[i][1] * xs[j][0] - bs[i][0] * xs[j][1]
            worst = max(worst, math.hypot(float(re), float(im)))
            scale = max(scale, math.hypot(float(fval(gA[:, 0, j, i])), float(fval(gA[:, 1, j, i]))))
    assert worst <= 100 * kap * kap * 8 * EPS[L] * scale
