"""Pins of the oracle's MGS QR, least squares and back substitution.

What the paper fixes (Section 3, Figure 1 and Equation (1); Section 6,
Figure 3): A = QR with Q^H Q = I and R upper triangular; MGS on [A b] gives
y = Q^H b and the residual norm z with ||b - Ax||^2 = ||Rx - y||^2 + z^2; x
solves R x = y and minimises ||b - Ax||.  With a real positive diagonal of R
the factorisation and the least-squares solution are unique, so the checks
below -- all evaluated in exact rational arithmetic -- pin the oracle to the
mathematics, not to itself.
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from paper_1210_0800_amd import inputs
from tests._exact import (EPS, cadd, cmat, cmul, cmulc, csub, cvec, fval, inner, kappa_eq,
                          planar_from_exact, vnorm)


def _solve(A, b):
    o = oracle.mgs(A, b)
    assert o["info"] == 0
    x, info = oracle.backsolve(o["R"], o["y"])
    assert info == 0
    return o, x


# ---------------------------------------------------------------- invariants --
@pytest.mark.parametrize("L", [1, 2, 4])
@pytest.mark.parametrize("m,n", [(1, 1), (3, 2), (5, 5), (8, 6), (8, 8)])
def test_exact_invariants(L, m, n):
    p = inputs.random_problem(L, m, n, seed=m * 10 + n, config=90)
    A, b = p["A"], p["b"]
    o, x = _solve(A, b)
    eps = EPS[L]
    kap = kappa_eq(A)
    Ac, Qc, Rc = cmat(A), cmat(o["Q"]), cmat(o["R"])
    bc, yc, xc = cvec(b), cvec(o["y"]), cvec(x)
    # R upper triangular, real positive diagonal (exact zeros)
    for j in range(n):
        for i in range(j + 1, n):
            assert Rc[j][i] == (0, 0)
        assert Rc[j][j][1] == 0 and Rc[j][j][0] > 0
    # backward error of the factorisation: ||a_j - Q r_j|| / ||a_j||
    for j in range(n):
        res = list(Ac[j])
        for l in range(j + 1):
            res = [csub(res[i], cmul(Qc[l][i], Rc[j][l])) for i in range(m)]
        assert vnorm(res) <= 4 * m * eps * vnorm(Ac[j]), j
    # orthogonality ||Q^H Q - I||
    for l in range(n):
        for j in range(n):
            g = inner(Qc[l], Qc[j])
            if l == j:
                g = (g[0] - 1, g[1])
            assert math.hypot(float(g[0]), float(g[1])) <= 10 * kap * n * eps
    # normal equations A^H (b - A x) = 0
    r = list(bc)
    for j in range(n):
        r = [csub(r[i], cmul(Ac[j][i], xc[j])) for i in range(m)]
    nA = math.sqrt(sum(vnorm(c) ** 2 for c in Ac))
    ne = math.sqrt(sum(abs(complex(*map(float, inner(Ac[j], r)))) ** 2 for j in range(n)))
    assert ne <= 10 * m * eps * kap * nA * (nA * vnorm(xc) + vnorm(bc))
    # Equation (1): ||b - Ax||^2 = ||Rx - y||^2 + z^2
    rho = fval(o["rho"])
    Rx = [(F(0), F(0))] * n
    for k in range(n):
        Rx = [cadd(Rx[i], cmul(Rc[k][i], xc[k])) for i in range(n)]
    lhs = sum(v[0] * v[0] + v[1] * v[1] for v in r)
    rhs = sum((a[0] - c[0]) ** 2 + (a[1] - c[1]) ** 2 for a, c in zip(Rx, yc)) + rho * rho
    assert abs(float(lhs - rhs)) <= 10 * m * eps * float(sum(v[0] ** 2 + v[1] ** 2 for v in bc))
    # y = Q^H b up to the conditioning of Q
    for k in range(n):
        d = csub(yc[k], inner(Qc[k], bc))
        assert math.hypot(float(d[0]), float(d[1])) <= 20 * kap * m * n * eps * vnorm(bc)


# ------------------------------------------- the error measures themselves --
def _exact_measures(A, Q, R):
    """(e_max of Equation (2), max_j ||a_j - Q r_j|| / ||a_j||, max |Q^H Q - I|)
    from exact rational arithmetic on the limbs, rounded at the end."""
    Ac, Qc, Rc = cmat(A), cmat(Q), cmat(R)
    n, m = len(Ac), len(Ac[0])
    emax = bw = orth = 0.0
    for j in range(n):
        res = list(Ac[j])
        for l in range(j + 1):
            res = [csub(res[i], cmul(Qc[l][i], Rc[j][l])) for i in range(m)]
        emax = max(emax, max(math.hypot(float(v[0]), float(v[1])) for v in res))
        bw = max(bw, vnorm(res) / vnorm(Ac[j]))
        for l in range(n):
            g = inner(Qc[l], Qc[j])
            if l == j:
                g = (g[0] - 1, g[1])
            orth = max(orth, math.hypot(float(g[0]), float(g[1])))
    return emax, bw, orth


def _close(a, b, rel=1e-13):
    return abs(a - b) <= rel * max(abs(a), abs(b)) or (a == 0.0 and b == 0.0)


@pytest.mark.parametrize("L", [1, 2, 4])
@pytest.mark.parametrize("m,n", [(4, 3), (7, 7), (9, 5)])
def test_error_measures_equal_exact_values(L, m, n):
    """oracle.errors returns what the exact rational computation of the three
    measures returns (to the FP64 rounding of the final value), on the
    oracle's own factors and on factors with planted defects: a column of Q
    scaled by 1 + 2^-30 (non-orthogonal, with a backward error), an entry
    of R with its imaginary sign flipped, and Q with a column leaking into
    another.  A dropped -1 on the diagonal, a wrong sign in the imaginary
    cross term or a norm over the wrong range changes these values."""
    p = inputs.random_problem(L, m, n, seed=m * 3 + n, config=94)
    A = p["A"]
    o = oracle.mgs(A)
    cases = [("factors", o["Q"], o["R"])]
    Q1 = o["Q"].copy()
    Q1[:, :, 1] *= 1.0 + 2.0 ** -30
    cases.append(("scaled q", Q1, o["R"]))
    R2 = o["R"].copy()
    R2[:, 1, n - 1, 0] *= -1.0
    cases.append(("conjugated r", o["Q"], R2))
    Q3 = o["Q"].copy()
    Q3[0, :, n - 1] += 2.0 ** -20 * o["Q"][0, :, 0]
    cases.append(("leaking q", Q3, o["R"]))
    for name, Qx, Rx in cases:
        got = oracle.errors(A, Qx, Rx)
        exact = _exact_measures(A, Qx, Rx)
        for k in range(3):
            assert _close(got[k], exact[k]), (name, k, got, exact)
    # the planted defects are reported at their size
    assert oracle.errors(A, Q1, o["R"])[2] >= 2.0 ** -30
    assert oracle.errors(A, Q3, o["R"])[2] >= 2.0 ** -21


def test_error_measures_zero_for_exact_factors():
    """Dyadic unitary Q and its exact R: all three measures are exactly 0."""
    v = np.array([1 + 1j, 1 + 1j, 1 - 1j, 1j, 1, 0, 0, 0])
    H = np.eye(8) - 2 * np.outer(v, v.conj()) / 8
    n = 5
    A = np.zeros((2, 2, n, 8))
    A[0, 0] = H[:, :n].real.T
    A[0, 1] = H[:, :n].imag.T
    R = np.zeros((2, 2, n, n))
    R[0, 0] = np.eye(n)
    assert list(oracle.errors(A, A, R)) == [0.0, 0.0, 0.0]


# ------------------------------------------------------ Cayley exact QR -----
def _cayley(n, rng):
    """Exact orthogonal Q0 = (I - S)(I + S)^-1 for a small-integer skew S, and det(I+S)."""
    S = [[F(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(i + 1, n):
            v = int(rng.integers(-2, 3))
            S[i][j], S[j][i] = F(v), F(-v)
    M = [[(F(1) if i == j else F(0)) + S[i][j] for j in range(n)] for i in range(n)]
    # Gauss-Jordan inverse and determinant
    aug = [row[:] + [F(int(i == j)) for j in range(n)] for i, row in enumerate(M)]
    det = F(1)
    for c in range(n):
        piv = next(r for r in range(c, n) if aug[r][c] != 0)
        if piv != c:
            aug[c], aug[piv] = aug[piv], aug[c]
            det = -det
        det *= aug[c][c]
        pv = aug[c][c]
        aug[c] = [v / pv for v in aug[c]]
        for r in range(n):
            if r != c and aug[r][c] != 0:
                f = aug[r][c]
                aug[r] = [a - f * b for a, b in zip(aug[r], aug[c])]
    Minv = [row[n:] for row in aug]
    ImS = [[(F(1) if i == j else F(0)) - S[i][j] for j in range(n)] for i in range(n)]
    Q0 = [[sum(ImS[i][k] * Minv[k][j] for k in range(n)) for j in range(n)] for i in range(n)]
    return Q0, det


UNITS = [(F(3, 5), F(4, 5)), (F(4, 5), F(-3, 5)), (F(-3, 5), F(4, 5)), (F(1), F(0)), (F(0), F(1)),
         (F(-4, 5), F(-3, 5))]


def _cayley_problem(m, n, seed):
    rng = np.random.default_rng([1210, m, n, seed])
    Q0, det = _cayley(m, rng)
    assert det > 0
    d = [UNITS[int(rng.integers(0, len(UNITS)))] for _ in range(m)]
    Qcols = [[cmul((Q0[i][j], F(0)), d[j]) for i in range(m)] for j in range(m)]
    t = det * 5
    R = [[(F(0), F(0))] * n for _ in range(n)]  # R[j][i]: column j, row i
    for j in range(n):
        for i in range(j):
            R[j][i] = (F(int(rng.integers(-2, 3))) * t, F(int(rng.integers(-2, 3))) * t)
        R[j][j] = (F(int(rng.integers(1, 4))) * t, F(0))
    Acols = []
    for j in range(n):
        col = [(F(0), F(0))] * m
        for l in range(j + 1):
            col = [cadd(col[i], cmul(Qcols[l][i], R[j][l])) for i in range(m)]
        Acols.append(col)
    for col in Acols:
        for v in col:
            assert v[0].denominator == 1 and v[1].denominator == 1 and abs(v[0]) < 2 ** 50
    xt = [(F(int(rng.integers(-3, 4))), F(int(rng.integers(-3, 4)))) for _ in range(n)]
    b = [(F(0), F(0))] * m
    for j in range(n):
        b = [cadd(b[i], cmul(Acols[j][i], xt[j])) for i in range(m)]
    resid = 0
    if m > n:
        b = [cadd(b[i], cmul(Qcols[n][i], (t, F(0)))) for i in range(m)]
        resid = t
    return Acols, Qcols[:n], R, xt, b, resid


@pytest.mark.parametrize("L", [2, 4])
@pytest.mark.parametrize("m,n,seed", [(4, 4, 0), (6, 5, 1), (7, 4, 2), (6, 6, 3)])
def test_cayley_exact_qr(L, m, n, seed):
    Acols, Qex, Rex, xt, bex, resid = _cayley_problem(m, n, seed)
    A = planar_from_exact(Acols, L)
    b = planar_from_exact([bex], L)[:, :, 0, :]
    # the inputs are Gaussian integers: exactly representable
    assert cmat(A) == Acols
    o, x = _solve(A, b)
    eps = EPS[L]
    kap = kappa_eq(A)
    tol = 20 * kap * m * eps
    Qc, Rc, xc, yc = cmat(o["Q"]), cmat(o["R"]), cvec(x), cvec(o["y"])
    for j in range(n):
        for i in range(m):
            d = csub(Qc[j][i], Qex[j][i])
            assert math.hypot(float(d[0]), float(d[1])) <= tol
        nr = math.sqrt(sum(float(v[0] ** 2 + v[1] ** 2) for v in Rex[j]))
        for i in range(n):
            d = csub(Rc[j][i], Rex[j][i])
            assert math.hypot(float(d[0]), float(d[1])) <= tol * nr
    nx = math.sqrt(sum(float(v[0] ** 2 + v[1] ** 2) for v in xt))
    for k in range(n):
        d = csub(xc[k], xt[k])
        assert math.hypot(float(d[0]), float(d[1])) <= tol * kap * max(nx, 1)
    # y = R x_true exactly in exact arithmetic
    Rx = [(F(0), F(0))] * n
    for k in range(n):
        Rx = [cadd(Rx[i], cmul(Rex[k][i], xt[k])) for i in range(n)]
    ny = math.sqrt(sum(float(v[0] ** 2 + v[1] ** 2) for v in Rx))
    for k in range(n):
        d = csub(yc[k], Rx[k])
        assert math.hypot(float(d[0]), float(d[1])) <= tol * ny + tol * float(resid)
    # z of Equation (1) = the planted residual
    assert abs(float(fval(o["rho"]) - resid)) <= tol * max(float(resid), ny)


# ------------------------------------------------------------- symmetries ---
def _prob(L, m=9, n=7, seed=3):
    p = inputs.random_problem(L, m, n, seed=seed, config=91)
    return p["A"], p["b"]


@pytest.mark.parametrize("L", [1, 2, 4])
def test_power_of_two_scaling_bitwise(L):
    A, b = _prob(L)
    o, x = _solve(A, b)
    o2, x2 = _solve(A * 2.0 ** 37, b * 2.0 ** 37)
    assert np.array_equal(o2["Q"], o["Q"])
    assert np.array_equal(o2["R"], o["R"] * 2.0 ** 37)
    assert np.array_equal(x2, x)
    # one column scaled: Q unchanged, that column of R scaled
    A3 = A.copy()
    A3[:, :, 2] *= 2.0 ** -20
    o3, _ = _solve(A3, b)
    assert np.array_equal(o3["Q"], o["Q"])
    R3 = o["R"].copy()
    R3[:, :, 2] *= 2.0 ** -20
    assert np.array_equal(o3["R"], R3)


@pytest.mark.parametrize("L", [1, 2, 4])
def test_real_input_gives_real_output(L):
    A, b = _prob(L)
    A[:, 1] = 0.0
    b[:, 1] = 0.0
    o, x = _solve(A, b)
    assert np.all(o["Q"][:, 1] == 0) and np.all(o["R"][:, 1] == 0) and np.all(x[:, 1] == 0)


@pytest.mark.parametrize("L", [1, 2])
def test_conjugation_and_rotation_by_i_bitwise(L):
    A, b = _prob(L)
    o, x = _solve(A, b)
    Ac, bc = A.copy(), b.copy()
    Ac[:, 1] *= -1
    bc[:, 1] *= -1
    oc, xcj = _solve(Ac, bc)
    conj = lambda X: np.stack([X[:, 0], -X[:, 1]], axis=1)
    assert np.array_equal(oc["Q"], conj(o["Q"]))
    assert np.array_equal(oc["R"], conj(o["R"]))
    assert np.array_equal(xcj, conj(x))
    # column j times i: q_j * i, r_kj * i (k < j), r_jl * (-i) (l > j)
    j = 3
    Ai = A.copy()
    Ai[:, 0, j], Ai[:, 1, j] = -A[:, 1, j], A[:, 0, j]
    oi, _ = _solve(Ai, b)
    Qe = o["Q"].copy()
    Qe[:, 0, j], Qe[:, 1, j] = -o["Q"][:, 1, j], o["Q"][:, 0, j]
    assert np.array_equal(oi["Q"], Qe)
    Re = o["R"].copy()
    Re[:, 0, j, :j], Re[:, 1, j, :j] = -o["R"][:, 1, j, :j], o["R"][:, 0, j, :j]
    Re[:, 0, j + 1:, j], Re[:, 1, j + 1:, j] = o["R"][:, 1, j + 1:, j], -o["R"][:, 0, j + 1:, j]
    assert np.array_equal(oi["R"], Re)


def test_qd_symmetries_within_rounding():
    """qd expansion rounding is not bitwise commutative; conjugation holds to eps."""
    A, b = _prob(4)
    o, x = _solve(A, b)
    Ac, bc = A.copy(), b.copy()
    Ac[:, 1] *= -1
    bc[:, 1] *= -1
    oc, xcj = _solve(Ac, bc)
    q = cmat(o["Q"])
    qc = cmat(oc["Q"])
    for j in range(len(q)):
        for i in range(len(q[0])):
            assert abs(float(qc[j][i][0] - q[j][i][0])) <= 1e-60
            assert abs(float(qc[j][i][1] + q[j][i][1])) <= 1e-60


# ---------------------------------------------------------- special cases ---
@pytest.mark.parametrize("L", [1, 2, 4])
def test_dyadic_unitary_columns_give_identity_R(L):
    # Householder reflector I - 2 v v^H / (v^H v) with v^H v = 8: dyadic entries
    v = np.array([1 + 1j, 1 + 1j, 1 - 1j, 1j, 1, 0, 0, 0])
    assert np.vdot(v, v).real == 8
    H = np.eye(8) - 2 * np.outer(v, v.conj()) / 8
    n = 5
    A = np.zeros((L, 2, n, 8))
    A[0, 0] = H[:, :n].real.T
    A[0, 1] = H[:, :n].imag.T
    o = oracle.mgs(A)
    R = np.zeros((L, 2, n, n))
    R[0, 0] = np.eye(n)
    assert np.array_equal(o["R"], R)
    assert np.array_equal(o["Q"], A)


@pytest.mark.parametrize("L", [1, 2, 4])
def test_upper_triangular_input(L):
    rng = np.random.default_rng(5)
    n = 6
    A = np.zeros((L, 2, n, n))
    for j in range(n):
        A[0, :, j, :j] = rng.uniform(-1, 1, (2, j))
        A[0, 0, j, j] = rng.uniform(0.5, 2)
    o = oracle.mgs(A)
    Q = np.zeros_like(A)
    Q[0, 0] = np.eye(n)
    assert np.array_equal(o["Q"], Q)
    assert np.array_equal(o["R"], A)


@pytest.mark.parametrize("L", [1, 2, 4])
def test_single_column_closed_form(L):
    p = inputs.random_problem(L, 11, 1, seed=4, config=92)
    o, x = _solve(p["A"], p["b"])
    a = cmat(p["A"])[0]
    bb = cvec(p["b"])
    na2 = sum(v[0] ** 2 + v[1] ** 2 for v in a)
    xe = inner(a, bb)
    xe = (xe[0] / na2, xe[1] / na2)
    xo = cvec(x)[0]
    d = csub(xo, xe)
    assert math.hypot(float(d[0]), float(d[1])) <= 20 * 11 * EPS[L] * math.hypot(float(xe[0]), float(xe[1]))
    assert abs(float(fval(o["R"][:, 0, 0, 0]) ** 2 - na2)) <= 8 * EPS[L] * float(na2)


def test_zero_and_nonfinite_columns_report_info():
    A, b = _prob(2)
    A2 = A.copy()
    A2[:, :, 4] = 0.0
    assert oracle.mgs(A2, b)["info"] == 5
    A3 = A.copy()
    A3[0, 0, 2, 1] = np.nan
    assert oracle.mgs(A3, b)["info"] == 3
    with pytest.raises(ValueError):
        oracle.mgs(np.zeros((2, 2, 5, 3)))  # m < n


@pytest.mark.parametrize("L", [1, 2, 4])
def test_ls_solve_equals_augmented_path(L):
    A, b = _prob(L)
    o, x = _solve(A, b)
    x2, info = oracle.ls_solve(o["Q"], o["R"], b)
    assert info == 0
    assert np.array_equal(x2, x)


def test_thread_count_does_not_change_bits():
    p = inputs.random_problem(2, 40, 30, seed=1, config=93)
    o1 = oracle.mgs(p["A"], p["b"], nthreads=1)
    o8 = oracle.mgs(p["A"], p["b"], nthreads=8)
    for k in ("Q", "R", "y", "rho"):
        assert np.array_equal(o1[k], o8[k])


def test_consistent_square_system_recovers_x_true():
    d = inputs.config1()
    o, x = _solve(d["A"], d["b"])
    kap = kappa_eq(d["A"])
    err = np.max(np.abs((x[0] + x[1]) - (d["x_true"][0] + d["x_true"][1])))
    assert err <= 100 * kap * EPS[2] * 32 * np.max(np.abs(d["x_true"][0]))
