"""GPU parity of the least-squares adjoint (ls_adjoint, LstsqFn).

Bar: the dd gradients agree with the oracle's closed form evaluated in qd
on the same input within 1e-28 * max(1, kappa^2 / 100) relative (the
adjoint involves two triangular solves with R, hence kappa^2); the qd
gradients within 1e-58 * max(1, kappa^2 / 100).  Central differences of L
from qd least-squares solves pin a sample of entries independently.
"""
from fractions import Fraction as F

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1210_0800_amd import api, inputs  # noqa: E402
from tests._exact import cvec, fval  # noqa: E402
from tests._parity import TAU, diff, kappa_eff, value  # noqa: E402

pytestmark = pytest.mark.gpu


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def N(t):
    return t.cpu().numpy()


def widen(X, L):
    """Embed a planar dd array into L >= 2 limbs (exact)."""
    Y = np.zeros((L,) + X.shape[1:])
    Y[: X.shape[0]] = X
    return Y


def gpu_adjoint(A, b, g):
    At, bt = T(A), T(b)
    f = api.mgs_qr(At, bt)
    x, _ = api.ls_backsolve(f["R"], f["y"])
    gA, gb, info = api.ls_adjoint(At, bt, f["Q"], f["R"], x, T(g))
    torch.cuda.synchronize()
    assert int(f["info"].item()) == 0 and int(info.item()) == 0
    return N(gA), N(gb), N(x)


def rel(Xg, Xo):
    d = diff(widen(Xg, Xo.shape[0]), Xo)
    v = value(Xo)
    return float(np.sqrt(np.sum(d ** 2)) / np.sqrt(np.sum(v ** 2)))


def test_config5_dd_512x384_against_qd_closed_form():
    d = inputs.config5()
    A, b, g = d["A"], d["b"], d["g"]
    gA, gb, x = gpu_adjoint(A, b, g)
    gAo, gbo, xo = oracle.adjoint(widen(A, 4), widen(b, 4), widen(g, 4))
    kap, _ = kappa_eff(A)
    tol = TAU[2] * max(1.0, kap * kap / 100.0)
    e = (rel(gA, gAo), rel(gb, gbo), rel(x, xo))
    print("config5 adjoint rel errors (gA, gb, x)", e, "kappa", kap)
    assert e[0] <= tol and e[1] <= tol and e[2] <= tol, (e, tol)
    # exact identities Re<gA, A> = -L and Re<gb, b> = L, L = Re(g^H x)
    Lv = float(np.sum(value(g) * value(x)))
    ipA = float(np.sum(value(gA) * value(A)))
    ipb = float(np.sum(value(gb) * value(b)))
    scale = np.sqrt(np.sum(value(gA) ** 2)) * np.sqrt(np.sum(value(A) ** 2))
    assert abs(ipA + Lv) <= 1e-12 * scale
    assert abs(ipb - Lv) <= 1e-12 * np.sqrt(np.sum(value(gb) ** 2)) * np.sqrt(np.sum(value(b) ** 2))


@pytest.mark.parametrize("prec,m,n", [(2, 70, 45), (4, 40, 24), (2, 300, 300)])
def test_adjoint_against_oracle_same_precision_inputs(prec, m, n):
    p = inputs.random_problem(prec, m, n, seed=m + n, config=64, dist="normal")
    g = inputs.random_complex(inputs.rng(64, m + n, 3), (n,), prec, "normal")
    gA, gb, x = gpu_adjoint(p["A"], p["b"], g)
    L = 4
    gAo, gbo, xo = oracle.adjoint(widen(p["A"], L), widen(p["b"], L), widen(g, L))
    kap, _ = kappa_eff(p["A"])
    tol = TAU[prec] * max(1.0, kap * kap / 100.0)
    assert rel(gA, gAo) <= tol and rel(gb, gbo) <= tol, (rel(gA, gAo), rel(gb, gbo), tol)


def test_adjoint_entries_against_qd_central_differences():
    m, n = 16, 10
    g0 = inputs.rng(65, 0, 0)
    A = np.zeros((2, 2, n, m))
    A[0] = g0.uniform(0.1, 1.0, (2, n, m)) * g0.choice([-1.0, 1.0], (2, n, m))
    b = np.zeros((2, 2, m))
    b[0] = g0.uniform(-1, 1, (2, m))
    g = np.zeros((2, 2, n))
    g[0] = g0.uniform(-1, 1, (2, n))
    gA, gb, _ = gpu_adjoint(A, b, g)
    h = 2.0 ** -70

    def loss(Ap):
        o = oracle.mgs(widen(Ap, 4), widen(b, 4))
        x, _ = oracle.backsolve(o["R"], o["y"])
        return sum(gv[0] * xv[0] + gv[1] * xv[1] for gv, xv in zip(cvec(g), cvec(x)))

    rng = np.random.default_rng(7)
    scale = np.max(np.abs(gA[0]))
    for _ in range(12):
        i, j, part = int(rng.integers(0, m)), int(rng.integers(0, n)), int(rng.integers(0, 2))
        Ap, Am = A.copy(), A.copy()
        Ap[1, part, j, i] = h   # hi limb |a| >= 0.1: (a, h) is a normalised dd
        Am[1, part, j, i] = -h
        fd = (loss(Ap) - loss(Am)) / (2 * F(h))
        assert abs(float(fd - fval(gA[:, part, j, i]))) <= 1e-26 * scale


def test_autograd_function_routes_the_adjoint():
    d = inputs.random_problem(2, 60, 40, seed=1, config=66, dist="normal")
    g = inputs.random_complex(inputs.rng(66, 1, 3), (40,), 2, "normal")
    A = T(d["A"]).requires_grad_(True)
    b = T(d["b"]).requires_grad_(True)
    x = api.LstsqFn.apply(A, b)
    x.backward(T(g))
    gA, gb, xr = gpu_adjoint(d["A"], d["b"], g)
    assert np.array_equal(N(x.detach()), xr)
    assert np.array_equal(N(A.grad), gA) and np.array_equal(N(b.grad), gb)
