"""Pins of the oracle's precision form (FP64 blocked MGS, then refinement
with the residual in quad-double): against the exact solution of a
constructed system, against the pinned FP64 MGS, and against its own
stopping rules.

The workload is configuration 4's recipe at small sizes: A = U diag(sigma)
V^H (FP64), b the exact product A x_true rounded to qd, so x_true solves the
stored system to about kappa 2^-212.
"""
import numpy as np
import pytest

import oracle
from paper_1210_0800_amd import inputs
from tests._parity import diff, value


def _planar(X, L):
    Y = np.zeros((L,) + X.shape[1:])
    Y[: min(L, X.shape[0])] = X[: min(L, X.shape[0])]
    return Y


def _rel(x, x_true):
    X = _planar(x, 4)
    Xt = _planar(x_true, 4)
    return float(np.sqrt(np.sum(diff(X, Xt) ** 2)) / np.sqrt(np.sum(value(Xt) ** 2)))


@pytest.fixture(scope="module")
def sys96():
    return inputs.config4(96, cond=1e3)


@pytest.mark.parametrize("L,bound", [(2, 1e-27), (4, 1e-58)])
def test_refine_converges_to_the_exact_solution(sys96, L, bound):
    A = _planar(sys96["A64"], L)
    b = sys96["b4"][:L].copy()
    r = oracle.refine(A, b, block=32)
    assert r["info"] == 0 and 1 <= r["iters"] <= 12
    assert _rel(r["x"], sys96["x_true"]) <= bound
    # the starting point is an FP64 solution
    assert 1e-17 < _rel(r["x0"], sys96["x_true"]) <= 1e-11


def test_each_step_contracts(sys96):
    A = _planar(sys96["A64"], 4)
    b = sys96["b4"].copy()
    errs = [_rel(oracle.refine(A, b, block=32, max_iter=k)["x"], sys96["x_true"]) for k in range(4)]
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 <= 1e-6 * e0, errs
    r = oracle.refine(A, b, block=32, max_iter=0)
    assert r["info"] == -2 and r["iters"] == 0
    assert np.array_equal(r["x"], r["x0"])


def test_block_of_one_is_plain_mgs(sys96):
    """With panels of one column the FP64 factorisation is MGS itself
    (Figure 1): x0 is bitwise the oracle's FP64 MGS least-squares solution."""
    A = _planar(sys96["A64"], 2)
    b = sys96["b4"][:2].copy()
    r = oracle.refine(A, b, block=1, max_iter=0)
    o = oracle.mgs(sys96["A64"], b[:1].copy())
    x64, _ = oracle.backsolve(o["R"], o["y"])
    assert np.array_equal(r["x0"][0], x64[0]) and np.all(r["x0"][1] == 0)


def test_fixed_point_does_not_depend_on_the_blocking(sys96):
    A = _planar(sys96["A64"], 4)
    b = sys96["b4"].copy()
    xs = [oracle.refine(A, b, block=bk)["x"] for bk in (1, 16, 64, 200)]
    for x in xs[1:]:
        assert _rel(x, xs[0]) <= 1e-60


def test_refine_reports_stagnation_on_a_singular_matrix():
    d = inputs.config4(64, cond=1e19)
    r = oracle.refine(_planar(d["A64"], 2), d["b4"][:2].copy(), block=16, max_iter=8)
    assert r["info"] in (-1, -2)


def test_refine_thread_count_invariance(sys96):
    A = _planar(sys96["A64"], 2)
    b = sys96["b4"][:2].copy()
    r1 = oracle.refine(A, b, block=32, nthreads=1)
    r4 = oracle.refine(A, b, block=32, nthreads=4)
    assert np.array_equal(r1["x"], r4["x"]) and r1["iters"] == r4["iters"]
