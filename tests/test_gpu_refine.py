"""GPU checks of the precision form (mgs_refine_solve).

Reference: config4 builds b as the exact product A x_true rounded to qd, so
x_true solves the stored system to about kappa 2^-212 (1e-53 at kappa 1e10).
Bar: the refined dd / qd solution reaches the error of the plain dd / qd
MGS solution on the same GPU (the residual is accumulated in qd, so the
refined error is not limited by the working precision's residual), and
the iteration converges.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1210_0800_amd import api, inputs  # noqa: E402
from tests._parity import diff, value  # noqa: E402

pytestmark = pytest.mark.gpu


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def planar(X, L):
    """First L limbs of a normalized expansion (zero-padded): for a qd vector
    truncated to dd this is within one dd ulp of its rounding."""
    Y = np.zeros((L,) + X.shape[1:])
    k = min(L, X.shape[0])
    Y[:k] = X[:k]
    return Y


def rel_err(x, x_true):
    X = np.zeros((4,) + x.shape[1:])
    X[: x.shape[0]] = x
    Xt = np.zeros((4,) + x_true.shape[1:])
    Xt[: x_true.shape[0]] = x_true
    d = diff(X, Xt)
    return float(np.sqrt(np.sum(d ** 2)) / np.sqrt(np.sum(value(Xt) ** 2)))


def solve_both(d, L, max_iter=30):
    A = planar(d["A64"], L)
    b = d["b4"][:L].copy()
    Ag, bg = T(A), T(b)
    f = api.lstsq(Ag, bg)
    r = api.refine_lstsq(Ag, bg, max_iter=max_iter)
    torch.cuda.synchronize()
    assert int(f["info"].item()) == 0
    plain = rel_err(f["x"].cpu().numpy(), d["x_true"])
    refined = rel_err(r["x"].cpu().numpy(), d["x_true"])
    return plain, refined, int(r["iters"].item()), int(r["info"].item()), float(r["err_est"].item())


@pytest.mark.parametrize("L", [2, 4])
def test_refined_matches_plain_accuracy_n256(L):
    d = inputs.config4(256)
    plain, refined, iters, info, est = solve_both(d, L)
    print("n=256 L=%d plain %.3e refined %.3e iters %d info %d est %.2e" % (L, plain, refined, iters, info, est))
    assert info == 0 and 1 <= iters <= 25
    assert refined <= plain
    assert plain <= (1e-19 if L == 2 else 1e-49)


@pytest.mark.parametrize("L", [2, 4])
def test_refine_against_the_oracle_refinement_n256(L):
    """The same method in the oracle (FP64 blocked MGS with panels of 64,
    residual in qd, projections replayed): same outcome, iteration counts
    within one, solutions equal to the working precision."""
    d = inputs.config4(256)
    A = planar(d["A64"], L)
    b = d["b4"][:L].copy()
    r = api.refine_lstsq(T(A), T(b), max_iter=30)
    torch.cuda.synchronize()
    o = oracle.refine(A, b, block=64, max_iter=30)
    print("n=256 L=%d gpu iters %d oracle iters %d" % (L, int(r["iters"].item()), o["iters"]))
    assert int(r["info"].item()) == 0 and o["info"] == 0
    assert abs(int(r["iters"].item()) - o["iters"]) <= 1
    assert rel_err(r["x"].cpu().numpy(), o["x"]) <= (1e-27 if L == 2 else 1e-57)


def test_refined_dd_config4_2048():
    d = inputs.config4(2048, workers=8)
    plain, refined, iters, info, est = solve_both(d, 2)
    print("n=2048 dd plain %.3e refined %.3e iters %d info %d" % (plain, refined, iters, info))
    assert info == 0 and iters <= 12
    assert refined <= plain


def solve_stored(A, b, x_true, max_iter=30):
    """Plain MGS and refined solutions of the stored system (A, b)."""
    Ag, bg = T(A), T(b)
    f = api.lstsq(Ag, bg)
    r = api.refine_lstsq(Ag, bg, max_iter=max_iter)
    torch.cuda.synchronize()
    assert int(f["info"].item()) == 0
    plain = rel_err(f["x"].cpu().numpy(), x_true)
    refined = rel_err(r["x"].cpu().numpy(), x_true)
    return plain, refined, int(r["iters"].item()), int(r["info"].item()), float(r["err_est"].item())


@pytest.fixture(scope="module")
def config4_tail():
    return inputs.config4(2048, workers=16, tail=True)


@pytest.mark.parametrize("L", [2, 4])
def test_refined_with_subfp64_matrix_2048(config4_tail, L):
    """A carries a limb below FP64 (relative 2^-60), so the FP64 factors
    are those of an approximation of A; the refinement (residual of the
    full A) still reaches the plain method's error, converging.  x_true
    solves the qd system exactly; the dd right-hand side is rounded."""
    d = config4_tail
    A, b = (d["A2"], d["b2"]) if L == 2 else (d["A4"], d["b4"])
    plain, refined, iters, info, est = solve_stored(A, b, d["x_true"])
    print("n=2048 tail L=%d plain %.3e refined %.3e iters %d info %d est %.2e" % (L, plain, refined, iters, info,
                                                                                   est))
    assert info == 0 and 1 <= iters <= 25
    assert np.isfinite(est) and est < 1.0
    # equal error: in qd both solutions sit at the accuracy the qd
    # arithmetic attains on this system, and which of the two lands lower
    # varies with rounding; a factor of 2 separates "reaches" from "misses"
    assert refined <= 2 * plain
    assert plain <= (1e-19 if L == 2 else 1e-49)


def test_refinement_reports_failure_to_converge():
    d = inputs.config4(128, cond=1e19)
    A = planar(d["A64"], 2)
    r = api.refine_lstsq(T(A), T(d["b4"][:2].copy()), max_iter=8)
    torch.cuda.synchronize()
    assert int(r["info"].item()) in (-1, -2)
