"""GPU parity of the precision form's factorisation on its own (mgs_qr64):
complex FP64 blocked MGS of [A b], panels of 64 columns with the trailing
products on the matrix cores, against the oracle's FP64 column MGS
(Figure 1 in FP64, pinned in test_oracle_mgs.py).

Bar: err_Q, err_R, ||y_gpu - y_orc|| below 5e-13 * max(1, kappa / 100)
(about 2^12 units of 2^-53, the ratio used for dd and qd); the exact
backward error max_j ||a_j - Q r_j|| / ||a_j|| <= 4 m 2^-53 and the
orthogonality ||Q^H Q - I|| <= 10 kappa n 2^-53 (Bjorck's O(kappa u) for
MGS), evaluated exactly by the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1210_0800_amd import api, inputs  # noqa: E402
from tests._parity import TAU, assert_parity, diff, errors  # noqa: E402

pytestmark = pytest.mark.gpu
EPS64 = 2.0 ** -53


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def run(A1, b1):
    """A1 (1, 2, n, m), b1 (1, 2, m) FP64 planar -> GPU Q, R, y (1, 2, ...)."""
    f = api.mgs_qr64(T(A1[0]), None if b1 is None else T(b1[0]))
    torch.cuda.synchronize()
    out = {k: (None if v is None else v.cpu().numpy()[None]) for k, v in f.items() if k != "info"}
    out["info"] = int(f["info"].item())
    return out


def problem(m, n, seed):
    p = inputs.random_problem(2, m, n, seed=seed, config=70, dist="normal")
    return p["A"][:1].copy(), p["b"][:1].copy()


@pytest.mark.parametrize("m,n", [(1, 1), (40, 17), (64, 64), (100, 65), (257, 129), (300, 255), (1000, 300),
                                 (2100, 130)])
def test_qr64_against_fp64_oracle(m, n):
    A, b = problem(m, n, m + 3 * n)
    g = run(A, b)
    o = oracle.mgs(A, b)
    assert g["info"] == 0 and o["info"] == 0
    e = errors(A, g["Q"], g["R"], o["Q"], o["R"])
    print("qr64 %dx%d" % (m, n), e)
    assert_parity(e, 1)
    tol = TAU[1] * max(1.0, e["kappa"] / 100.0)
    dy = diff(g["y"], o["y"])
    assert np.sqrt(np.sum(dy ** 2)) <= 10 * tol * np.sqrt(np.sum(b[0] ** 2))
    n_ = A.shape[2]
    il = np.tril_indices(n_, -1)
    assert np.all(g["R"][:, :, il[1], il[0]] == 0)
    assert np.all(g["R"][0, 1, np.arange(n_), np.arange(n_)] == 0)
    assert np.all(g["R"][0, 0, np.arange(n_), np.arange(n_)] > 0)
    if m * n <= 300 * 255:
        ev = oracle.errors(A, g["Q"], g["R"])
        assert ev[1] <= 4 * m * EPS64, ev
        assert ev[2] <= 10 * e["kappa"] * n * EPS64, ev


def test_qr64_without_rhs_and_zero_column():
    A, b = problem(150, 90, 11)
    g = run(A, None)
    o = oracle.mgs(A)
    assert g["info"] == 0 and g["y"] is None
    assert_parity(errors(A, g["Q"], g["R"], o["Q"], o["R"]), 1)
    A[:, :, 70] = 0.0
    assert run(A, b)["info"] == 71


def test_qr64_reproducible_bitwise():
    A, b = problem(700, 333, 12)
    g1, g2 = run(A, b), run(A, b)
    for k in ("Q", "R", "y"):
        assert np.array_equal(g1[k], g2[k]), k


def test_qr64_orthogonality_config4():
    """Precision-form workload, 2048 x 2048, kappa 1e10: MGS loses
    orthogonality like kappa u (Bjorck); reported and bounded."""
    d = inputs.config4(2048, workers=8)
    g = run(d["A64"], d["b4"][:1].copy())
    assert g["info"] == 0
    Q = (g["Q"][0, 0] + 1j * g["Q"][0, 1]).T
    loss = float(np.linalg.norm(Q.conj().T @ Q - np.eye(Q.shape[1]), 2))
    print("config4 qr64 ||Q^H Q - I||_2 = %.3e (kappa 1e10, kappa u = %.1e)" % (loss, 1e10 * EPS64))
    assert loss <= 10 * 1e10 * 2048 * EPS64
    # backward error in FP64 arithmetic (checked to within the check's own rounding)
    Rm = (g["R"][0, 0] + 1j * g["R"][0, 1]).T
    Am = (d["A64"][0, 0] + 1j * d["A64"][0, 1]).T
    back = float(np.max(np.linalg.norm(Am - Q @ Rm, axis=0) / np.linalg.norm(Am, axis=0)))
    print("config4 qr64 max_j ||a_j - Q r_j|| / ||a_j|| = %.3e" % back)
    assert back <= 4 * 2048 * EPS64
