"""Checks of the seeded generators (no solver arithmetic involved)."""
from fractions import Fraction as F

import numpy as np

from paper_1210_0800_amd import inputs
from tests._exact import fval


def test_limbs_are_normalised_and_seeded():
    a = inputs.random_complex(inputs.rng(9, 1, 0), (50,), 4)
    b = inputs.random_complex(inputs.rng(9, 1, 0), (50,), 4)
    assert np.array_equal(a, b)
    for k in range(3):
        assert np.all(np.abs(a[k + 1]) <= 0.5 * np.spacing(np.abs(a[k])))


def test_config4_rhs_is_the_exact_product_rounded_to_qd():
    d = inputs.config4(48)
    A, x, b = d["A64"], d["x_true"], d["b4"]
    M = (A[0, 0] + 1j * A[0, 1]).T
    s = np.linalg.svd(M, compute_uv=False)
    assert 0.5e10 < s[0] / s[-1] < 2e10
    for i in (0, 17, 47):
        re = sum(F(A[0, 0, j, i]) * F(x[0, 0, j]) - F(A[0, 1, j, i]) * F(x[0, 1, j]) for j in range(48))
        im = sum(F(A[0, 0, j, i]) * F(x[0, 1, j]) + F(A[0, 1, j, i]) * F(x[0, 0, j]) for j in range(48))
        assert abs(float(fval(b[:, 0, i]) - re)) <= 2.0 ** -210 * abs(float(re))
        assert abs(float(fval(b[:, 1, i]) - im)) <= 2.0 ** -210 * abs(float(im))


def test_polysys_shape_seeding_and_root():
    s = inputs.polysys(system=5)
    t = inputs.polysys(system=5)
    for k in ("vars", "exps", "coef", "root"):
        assert np.array_equal(s[k], t[k]), k
    neq, nmon, nvpm = s["vars"].shape
    assert (neq, nmon, nvpm) == (32, 32, 5) and s["nvar"] == 32
    # distinct variables per monomial, degrees 1..5
    assert all(len(set(s["vars"][e, m])) == nvpm for e in range(neq) for m in range(nmon))
    assert s["exps"].min() >= 1 and s["exps"].max() <= 5
    # root entries are powers of i
    r = s["root"][0, 0] + 1j * s["root"][0, 1]
    assert np.all(np.isin(np.round(r), [1, -1, 1j, -1j])) and np.all(np.abs(r) == 1)
    # coefficients: dyadic (k / 64) except the first of each equation, set
    # so that f(x*) = 0; all of them exact in FP64, no lower limbs
    c = s["coef"]
    assert np.all(c[1:] == 0)
    assert np.all(c[0, :, :, 1:] * 64 == np.round(c[0, :, :, 1:] * 64))
    # the start point is the root plus a perturbation of the given size
    x0 = inputs.near_root(s, 1e-3, system=5)
    d = x0[0] - s["root"][0]
    assert 0 < np.max(np.abs(d)) <= 1e-3 and np.all(x0[1:] == 0)
