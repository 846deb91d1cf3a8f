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
