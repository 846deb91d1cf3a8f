"""Pins of the oracle's dd / qd arithmetic against exact rational arithmetic.

The paper computes in double double and quad double numbers (Section 1); each
operation below must reproduce the exact rational result within the error
bound of the formulation, and return normalised limbs.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from tests._exact import fval

U = 2.0 ** -53


def _normal_limbs(rng, count, L, emin=-30, emax=30):
    """Normalised random limbs with random exponents and signs."""
    out = np.zeros((count, L))
    hi = rng.uniform(0.5, 1.0, count) * 2.0 ** rng.integers(emin, emax, count) * rng.choice([-1, 1], count)
    out[:, 0] = hi
    for k in range(1, L):
        prev = out[:, k - 1]
        # strictly below half an ulp of the previous limb, random sign
        out[:, k] = np.spacing(np.abs(prev)) * 0.5 * rng.uniform(-0.999, 0.999, count)
    return out


def _cases(L, count=1500, seed=7):
    rng = np.random.default_rng([1210, L, seed])
    a = _normal_limbs(rng, count, L)
    b = _normal_limbs(rng, count, L)
    n4 = count // 4
    # heavy cancellation: b = -a + small perturbation in the lower limbs
    b[:n4] = -a[:n4]
    b[:n4, L - 1] += np.spacing(np.abs(a[:n4, L - 1])) * rng.integers(-5, 6, n4)
    # b = -a exactly (result must be exactly zero)
    b[n4:n4 + 20] = -a[n4:n4 + 20]
    # large exponent gaps
    b[n4 + 20:2 * n4] *= 2.0 ** rng.integers(-120, -40, 2 * n4 - n4 - 20)[:, None]
    # equal leading limbs, opposite lower limbs
    b[2 * n4:2 * n4 + 50, 0] = a[2 * n4:2 * n4 + 50, 0]
    b[2 * n4:2 * n4 + 50, 1:] = -0.5 * a[2 * n4:2 * n4 + 50, 1:]
    return a, b


def _check_normalised(z, L, strict_half):
    for k in range(L - 1):
        lim = np.spacing(np.abs(z[:, k])) * (0.5 if strict_half else 1.0)
        bad = np.abs(z[:, k + 1]) > lim
        assert not np.any(bad), "limbs not normalised at limb %d: %r" % (k, z[bad][:3])


BOUND = {  # relative error bounds in units of 2^-106 (dd) / 2^-209 (qd)
    2: {"add": 3.1, "sub": 3.1, "mul": 4.0, "div": 6.0, "sqrt": 6.0},
    4: {"add": 1.0, "sub": 1.0, "mul": 1.0, "div": 1.0, "sqrt": 1.0},
}
SCALE = {2: U * U, 4: 2.0 ** -209}


@pytest.mark.parametrize("L", [2, 4])
@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_binary_ops_exact(L, op):
    a, b = _cases(L, count=1200 if L == 2 else 500)
    if op == "div":
        b[b[:, 0] == 0] = 1.0
    z = oracle.arith(L, op, a, b)
    worst = 0.0
    for i in range(a.shape[0]):
        fa, fb = fval(a[i]), fval(b[i])
        ex = {"add": fa + fb, "sub": fa - fb, "mul": fa * fb, "div": fa / fb if fb != 0 else None}[op]
        fz = fval(z[i])
        if ex == 0:
            assert fz == 0, (op, a[i], b[i], z[i])
            continue
        rel = abs(float((fz - ex) / ex))
        worst = max(worst, rel)
    assert worst <= BOUND[L][op] * SCALE[L], (op, worst / SCALE[L])
    _check_normalised(z, L, strict_half=(L == 2))


@pytest.mark.parametrize("L", [2, 4])
def test_sqrt_exact(L):
    rng = np.random.default_rng([1210, L, 99])
    a = np.abs(_normal_limbs(rng, 600 if L == 2 else 300, L))
    a[:, 1:] *= np.sign(a[:, :1])  # keep lower limbs' relative signs random but value positive
    # perfect squares must come back exactly
    sq = np.zeros((20, L))
    sq[:, 0] = (np.arange(1, 21) * 3.0) ** 2
    a = np.vstack([a, sq])
    z = oracle.arith(L, "sqrt", a)
    worst = 0.0
    for i in range(a.shape[0]):
        fa, fz = fval(a[i]), fval(z[i])
        # |z^2 - a| / a ~ 2 * relative error of z
        rel = abs(float((fz * fz - fa) / fa)) / 2.0
        worst = max(worst, rel)
    assert worst <= BOUND[L]["sqrt"] * SCALE[L], worst / SCALE[L]
    for i in range(20):
        assert fval(z[-20 + i]) == F(3 * (i + 1))
    _check_normalised(z, L, strict_half=(L == 2))


def test_double_ops_are_ieee():
    a = np.array([[1.0], [3.0], [2.0]])
    b = np.array([[3.0], [7.0], [5.0]])
    assert oracle.arith(1, "div", a, b)[1, 0] == 3.0 / 7.0
    assert oracle.arith(1, "sqrt", b)[2, 0] == np.sqrt(5.0)
