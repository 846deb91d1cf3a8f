"""Pins of the oracle's polynomial evaluation and Newton corrector (Section
7: Newton's method as the corrector of a path tracker; the system shape of
Table 6: 32 equations, 32 variables, 32 monomials of 5 variables, degrees
1..5).

What fixes the results independently of the oracle's own code:
* the constructed root x* (entries 1, -1, i, -i, dyadic coefficients): f(x*)
  is exactly zero, every limb;
* tiny systems at dyadic points: f and J by exact rational arithmetic;
* J against central differences of f in qd along real and imaginary
  directions (Cauchy-Riemann: f is complex analytic);
* Newton from a perturbed root converges to x* quadratically.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from paper_1210_0800_amd import inputs
from tests._exact import fval
from tests._parity import diff, value


def _at(x, L):
    y = np.zeros((L,) + x.shape[1:])
    y[: min(L, x.shape[0])] = x[: min(L, x.shape[0])]
    return y


def _sys_at(sys_, L):
    s = dict(sys_)
    s["coef"] = _at(sys_["coef"], L)
    return s


@pytest.mark.parametrize("L", [1, 2, 4])
@pytest.mark.parametrize("system", [0, 1])
def test_root_is_an_exact_zero(L, system):
    s = _sys_at(inputs.polysys(system=system, L=L), L)
    F, J = oracle.poly_eval(s, _at(s["root"], L))
    assert np.all(F == 0.0)
    assert np.all(np.isfinite(J)) and np.max(np.abs(J[0])) > 1.0
    x0 = inputs.near_root(s, 1e-3, L=L, system=system)
    F0, _ = oracle.poly_eval(s, x0)
    assert np.max(np.abs(F0[0])) > 1e-4


def _exact_eval(s, xq):
    """f and J of system s at the exact complex point xq (list of pairs)."""
    v, d = s["vars"], s["exps"]
    neq, nmon, nvpm = v.shape
    nvar = s["nvar"]
    coef = s["coef"]
    one = (Fr(1), Fr(0))

    def mul(a, b):
        return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])

    def pw(a, k):
        r = one
        for _ in range(k):
            r = mul(r, a)
        return r

    F = [(Fr(0), Fr(0)) for _ in range(neq)]
    J = [[(Fr(0), Fr(0)) for _ in range(neq)] for _ in range(nvar)]
    for e in range(neq):
        for m in range(nmon):
            c = (fval(coef[:, 0, e, m]), fval(coef[:, 1, e, m]))
            mono = c
            for t in range(nvpm):
                mono = mul(mono, pw(xq[v[e, m, t]], int(d[e, m, t])))
            F[e] = (F[e][0] + mono[0], F[e][1] + mono[1])
            for t in range(nvpm):
                if d[e, m, t] == 0:
                    continue
                term = mul(c, (Fr(int(d[e, m, t])), Fr(0)))
                for u in range(nvpm):
                    term = mul(term, pw(xq[v[e, m, u]], int(d[e, m, u]) - (1 if u == t else 0)))
                j = v[e, m, t]
                J[j][e] = (J[j][e][0] + term[0], J[j][e][1] + term[1])
    return F, J


@pytest.mark.parametrize("L", [2, 4])
def test_tiny_system_exact_at_a_dyadic_point(L):
    s = _sys_at(inputs.polysys(neq=3, nvar=3, nmon=4, nvpm=2, maxdeg=3, L=L, system=3), L)
    g = np.random.default_rng(11)
    re = g.integers(-16, 17, size=3) / 16.0
    im = g.integers(-16, 17, size=3) / 16.0
    x = np.zeros((L, 2, 3))
    x[0, 0], x[0, 1] = re, im
    F, J = oracle.poly_eval(s, x)
    Fe, Je = _exact_eval(s, [(Fr(float(a)), Fr(float(b))) for a, b in zip(re, im)])
    # dyadic inputs of few bits: every product and sum is exact in dd / qd
    for e in range(3):
        assert (fval(F[:, 0, e]), fval(F[:, 1, e])) == Fe[e]
        for j in range(3):
            assert (fval(J[:, 0, j, e]), fval(J[:, 1, j, e])) == Je[j][e]


def test_jacobian_matches_central_differences_in_qd():
    L = 4
    s = _sys_at(inputs.polysys(system=2, L=L), L)
    x = inputs.near_root(s, 1e-2, L=L, system=2)
    _, J = oracle.poly_eval(s, x)
    Jv = value(J)
    scale = np.max(np.abs(Jv))

    def step(x0):
        # a step h near 2^-60 that keeps x0 +- h a normalised qd: below half
        # an ulp of the leading limb (h goes to the second limb) or a multiple
        # of that ulp (added exactly to it)
        u = np.spacing(abs(x0))
        for h in (2.0 ** -60, 2.0 ** -61, 2.0 ** -62):
            if h < u / 2 or h >= u:
                return h
        raise AssertionError(x0)

    def shifted(part, j, h):
        y = x.copy()
        x0 = x[0, part, j]
        if abs(h) < np.spacing(abs(x0)) / 2:
            y[1, part, j] = h
        else:
            y[0, part, j] = x0 + h
            assert y[0, part, j] - x0 == h
        return y

    for part in (0, 1):  # real and imaginary direction
        for j in range(0, s["nvar"], 3):
            h = step(x[0, part, j])
            xp, xm = shifted(part, j, h), shifted(part, j, -h)
            Fp, _ = oracle.poly_eval(s, xp)
            Fm, _ = oracle.poly_eval(s, xm)
            fd = diff(Fp, Fm) / (2 * h)  # (2, neq): d f / d(re or im of x_j)
            if part == 1:  # d/d(im x_j) = i d/dx_j
                fd = np.stack([fd[1], -fd[0]])
            err = np.max(np.abs(fd - Jv[:, j, :]))
            assert err < 1e-28 * scale, (part, j, err)


@pytest.mark.parametrize("L,iters,floor", [(2, 6, 1e-28), (4, 7, 1e-58)])
@pytest.mark.parametrize("neq", [32, 40])
def test_newton_converges_quadratically_to_the_root(L, iters, floor, neq):
    s = _sys_at(inputs.polysys(neq=neq, L=L, system=0), L)
    x0 = inputs.near_root(s, 1e-3, L=L, system=0)
    x, dn = oracle.newton(s, x0, iters)
    delta0 = float(np.sqrt(np.sum(diff(x0, _at(s["root"], L)) ** 2)))
    # the first correction removes nearly all of the perturbation
    assert abs(dn[0] - delta0) < 0.05 * delta0
    # quadratic decrease until the precision floor
    for k in range(iters - 1):
        if dn[k] > floor * 1e3:
            assert dn[k + 1] <= 1e3 * dn[k] ** 2 + floor, (k, dn)
    err = float(np.sqrt(np.sum(diff(x, _at(s["root"], L)) ** 2)))
    assert err < floor, (err, dn)


def test_newton_from_the_root_stays_there():
    L = 2
    s = _sys_at(inputs.polysys(L=L, system=1), L)
    x, dn = oracle.newton(s, _at(s["root"], L), 2)
    assert np.all(dn == 0.0)
    assert np.all(diff(x, _at(s["root"], L)) == 0.0)
