"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar (dd / qd): err_Q, err_R (column relative) and err_x (equilibrated) below
1e-28 / 1e-58 times max(1, kappa / 100), kappa = kappa_2(A D^-1) for Q and R
and the least-squares condition number for x.  Reductions run in a fixed
order, so repeated runs are bitwise identical; exact scaling symmetries hold
bitwise.

Both schedules of the factorisation are checked on every random shape: the
automatic choice (in dd the single cooperative launch whenever the columns
fit in registers, m <= 1024) and the per-panel launches
(mgs_qr_schedule with the panel schedule).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1210_0800_amd import api, inputs  # noqa: E402
from tests._exact import EPS  # noqa: E402
from tests._parity import TAU, assert_parity, diff, errors, value  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev():
    return torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(_dev())


def N(t):
    return None if t is None else t.cpu().numpy()


def gpu_lstsq(A, b, sched="auto"):
    f = api.lstsq(T(A), T(b), schedule=None if sched == "auto" else sched)
    torch.cuda.synchronize()
    return {k: N(v) for k, v in f.items()}


def oracle_lstsq(A, b):
    o = oracle.mgs(A, b)
    x, _ = oracle.backsolve(o["R"], o["y"])
    o["x"] = x
    return o


def check_case(A, b, prec, invariants=False, schedules=("auto",)):
    o = oracle_lstsq(A, b)
    assert o["info"] == 0
    for sched in schedules:
        e, g = check_gpu(A, b, prec, o, invariants, sched)
    return e, g, o


def check_gpu(A, b, prec, o, invariants, sched):
    g = gpu_lstsq(A, b, sched)
    assert int(g["info"][0]) == 0, sched
    assert int(g["info_backsolve"][0]) == 0
    e = errors(A, g["Q"], g["R"], o["Q"], o["R"], g["x"], o["x"], o["rho"])
    assert_parity(e, prec)
    # y = Q^H b and rho, relative to ||b||
    tol = TAU[prec] * max(1.0, e["kappa"] / 100.0)
    nb = np.sqrt(np.sum(b[0] ** 2))
    dy = diff(g["y"], o["y"])
    assert np.sqrt(np.sum(dy ** 2)) <= 10 * tol * nb
    drho = abs(float(diff(g["rho"][:, None], o["rho"][:, None])[0]))
    assert drho <= 10 * tol * nb
    # R: exact zeros below the diagonal, real positive diagonal
    n = A.shape[2]
    il = np.tril_indices(n, -1)
    assert np.all(g["R"][:, :, il[1], il[0]] == 0)
    assert np.all(g["R"][:, 1, np.arange(n), np.arange(n)] == 0)
    assert np.all(g["R"][0, 0, np.arange(n), np.arange(n)] > 0)
    if invariants:
        ev = oracle.errors(A, g["Q"], g["R"])
        m = A.shape[3]
        assert ev[1] <= 4 * m * EPS[prec], ev
        assert ev[2] <= 10 * e["kappa"] * n * EPS[prec], ev
    return e, g


DD_SHAPES = [(1, 1), (5, 1), (32, 32), (33, 7), (64, 64), (65, 65), (100, 37), (200, 200), (257, 129),
             (300, 255), (513, 300), (1100, 40), (2100, 20), (4096, 6)]
QD_SHAPES = [(1, 1), (9, 3), (32, 32), (64, 20), (100, 100), (257, 40), (513, 30), (1030, 12), (2048, 6)]


@pytest.mark.parametrize("m,n", DD_SHAPES)
def test_dd_random_parity(m, n):
    p = inputs.random_problem(2, m, n, seed=m * 7 + n, config=50)
    check_case(p["A"], p["b"], 2, invariants=(m * n <= 300 * 255), schedules=("auto", "panel"))


@pytest.mark.parametrize("m,n", QD_SHAPES)
def test_qd_random_parity(m, n):
    p = inputs.random_problem(4, m, n, seed=m * 7 + n, config=51)
    check_case(p["A"], p["b"], 4, invariants=(m * n <= 100 * 100), schedules=("auto", "panel"))


SMALL_SHAPES = [(1, 1), (5, 1), (17, 16), (32, 32), (33, 7), (64, 40), (64, 63)]


@pytest.mark.parametrize("m,n", SMALL_SHAPES)
def test_dd_small_schedule_parity(m, n):
    """The one-workgroup schedule (dd, m <= 64, at most 64 columns of [A b])
    against the oracle, and against the single-launch schedule."""
    p = inputs.random_problem(2, m, n, seed=m * 5 + n, config=54)
    e, g, o = check_case(p["A"], p["b"], 2, invariants=True, schedules=("small", "resident"))
    print("small %dx%d" % (m, n), e)


def test_dd_small_schedule_in_place_and_refusals():
    from paper_1210_0800_amd import _lib

    p = inputs.random_problem(2, 40, 30, seed=11, config=55)
    f = api.mgs_qr(T(p["A"]), schedule="small")
    Q1, R1 = N(f["Q"]), N(f["R"])
    Ain = T(p["A"])
    f2 = api.mgs_qr(Ain, Q=Ain, schedule="small")
    torch.cuda.synchronize()
    assert np.array_equal(N(Ain), Q1) and np.array_equal(N(f2["R"]), R1)
    # refused: more rows than lanes, more than 64 columns of [A b], and (qd)
    # q vectors beyond the LDS budget of the one-workgroup kernel
    for prec, m, n in ((2, 65, 20), (2, 64, 64), (4, 64, 45), (1, 70, 10)):
        q = inputs.random_problem(prec, m, n, seed=3, config=55)
        with pytest.raises(_lib.MgsError) as err:
            api.mgs_qr(T(q["A"]), T(q["b"]), schedule="small")
        assert err.value.status == -1


def test_config1_dd_32x32():
    d = inputs.config1()
    e, g, o = check_case(d["A"], d["b"], 2, invariants=True, schedules=("auto", "resident"))
    # consistent square system: x_true recovered
    dx = np.abs((g["x"][0] + g["x"][1]) - (d["x_true"][0] + d["x_true"][1]))
    assert dx.max() <= 1e-27 * e["kappa"]


def test_config2_qd_320x256():
    d = inputs.config2()
    e, g, o = check_case(d["A"], d["b"], 4, schedules=("auto", "panel"))
    print("config2 parity", e)


@pytest.mark.parametrize("system", [0, 63])
def test_config3_dd_1024_jacobian(system):
    d = inputs.config3(system)
    e, g, o = check_case(d["A"], d["b"], 2, schedules=("resident", "panel"))
    print("config3 system %d parity" % system, e)


def test_no_rhs_and_in_place():
    p = inputs.random_problem(2, 150, 90, seed=3, config=52)
    A = T(p["A"])
    f = api.mgs_qr(A)
    Q1, R1 = N(f["Q"]), N(f["R"])
    assert f["y"] is None
    Ain = A.clone()
    f2 = api.mgs_qr(Ain, Q=Ain)
    torch.cuda.synchronize()
    assert np.array_equal(N(Ain), Q1)
    assert np.array_equal(N(f2["R"]), R1)
    o = oracle.mgs(p["A"])
    assert_parity(errors(p["A"], Q1, R1, o["Q"], o["R"]), 2)


@pytest.mark.parametrize("prec,m,n", [(2, 300, 200), (4, 90, 60)])
def test_ls_solve_projections(prec, m, n):
    p = inputs.random_problem(prec, m, n, seed=9, config=53)
    f = api.mgs_qr(T(p["A"]))
    x, info = api.ls_solve(f["Q"], f["R"], T(p["b"]))
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    o = oracle.mgs(p["A"])
    xo, _ = oracle.ls_solve(o["Q"], o["R"], p["b"])
    e = errors(p["A"], N(f["Q"]), N(f["R"]), o["Q"], o["R"], N(x), xo, None)
    assert_parity(e, prec)
    # the augmented path performs the same operations (different reduction tree)
    g = gpu_lstsq(p["A"], p["b"])
    assert_parity(errors(p["A"], g["Q"], g["R"], o["Q"], o["R"], g["x"], xo, None), prec)


@pytest.mark.parametrize("prec", [2, 4])
def test_backsolve_against_oracle(prec):
    p = inputs.random_problem(prec, 300, 300, seed=2, config=54)
    o = oracle.mgs(p["A"], p["b"])
    x, info = api.ls_backsolve(T(o["R"]), T(o["y"]))
    torch.cuda.synchronize()
    xo, _ = oracle.backsolve(o["R"], o["y"])
    d = diff(N(x), xo)
    assert int(info.item()) == 0
    assert np.sqrt(np.sum(d ** 2)) <= (1e-27 if prec == 2 else 1e-57) * np.sqrt(np.sum(value(xo) ** 2))


def test_zero_column_and_zero_pivot_report_info():
    p = inputs.random_problem(2, 80, 40, seed=4, config=55)
    A = p["A"].copy()
    A[:, :, 17] = 0.0
    for sched in ("auto", "panel"):
        g = gpu_lstsq(A, p["b"], sched)
        assert int(g["info"][0]) == 18, sched
    R = np.zeros((2, 2, 5, 5))
    R[0, 0, np.arange(5), np.arange(5)] = [1, 2, 0, 4, 5]
    y = np.ones((2, 2, 5))
    y[1] = 0
    x, info = api.ls_backsolve(T(R), T(y))
    torch.cuda.synchronize()
    assert int(info.item()) == 3


@pytest.mark.parametrize("m,n,sched", [(48, 30, "small"), (48, 30, "resident"), (48, 30, "panel"),
                                       (300, 200, "resident")])
def test_non_finite_column_reports_first(m, n, sched):
    """A NaN in column 7 and a zero column 12: info names column 8 (the
    first bad one, 1-based) on every schedule, and the run ends normally
    (the hand-offs carry NaNs without stalling)."""
    p = inputs.random_problem(2, m, n, seed=8, config=57)
    A = p["A"].copy()
    A[0, 0, 7, 3] = np.nan
    A[:, :, 12] = 0.0
    g = gpu_lstsq(A, p["b"], sched)
    assert int(g["info"][0]) == 8, sched


@pytest.mark.parametrize("m,n,sched", [(48, 30, "small"), (48, 30, "resident"), (48, 30, "panel"),
                                       (300, 200, "resident"), (300, 200, "panel")])
def test_marker_bit_pattern_input_reports_info(m, n, sched):
    """Entries holding the exact bit pattern the single-launch schedule uses
    to mark not-yet-written data (a signalling NaN) in columns 1 and 6:
    info names column 1 and the run ends normally on every schedule."""
    p = inputs.random_problem(2, m, n, seed=9, config=57)
    A = p["A"].copy()
    marker = np.array([0x7FF4A5A5A5A5A5A5], dtype=np.uint64).view(np.float64)[0]
    A[0, 0, 0, 5] = marker
    A[1, 1, 0, 9] = marker
    A[0, 1, 5, 2] = marker
    g = gpu_lstsq(A, p["b"], sched)
    assert int(g["info"][0]) == 1, sched


@pytest.mark.parametrize("sched", ["auto", "panel"])
def test_reproducible_bitwise(sched):
    p = inputs.random_problem(2, 700, 400, seed=5, config=56)
    g1 = gpu_lstsq(p["A"], p["b"], sched)
    g2 = gpu_lstsq(p["A"], p["b"], sched)
    for k in ("Q", "R", "y", "rho", "x"):
        assert np.array_equal(g1[k], g2[k]), k


@pytest.mark.parametrize("prec", [2, 4])
def test_scaling_and_real_symmetries_bitwise(prec):
    p = inputs.random_problem(prec, 130, 70, seed=6, config=57)
    A, b = p["A"], p["b"]
    g = gpu_lstsq(A, b)
    g2 = gpu_lstsq(A * 2.0 ** 40, b * 2.0 ** 40)
    assert np.array_equal(g2["Q"], g["Q"])
    assert np.array_equal(g2["R"], g["R"] * 2.0 ** 40)
    assert np.array_equal(g2["x"], g["x"])
    Ar, br = A.copy(), b.copy()
    Ar[:, 1] = 0
    br[:, 1] = 0
    gr = gpu_lstsq(Ar, br)
    assert np.all(gr["Q"][:, 1] == 0) and np.all(gr["R"][:, 1] == 0) and np.all(gr["x"][:, 1] == 0)


def test_resident_schedule_applies_where_documented():
    """The single-launch schedule is taken for dd with m <= 1024 and for
    double with m <= 2048, and refused (MGS_ERR_DIMS when it is required)
    for qd and beyond those rows."""
    from paper_1210_0800_amd import _lib

    for prec, m, n, ok in ((2, 1024, 1024, True), (2, 300, 200, True), (2, 1100, 40, False), (4, 300, 200, False),
                           (1, 2048, 64, True), (1, 700, 500, True), (1, 2100, 20, False)):
        p = inputs.random_problem(prec, m, n, seed=m + n, config=58)
        if ok:
            f = api.mgs_qr(T(p["A"]), T(p["b"]), schedule="resident")
            torch.cuda.synchronize()
            assert int(f["info"].item()) == 0
        else:
            with pytest.raises(_lib.MgsError) as e:
                api.mgs_qr(T(p["A"]), T(p["b"]), schedule="resident")
            assert e.value.status == -1
