"""Seeded synthetic inputs for the complex MGS least-squares solver.

This module only draws random numbers and assembles inputs; it holds none of
the solver's arithmetic and is the one piece shared by the HIP path's tests
and benchmark and by the CPU oracle's tests.

Every array is "planar" float64: a complex matrix of n columns and m rows in
L-limb precision has shape (L, 2, n, m) (limb, real/imag, column, row); a
vector has shape (L, 2, m).  Limbs are normalised, |x_{k+1}| <= ulp(x_k)/2.

Seeds: ``numpy.random.default_rng([12100800, config, system, role])`` with
roles 0 = A, 1 = x_true, 2 = b or noise, 3 = g (adjoint seed), 4 = sampled
entries.

Workloads (the paper draws random complex matrices, Section 8; the Jacobian
of a polynomial system of degree d holds values of modulus 10^(+-d),
Section 4):

* ``config1`` -- dd, 32 x 32, re/im hi limbs U[-1,1], lo = hi 2^-53 U[-1,1];
  x_true alike; b = A x_true rounded to dd from the exact sum
  (``config1_batch``: systems 0, 1, ... of the same recipe, for batches).
* ``config2`` -- qd, 320 x 256, limb k = hi 2^(-53k) U_k[-1,1]; b = A x_true
  + noise of modulus 1e-40, rounded to qd from the exact sum.
* ``config3`` -- dd, 1024 x 1024 systems (64 back to back): re, im ~ N(0,1),
  column j scaled by fl(10^s_j), s_j ~ U[-12,12]; each entry is the exact
  dd product of the scale and the Gaussian; x_true complex N(0,1);
  b = A x_true to dd accuracy.
* ``config4`` -- n x n (2048) A = U diag(sigma) V^H in FP64, U and V products
  of 4 Householder reflectors with complex N(0,1) vectors, sigma geometric
  from 1 to 1e-10; x_true complex N(0,1); b = A x_true rounded to qd from the
  exact sum, so that x_true solves the stored system to about
  kappa 2^-212 (the reference for the precision form); with ``tail`` the
  matrix carries a second limb below FP64 (relative 2^-60), so the FP64
  factorisation factors only an approximation of it, and b stays exact in
  qd.
* ``config5`` -- dd, 512 x 384, A, b, g with N(0,1) hi limbs.
* ``table2_matrix`` -- 32 x 32 entries r e^{i theta}, theta ~ U[0, 2 pi),
  log10 r ~ U[-g, g] (Section 4, Table 2).
"""
import numpy as np

SEED0 = 12100800


def rng(config, system=0, role=0):
    return np.random.default_rng([SEED0, int(config), int(system), int(role)])


# ----------------------------------------------------------- limb assembly --
def _two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def normalize(limbs):
    """Exactly re-express sum(limbs) as normalised limbs (same count).

    Repeated TwoSum distillation; every step is error free, so the value is
    unchanged.  Verifies |x_{k+1}| <= ulp(x_k)/2 on return.
    """
    x = [np.array(v, dtype=np.float64, copy=True) for v in limbs]
    L = len(x)
    out = []
    rest = x
    for _ in range(L):
        for _ in range(4):
            for i in range(len(rest) - 1, 0, -1):
                rest[i - 1], rest[i] = _two_sum(rest[i - 1], rest[i])
        out.append(rest[0])
        rest = rest[1:]
    for _ in range(8):
        ok = True
        for k in range(L - 1):
            s, e = _two_sum(out[k], out[k + 1])
            out[k], out[k + 1] = s, e
        for k in range(L - 1):
            if np.any(np.abs(out[k + 1]) > 0.5 * np.spacing(np.abs(out[k]))):
                ok = False
        if ok:
            break
    else:
        raise RuntimeError("limb normalisation did not converge")
    return out


def random_limbs(g, shape, L, dist="uniform"):
    """Random L-limb reals: hi from `dist`, limb k = hi 2^(-53k) U_k[-1,1]."""
    if dist == "uniform":
        hi = g.uniform(-1.0, 1.0, shape)
    elif dist == "normal":
        hi = g.standard_normal(shape)
    else:
        raise ValueError(dist)
    limbs = [hi] + [hi * 2.0 ** (-53 * k) * g.uniform(-1.0, 1.0, shape) for k in range(1, L)]
    return np.stack(normalize(limbs)) if L > 1 else hi[None]


def random_complex(g, shape, L, dist="uniform"):
    """Planar (L, 2, *shape) complex numbers, real then imaginary draws."""
    re = random_limbs(g, shape, L, dist)
    im = random_limbs(g, shape, L, dist)
    return np.ascontiguousarray(np.stack([re, im], axis=1))


# ------------------------------------------------- exact right-hand sides --
def _to_int(v, S):
    """Exact integer v * 2^S for a float64 array v (|v| >= 2^-S)."""
    out = []
    for f in np.asarray(v, dtype=np.float64).ravel().tolist():
        num, den = f.as_integer_ratio()
        out.append(num << (S - den.bit_length() + 1))
    return out


def _round_int(t, S, L):
    """Round the exact value t / 2^S to L normalised float64 limbs."""
    limbs = []
    for _ in range(L):
        f = t / (1 << S) if t != 0 else 0.0  # int / int is correctly rounded
        limbs.append(f)
        if f != 0.0:
            num, den = f.as_integer_ratio()
            t -= num << (S - den.bit_length() + 1)
    return limbs


def _exact_rows(args):
    """Rows [i0, i1) of the exact product, rounded to L_out limbs."""
    Ar, Ai, xr, xi, er, ei, m, n, i0, i1, S, L_out = args
    out = np.zeros((L_out, 2, i1 - i0))
    for i in range(i0, i1):
        sr, si = er[i], ei[i]
        for j in range(n):
            a_r, a_i = Ar[j * m + i], Ai[j * m + i]
            sr += a_r * xr[j] - a_i * xi[j]
            si += a_r * xi[j] + a_i * xr[j]
        out[:, 0, i - i0] = _round_int(sr, 2 * S, L_out)
        out[:, 1, i - i0] = _round_int(si, 2 * S, L_out)
    return out


def exact_matvec(A, x, L_out, extra=None, workers=1):
    """Round-to-L_out-limbs of the exact product A x (+ extra), Python integers.

    Rows are independent; `workers` > 1 splits them over forked processes.
    """
    La, _, n, m = A.shape
    S = 1200
    Ar = [sum(col) for col in zip(*[_to_int(A[l, 0], S) for l in range(La)])]
    Ai = [sum(col) for col in zip(*[_to_int(A[l, 1], S) for l in range(La)])]
    Lx = x.shape[0]
    xr = [sum(c) for c in zip(*[_to_int(x[l, 0], S) for l in range(Lx)])]
    xi = [sum(c) for c in zip(*[_to_int(x[l, 1], S) for l in range(Lx)])]
    if extra is not None:
        Le = extra.shape[0]
        er = [sum(c) << S for c in zip(*[_to_int(extra[l, 0], S) for l in range(Le)])]
        ei = [sum(c) << S for c in zip(*[_to_int(extra[l, 1], S) for l in range(Le)])]
    else:
        er = [0] * m
        ei = [0] * m
    if workers <= 1 or m < 64:
        return _exact_rows((Ar, Ai, xr, xi, er, ei, m, n, 0, m, S, L_out))
    import multiprocessing as mp
    bounds = np.linspace(0, m, workers + 1).astype(int)
    global _EXACT_SHARED
    _EXACT_SHARED = (Ar, Ai, xr, xi, er, ei)
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_exact_rows_shared, [(m, n, int(a), int(b), S, L_out) for a, b in zip(bounds[:-1], bounds[1:])])
    return np.concatenate(parts, axis=2)


_EXACT_SHARED = None


def _exact_rows_shared(args):
    m, n, i0, i1, S, L_out = args
    return _exact_rows(_EXACT_SHARED + (m, n, i0, i1, S, L_out))


def _split(a):
    c = 134217729.0 * a
    h = c - (c - a)
    return h, a - h


def _two_prod(a, b):
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    return p, ((ah * bh - p) + ah * bl + al * bh) + al * bl


def dd_matvec_dx(A, x):
    """b = A x for dd A (2,2,n,m) and FP64 x (1,2,n), to dd accuracy.

    Leading products split exactly (TwoProd), summed over the columns by a
    pairwise TwoSum tree; every rounding error and every low-limb product is
    gathered in one FP64 array; the pair is renormalised at the end.
    """
    _, _, n, m = A.shape
    xr, xi = x[0, 0][:, None], x[0, 1][:, None]
    b = np.zeros((2, 2, m))
    for comp in range(2):
        if comp == 0:  # ar xr - ai xi
            terms = ((A[0, 0], A[1, 0], xr), (A[0, 1], A[1, 1], -xi))
        else:  # ar xi + ai xr
            terms = ((A[0, 0], A[1, 0], xi), (A[0, 1], A[1, 1], xr))
        hs, lows = [], 0.0
        for h, lo, xv in terms:
            p, e = _two_prod(h, np.broadcast_to(xv, h.shape))
            hs.append(p)
            lows = lows + np.sum(e + lo * xv, axis=0)
        S = np.concatenate(hs, axis=0)
        while S.shape[0] > 1:
            if S.shape[0] % 2:
                S = np.concatenate([S, np.zeros((1, m))], axis=0)
            s, t = _two_sum(S[0::2], S[1::2])
            lows = lows + np.sum(t, axis=0)
            S = s
        b[0, comp], b[1, comp] = _two_sum(S[0], lows)
    return b


# ----------------------------------------------------------------- configs --
def config1(system=0):
    """dd 32 x 32 (configuration 1; `system` numbers independent draws).
    Returns dict(A, b, x_true, prec)."""
    m = n = 32
    A = random_complex(rng(1, system, 0), (n, m), 2)
    x = random_complex(rng(1, system, 1), (n,), 2)
    b = exact_matvec(A, x, 2)
    return dict(A=A, b=b, x_true=x, prec=2, m=m, n=n)


def _config1_arrays(system):
    d = config1(system)
    return d["A"], d["b"], d["x_true"]


def config1_batch(count, first=0, workers=1):
    """Systems first .. first+count-1 of configuration 1, stacked on a leading
    batch axis: dict(A (count,2,2,32,32), b, x_true (count,2,2,32))."""
    ids = range(first, first + count)
    if workers > 1 and count > 1:
        import multiprocessing as mp

        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_config1_arrays, ids, chunksize=max(1, count // (4 * workers)))
    else:
        parts = [_config1_arrays(i) for i in ids]
    return dict(A=np.ascontiguousarray(np.stack([p[0] for p in parts])),
                b=np.ascontiguousarray(np.stack([p[1] for p in parts])),
                x_true=np.ascontiguousarray(np.stack([p[2] for p in parts])), prec=2, m=32, n=32)


def config2():
    """qd 320 x 256 overdetermined with 1e-40 noise (configuration 2)."""
    m, n = 320, 256
    A = random_complex(rng(2, 0, 0), (n, m), 4)
    x = random_complex(rng(2, 0, 1), (n,), 4)
    noise = random_complex(rng(2, 0, 2), (m,), 4) * 1e-40
    noise = np.stack([np.stack(normalize(list(noise[:, p]))) for p in range(2)], axis=1)
    b = exact_matvec(A, x, 4, extra=noise)
    return dict(A=A, b=b, x_true=x, prec=4, m=m, n=n)


def config3(system=0, m=1024, n=1024):
    """One dd Jacobian-like system with column scales 10^s, s ~ U[-12,12]."""
    g = rng(3, system, 0)
    G = g.standard_normal((2, n, m))
    s = g.uniform(-12.0, 12.0, n)
    c = 10.0 ** s
    A = np.zeros((2, 2, n, m))
    for p in range(2):
        # TwoProd output is a normalised dd: |lo| <= ulp(hi) / 2
        A[0, p], A[1, p] = _two_prod(c[:, None], G[p])
    xg = rng(3, system, 1)
    x = np.zeros((1, 2, n))
    x[0] = xg.standard_normal((2, n))
    b = dd_matvec_dx(A, x)
    x2 = np.zeros((2, 2, n))
    x2[0] = x[0]
    return dict(A=np.ascontiguousarray(A), b=np.ascontiguousarray(b), x_true=x2, prec=2, m=m, n=n,
                scales=c)


def config4(n=2048, reflectors=4, cond=1e10, workers=1, tail=False):
    """Precision-form workload: FP64 A = U diag(sigma) V^H, b exact to qd.

    With tail=True the matrix also carries information below FP64: entry a
    becomes a + a 2^-60 u, u ~ U[-1,1] (role 6), a second limb that FP64
    drops, stored with 2 limbs ("A2") and with 4 ("A4", two zero limbs).
    Each product of A and x_true then has at most 166 significant bits, so
    b4 = A x_true is exact in qd (x_true solves the qd system exactly) and
    b2 is its leading two limbs."""
    g = rng(4, 0, 5)
    sigma = cond ** (-np.arange(n) / (n - 1.0))
    M = np.diag(sigma).astype(np.complex128)
    for _ in range(reflectors):  # M <- M H, H = I - 2 v v^H / (v^H v)
        v = g.standard_normal(n) + 1j * g.standard_normal(n)
        M = M - (2.0 / np.vdot(v, v).real) * np.outer(M @ v, v.conj())
    for _ in range(reflectors):  # M <- H M
        u = g.standard_normal(n) + 1j * g.standard_normal(n)
        M = M - (2.0 / np.vdot(u, u).real) * np.outer(u, u.conj() @ M)
    A1 = np.zeros((1, 2, n, n))
    A1[0, 0] = M.real.T
    A1[0, 1] = M.imag.T
    xg = rng(4, 0, 1)
    x = np.zeros((1, 2, n))
    x[0] = xg.standard_normal((2, n))
    if not tail:
        b4 = exact_matvec(A1, x, 4, workers=workers)
        return dict(A64=np.ascontiguousarray(A1), b4=b4, x_true=x, sigma=sigma, n=n, m=n)
    tg = rng(4, 0, 6)
    A2 = np.zeros((2,) + A1.shape[1:])
    A2[0] = A1[0]
    A2[1] = A1[0] * 2.0 ** -60 * tg.uniform(-1.0, 1.0, A1[0].shape)  # |.| <= ulp(a) / 2: normalised
    A4 = np.zeros((4,) + A1.shape[1:])
    A4[:2] = A2
    b4 = exact_matvec(A2, x, 4, workers=workers)
    return dict(A64=np.ascontiguousarray(A1), A4=A4, A2=A2, b4=b4, b2=np.ascontiguousarray(b4[:2]), x_true=x,
                sigma=sigma, n=n, m=n)


def config5():
    """dd 512 x 384 Gaussian A, b and adjoint seed g (configuration 5)."""
    m, n = 512, 384
    A = random_complex(rng(5, 0, 0), (n, m), 2, "normal")
    b = random_complex(rng(5, 0, 2), (m,), 2, "normal")
    gx = random_complex(rng(5, 0, 3), (n,), 2, "normal")
    return dict(A=A, b=b, g=gx, prec=2, m=m, n=n)


def polysys(neq=32, nvar=32, nmon=32, nvpm=5, maxdeg=5, L=2, system=0):
    """Polynomial system of the paper's Table 6 shape (Section 7: Newton
    corrector; 32 equations in 32 variables, 32 monomials per equation, 5
    distinct variables per monomial, degrees uniform in 1..maxdeg), with a
    known root x* whose entries are 1, -1, i or -i (role 6).

    Coefficients are dyadic complex numbers k/64, |k| <= 64 (role 0); the
    first monomial's coefficient of each equation is then set to
    -sum_{m>0} c_m mono_m(x*) / mono_0(x*), exact in FP64 since every
    monomial value at x* is a power of i.  So f(x*) = 0 exactly.  Returns
    dict(vars, exps [neq, nmon, nvpm] int32, coef (L, 2, neq, nmon), nvar,
    root (L, 2, nvar))."""
    g = rng(6, system, 0)
    vars_ = np.zeros((neq, nmon, nvpm), dtype=np.int32)
    exps = g.integers(1, maxdeg + 1, size=(neq, nmon, nvpm)).astype(np.int32)
    for e in range(neq):
        for m in range(nmon):
            vars_[e, m] = g.choice(nvar, nvpm, replace=False)
    cre = g.integers(-64, 65, size=(neq, nmon)) / 64.0
    cim = g.integers(-64, 65, size=(neq, nmon)) / 64.0
    rg = rng(6, system, 6)
    root_pow = rg.integers(0, 4, size=nvar)  # x*_j = i^root_pow[j]
    units = [1, 1j, -1, -1j]
    coef = cre + 1j * cim
    for e in range(neq):
        vals = [units[int(np.sum(exps[e, m] * root_pow[vars_[e, m]])) % 4] for m in range(nmon)]
        rest = sum(coef[e, m] * vals[m] for m in range(1, nmon))
        coef[e, 0] = -rest / vals[0]
    C = np.zeros((L, 2, neq, nmon))
    C[0, 0], C[0, 1] = coef.real, coef.imag
    root = np.zeros((L, 2, nvar))
    rv = np.array([units[p] for p in root_pow])
    root[0, 0], root[0, 1] = rv.real, rv.imag
    return dict(vars=vars_, exps=exps, coef=C, nvar=nvar, root=root)


def near_root(sys, scale=1e-3, L=2, system=0):
    """A start point x* + delta, delta complex with entries scale * U[-1,1]
    (role 7), as the predictor of a path tracker would hand the corrector."""
    g = rng(6, system, 7)
    x = np.zeros((L,) + sys["root"].shape[1:])
    x[0] = sys["root"][0] + scale * g.uniform(-1.0, 1.0, sys["root"].shape[1:])
    return x


def random_problem(prec, m, n, seed=0, dist="uniform", config=0):
    """Generic seeded test problem: A (prec,2,n,m) and b (prec,2,m)."""
    A = random_complex(rng(config, seed, 0), (n, m), prec, dist)
    b = random_complex(rng(config, seed, 2), (m,), prec, dist)
    return dict(A=A, b=b, prec=prec, m=m, n=n)


def table2_matrix(g_rng, g, L, m=32, n=32):
    """Table 2 workload: entries r e^{i theta}, log10 r ~ U[-g, g] (FP64 values)."""
    th = g_rng.uniform(0.0, 2.0 * np.pi, (n, m))
    r = 10.0 ** g_rng.uniform(-g, g, (n, m))
    A = np.zeros((L, 2, n, m))
    A[0, 0] = r * np.cos(th)
    A[0, 1] = r * np.sin(th)
    return A
