"""Benchmark: complex double-double MGS least squares on MI355X.

Workload (one "step"): 64 Jacobian-like complex dd systems of size
1024 x 1024 (columns scaled by 10^s, s ~ U[-12, 12]) solved back to back on
one stream, as the Newton corrections along one path: for each system, MGS
on [A b] (mgs_qr) then back substitution (ls_backsolve).  Inputs are
resident in HBM before the timed region.

Prints one JSON line: solves/s, the roofline of the dominant kernel sequence
(the MGS factorisation, FP64 vector ALU bound), the CPU oracle baseline and
the precision form measured against plain MGS at equal error on the
2048 x 2048, kappa = 1e10 workload (time, error against x_true, iterations,
in dd and qd), small square solves beside the paper's Tesla C2050
figures (context only), and batches of 10,000 independent 32 x 32 systems
in one call (double, dd, qd).

--copy-probe BYTES only copies a device buffer of that size (for scaling the
HBM counters of a profiler run) and exits.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dd/qd MGS least-squares solves/s & %FP64 peak; refined vs plain at equal error"
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk

# FP64 flops per operation of the dd kernels (FMA = 2), counted from the
# formulations in paper_1210_0800_amd/csrc/ddqd.hpp.
F_DD = dict(cmulc=60, upd=66, abs2=28, scale=20, merge=16)


# HBM bytes per launch of the resident factorisation kernel (dd 1024 x 1024
# with b), from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs of this
# benchmark, each scaled by the same counter on a device copy of known size
# (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0; see profiles/).  Valid only for the
# kernel sources and the launch code they were taken on (hash below: the
# kernel's header whole, the dd and FP64 arithmetic and the precision
# policies (not the qd functions, which it does not use), of mgs_kernels.hpp
# the helpers it uses, of mgsqr.hip the part that plans and launches the
# single-launch factorisation); reported as null otherwise.
TRAFFIC = dict(fetch_bytes=2.0 * 1.595e5 * 1024, write_bytes=1.687e5 * 1024, sources="6b02a83aa1e85c44")
KERNEL_SOURCES = ["paper_1210_0800_amd/csrc/resident_kernels.hpp",
                  ("paper_1210_0800_amd/csrc/ddqd.hpp", "// Device arithmetic", "// " + "-" * 67 + " qd --"),
                  ("paper_1210_0800_amd/csrc/ddqd.hpp", "// " + "-" * 57 + " precisions ----", None),
                  ("paper_1210_0800_amd/csrc/mgs_kernels.hpp", "// MGS QR, least-squares", "struct StepArgs {"),
                  ("paper_1210_0800_amd/csrc/mgsqr.hip", "// Columns held by the workgroup holding the most",
                   "// dd systems of at most SMALL_MAX_ROWS")]


def _source_part(entry):
    if isinstance(entry, str):
        with open(os.path.join(ROOT, entry), "rb") as fh:
            return fh.read()
    path, start, end = entry
    with open(os.path.join(ROOT, path), "rb") as fh:
        text = fh.read()
    i = text.find(start.encode())
    j = len(text) if end is None else text.find(end.encode(), i + 1)
    return text[i:j] if 0 <= i < j else text


def traffic_bytes():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(_source_part(f))
    if h.hexdigest()[:16] != TRAFFIC["sources"]:
        return None
    return TRAFFIC["fetch_bytes"] + TRAFFIC["write_bytes"]


def mgs_flops(m, n, ncols, F=F_DD):
    """Algorithmic FP64 flops of MGS on m x ncols (n normalised columns)."""
    total = 0
    for k in range(n):
        rest = ncols - k - 1
        total += m * F["abs2"] + (m - 1) * F["merge"] // 2 + m * F["scale"]
        total += rest * (m * (F["cmulc"] + F["upd"]) + (m - 1) * F["merge"])
    return total


def backsolve_flops(n, F=F_DD):
    return n * (n - 1) // 2 * F["upd"] + n * F["scale"]


def _gen(i):
    from paper_1210_0800_amd import inputs

    d = inputs.config3(i)
    return d["A"], d["b"]


def make_inputs(nsys, workers):
    if workers <= 1:
        return [_gen(i) for i in range(nsys)]
    import multiprocessing as mp

    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_gen, range(nsys))


def cpu_baseline(inputs_np, budget_s=20.0):
    """Oracle (test infrastructure) timed on the host: whole dd 1024x1024 solves."""
    import oracle

    threads = len(os.sched_getaffinity(0))
    done, t0 = 0, time.perf_counter()
    for A, b in inputs_np:
        o = oracle.mgs(A, b, nthreads=threads)
        oracle.backsolve(o["R"], o["y"])
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="solves/s", cores=threads, kind="oracle",
                sample="%d of the 64 dd 1024x1024 systems (MGS on [A b] + back substitution), %.1f s" %
                (done, dt))


def _exact_rel_err(x, x_true):
    """||x - x_true|| / ||x_true|| with the differences formed exactly
    (limb sums as rationals), then rounded to FP64."""
    from fractions import Fraction

    def vals(X):
        Xs = X.reshape(X.shape[0], -1)
        return [sum(Fraction(float(v)) for v in Xs[:, i]) for i in range(Xs.shape[1])]

    a, t = vals(x), vals(x_true)
    num = sum(float(u - v) ** 2 for u, v in zip(a, t))
    den = sum(float(v) ** 2 for v in t)
    return (num / den) ** 0.5


def precision_form(torch, api, n=2048, reps=2):
    """Refined (FP64 blocked MGS + dd/qd refinement) vs plain dd/qd MGS on
    A = U diag(sigma) V^H, kappa 1e10, b the exact product A x_true rounded
    to qd: time of each, relative error against x_true, iterations."""
    from paper_1210_0800_amd import inputs

    t_gen = time.perf_counter()
    d = inputs.config4(n, workers=min(16, len(os.sched_getaffinity(0))))
    t_gen = time.perf_counter() - t_gen
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = {"workload": "complex %dx%d A = U diag(sigma) V^H (4+4 Householder reflectors, sigma log-spaced, "
                       "kappa 1e10), b = A x_true exactly rounded to qd" % (n, n),
           "inputs_s": t_gen}
    # loss of orthogonality of the FP64 blocked factors (mgs_qr64)
    f64 = api.mgs_qr64(torch.from_numpy(np.ascontiguousarray(d["A64"][0])).to(dev))
    torch.cuda.synchronize()
    Qh = f64["Q"].cpu().numpy()
    Qc = (Qh[0] + 1j * Qh[1]).T
    out["fp64_orthogonality"] = float(np.linalg.norm(Qc.conj().T @ Qc - np.eye(n), 2))
    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            r = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1) / reps

    for L, name in ((2, "dd"), (4, "qd")):
        A = np.zeros((L,) + d["A64"].shape[1:])
        A[0] = d["A64"][0]
        At = torch.from_numpy(A).to(dev)
        bt = torch.from_numpy(np.ascontiguousarray(d["b4"][:L])).to(dev)
        fp, tp = timed(lambda: api.lstsq(At, bt))
        fr, tr = timed(lambda: api.refine_lstsq(At, bt, max_iter=30))
        ep = _exact_rel_err(fp["x"].cpu().numpy(), d["x_true"])
        er = _exact_rel_err(fr["x"].cpu().numpy(), d["x_true"])
        iters = int(fr["iters"].item())
        # error after 0, 1, ..., iters refinement steps (x_0: the FP64 solve)
        hist = []
        for k in range(iters + 1):
            fk = api.refine_lstsq(At, bt, max_iter=k)
            torch.cuda.synchronize()
            hist.append(_exact_rel_err(fk["x"].cpu().numpy(), d["x_true"]))
        out[name] = {"plain_ms": tp, "refined_ms": tr, "plain_err": ep, "refined_err": er,
                     "iters": iters, "info": int(fr["info"].item()),
                     "speedup": tp / tr, "refined_reaches_plain_error": er <= ep,
                     "refined_within_10x_plain_error": er <= 10 * ep,
                     "err_by_iteration": hist,
                     "contraction": [hist[k + 1] / hist[k] for k in range(len(hist) - 1) if hist[k] > 0]}
        print("bench: precision form %s plain %.1f ms err %.2e | refined %.1f ms err %.2e iters %d" %
              (name, tp, ep, tr, er, out[name]["iters"]), file=sys.stderr, flush=True)
    # the same matrix with a second limb of relative size 2^-60 (below what
    # the FP64 factorisation sees), b = A x_true still exact in qd
    del d
    t_gen = time.perf_counter()
    dt = inputs.config4(n, workers=min(16, len(os.sched_getaffinity(0))), tail=True)
    sub = {"workload": "the same A with a second limb a 2^-60 u, u ~ U[-1,1]; b = A x_true exact in qd",
           "inputs_s": time.perf_counter() - t_gen}
    for L, name, Ak, bk in ((2, "dd", "A2", "b2"), (4, "qd", "A4", "b4")):
        At = torch.from_numpy(np.ascontiguousarray(dt[Ak])).to(dev)
        bt = torch.from_numpy(np.ascontiguousarray(dt[bk])).to(dev)
        fp, tp = timed(lambda: api.lstsq(At, bt))
        fr, tr = timed(lambda: api.refine_lstsq(At, bt, max_iter=30))
        ep = _exact_rel_err(fp["x"].cpu().numpy(), dt["x_true"])
        er = _exact_rel_err(fr["x"].cpu().numpy(), dt["x_true"])
        sub[name] = {"plain_ms": tp, "refined_ms": tr, "plain_err": ep, "refined_err": er,
                     "iters": int(fr["iters"].item()), "info": int(fr["info"].item()), "speedup": tp / tr,
                     "refined_reaches_plain_error": er <= ep}
        print("bench: precision form (sub-FP64 limb) %s plain %.1f ms err %.2e | refined %.1f ms err %.2e iters %d"
              % (name, tp, ep, tr, er, sub[name]["iters"]), file=sys.stderr, flush=True)
    out["subfp64_A"] = sub
    return out


# The paper's Tesla C2050 figures (Table 5: 10,000 runs of MGS followed by
# one back substitution, square random complex matrices), as solves/s.
PAPER_C2050_SOLVES_PER_S = {("dd", 32): 10000 / 22.44, ("dd", 80): 10000 / 79.11,
                            ("qd", 32): 10000 / 155.32, ("qd", 80): 10000 / 597.47,
                            # Table 4: complex double
                            ("d", 32): 10000 / 6.52, ("d", 80): 10000 / 22.89, ("d", 128): 10000 / 49.10,
                            ("d", 256): 10000 / 234.29}


def paper_context(torch, api, solves=2000):
    """Small square solves back to back on one stream, as the paper times
    them, beside its C2050 numbers (other hardware: context, not a target)."""
    from paper_1210_0800_amd import inputs

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = {"protocol": "%d back-to-back MGS on [A b] + back substitution, square random complex A "
                       "(re/im of every limb level ~ U[-1,1]), one stream" % solves,
           "paper_hardware": "NVIDIA Tesla C2050 (1147 MHz), CUDA 4.0; paper Tables 4 (double) and 5 (dd, qd)"}
    for prec, name, sizes in ((1, "d", (32, 80, 128, 256)), (2, "dd", (32, 80)), (4, "qd", (32, 80))):
        for n in sizes:
            p = inputs.random_problem(prec, n, n, seed=n, config=80)
            A, b = torch.from_numpy(p["A"]).to(dev), torch.from_numpy(p["b"]).to(dev)
            Q = torch.empty_like(A)
            R = torch.empty((prec, 2, n, n), dtype=torch.float64, device=dev)
            y = torch.empty((prec, 2, n), dtype=torch.float64, device=dev)
            x = torch.empty_like(y)
            info = torch.empty(1, dtype=torch.int32, device=dev)
            info2 = torch.empty(1, dtype=torch.int32, device=dev)
            work = api.workspace(n, n, prec, 0, dev)

            def one():
                api.mgs_qr(A, b, Q=Q, R=R, y=y, info=info, work=work, with_rho=False)
                api.ls_backsolve(R, y, x=x, info=info2)

            for _ in range(20):
                one()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(solves):
                one()
            e1.record(stream)
            torch.cuda.synchronize()
            rate = solves / (e0.elapsed_time(e1) * 1e-3)
            paper = PAPER_C2050_SOLVES_PER_S[(name, n)]
            out["%s_n%d" % (name, n)] = {"solves_per_s": rate, "paper_c2050_solves_per_s": paper,
                                         "ratio": rate / paper}
            print("bench: context %s n=%d: %.0f solves/s (paper C2050 %.1f)" % (name, n, rate, paper),
                  file=sys.stderr, flush=True)
    return out


def _rate(torch, fn, reps, warm=5):
    """Calls per second of fn() back to back on the current stream."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return reps / (e0.elapsed_time(e1) * 1e-3)


def workloads(torch, api):
    """The other configurations of the workload table, each with its own
    protocol: dd 32 x 32 (10,000 back-to-back solves, as the paper times its
    small systems), qd 320 x 256 overdetermined (200 back-to-back solves),
    and dd 512 x 384 with the adjoint (forward and backward timed apart)."""
    from paper_1210_0800_amd import inputs

    dev = torch.device("cuda:0")
    out = {}

    def solver(d, prec):
        A, b = torch.from_numpy(d["A"]).to(dev), torch.from_numpy(d["b"]).to(dev)
        m, n = d["m"], d["n"]
        Q = torch.empty_like(A)
        R = torch.empty((prec, 2, n, n), dtype=torch.float64, device=dev)
        y = torch.empty((prec, 2, n), dtype=torch.float64, device=dev)
        x = torch.empty_like(y)
        info = torch.empty(1, dtype=torch.int32, device=dev)
        info2 = torch.empty(1, dtype=torch.int32, device=dev)
        work = api.workspace(m, n, prec, 0, dev)

        def one():
            api.mgs_qr(A, b, Q=Q, R=R, y=y, info=info, work=work, with_rho=False)
            api.ls_backsolve(R, y, x=x, info=info2)

        return one, (A, b, Q, R, x, info, info2)

    d1 = inputs.config1()
    one, _ = solver(d1, 2)
    r1 = _rate(torch, one, 10000)
    out["dd_32x32"] = {"solves_per_s": r1, "protocol": "10000 back-to-back solves (MGS on [A b] + back substitution)"}
    print("bench: workload dd 32x32: %.0f solves/s" % r1, file=sys.stderr, flush=True)

    d2 = inputs.config2()
    one, _ = solver(d2, 4)
    r2 = _rate(torch, one, 200)
    out["qd_320x256"] = {"solves_per_s": r2, "protocol": "200 back-to-back solves, noise 1e-40"}
    print("bench: workload qd 320x256: %.0f solves/s" % r2, file=sys.stderr, flush=True)

    d5 = inputs.config5()
    one, (A, b, Q, R, x, info, info2) = solver(d5, 2)
    fwd = _rate(torch, one, 200)
    g = torch.from_numpy(d5["g"]).to(dev)
    gA, gb = torch.empty_like(A), torch.empty_like(b)
    ia = torch.empty(1, dtype=torch.int32, device=dev)
    wa = api.workspace(d5["m"], d5["n"], 2, 2, dev)

    def back():
        api.ls_adjoint(A, b, Q, R, x, g, gA=gA, gb=gb, info=ia, work=wa)

    bwd = _rate(torch, back, 200)
    out["dd_512x384_adjoint"] = {"forward_ms": 1e3 / fwd, "backward_ms": 1e3 / bwd,
                                 "protocol": "200 forward solves, then 200 adjoint evaluations (dL/dA, dL/db)"}
    print("bench: workload dd 512x384: forward %.3f ms, backward %.3f ms" % (1e3 / fwd, 1e3 / bwd),
          file=sys.stderr, flush=True)
    return out


def batched(torch, api, count=10000, reps=5):
    """Many independent systems in one call (mgs_lstsq_batched, one
    workgroup per system): `count` dd systems of configuration 1 (32 x 32),
    and as many random 32 x 32 systems in complex double and qd."""
    from paper_1210_0800_amd import inputs

    dev = torch.device("cuda:0")
    out = {"protocol": "one mgs_lstsq_batched call of %d systems (MGS on [A b] + back substitution each), "
                       "mean of %d calls after one warm-up" % (count, reps)}
    t = time.perf_counter()
    d1 = inputs.config1_batch(count, workers=min(16, len(os.sched_getaffinity(0))))
    gen = time.perf_counter() - t
    cases = [("dd_32x32_config1", d1["A"], d1["b"], 2)]
    for prec, name in ((1, "d_32x32"), (4, "qd_32x32")):
        g = inputs.rng(81, prec, 0)
        A = np.stack([inputs.random_complex(g, (32, 32), prec) for _ in range(count)])
        b = np.stack([inputs.random_complex(g, (32,), prec) for _ in range(count)])
        cases.append((name, A, b, prec))
    for name, A, b, prec in cases:
        At, bt = torch.from_numpy(np.ascontiguousarray(A)).to(dev), torch.from_numpy(np.ascontiguousarray(b)).to(dev)
        f = api.lstsq_batched(At, bt)
        torch.cuda.synchronize()
        bad = int((f["info"] != 0).sum().item())

        def one():
            api.lstsq_batched(At, bt, Q=f["Q"], R=f["R"], x=f["x"], info=f["info"])

        rate = _rate(torch, one, reps, warm=1) * count
        out[name] = {"systems_per_s": rate, "failed_systems": bad, "systems": count}
        print("bench: batched %s: %.0f systems/s (%d systems per call)" % (name, rate, count),
              file=sys.stderr, flush=True)
    out["inputs_s"] = gen
    return out


# The paper's Table 6, GPU column: seconds for 10,000 polynomial evaluations
# and differentiations plus 10,000 MGS orthogonalisations of the 32 x 32
# system (C2050; other hardware: context, not a target).
PAPER_C2050_PE_MGS_S = {"d": 6.6, "dd": 18.6, "qd": 122.2}


def newton_context(torch, api, steps=None, paths=1024, path_steps=5):
    """The on-card Newton corrector on the Table 6 system shape (32
    equations, 32 variables, 32 monomials of 5 variables, degrees 1..5):
    one path, `steps` sequential Newton steps (evaluation, MGS on [J -f],
    back substitution, update) in one mgs_newton_batched call; and `paths`
    independent paths, `path_steps` steps each, in one call."""
    from paper_1210_0800_amd import inputs

    dev = torch.device("cuda:0")
    steps = steps or {"d": 2000, "dd": 2000, "qd": 400}
    out = {"protocol": "mgs_newton_batched on a seeded system with a known root, start 1e-3 from it; "
                       "sequential: one path, steps back to back in one call; batched: %d paths x %d steps "
                       "in one call" % (paths, path_steps),
           "paper_hardware": "NVIDIA Tesla C2050; paper Table 6 (PE + MGS, GPU, per 10,000)"}
    for prec, name in ((1, "d"), (2, "dd"), (4, "qd")):
        s = inputs.polysys(L=prec, system=0)
        sysd = api.PolySystem(s["vars"], s["exps"], s["coef"], s["nvar"], dev)
        x0 = np.stack([inputs.near_root(s, 1e-3, L=prec, system=k) for k in range(paths)])
        X1 = torch.from_numpy(x0[:1]).to(dev)
        Xb = torch.from_numpy(x0).to(dev)
        k = steps[name]
        x = X1.clone()
        r = api.newton_batched(sysd, x, k, dnorm=False)
        torch.cuda.synchronize()
        ok = int((r["info"] != 0).sum().item()) == 0
        seq = _rate(torch, lambda: api.newton_batched(sysd, x, k, dnorm=False), 2, warm=1) * k
        xb = Xb.clone()
        bat = _rate(torch, lambda: api.newton_batched(sysd, xb, path_steps, dnorm=False), 3, warm=1)
        bat *= paths * path_steps
        paper = 10000 / PAPER_C2050_PE_MGS_S[name]
        out[name] = {"sequential_steps_per_s": seq, "batched_point_steps_per_s": bat, "info_ok": ok,
                     "paper_c2050_pe_mgs_per_s": paper, "sequential_ratio": seq / paper}
        print("bench: newton %s: %.0f steps/s on one path, %.0f point-steps/s over %d paths (paper C2050 %.0f/s)"
              % (name, seq, bat, paths, paper), file=sys.stderr, flush=True)
    return out


# FP64 flops of one qd 1024 x 1024 factorisation of [A b] (per-panel
# schedule), counted by rocprofv3 (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 x 64
# lanes, FMA = 2) over all step launches of one mgs_qr call
# (profiles/mgs_step_qd_1024x1024.md).
QD1024_FLOPS = 9.632e11


def qd_large(torch, api, n=1024, reps=2):
    """Plain qd MGS on [A b] + back substitution at n = 1024 (random square
    A, every limb level U[-1,1]): time per solve and, when the instruction
    counts are known, the FP64 rate of the factorisation."""
    from paper_1210_0800_amd import inputs

    dev = torch.device("cuda:0")
    p = inputs.random_problem(4, n, n, seed=7, config=85)
    A, b = torch.from_numpy(p["A"]).to(dev), torch.from_numpy(p["b"]).to(dev)
    Q = torch.empty_like(A)
    R = torch.empty((4, 2, n, n), dtype=torch.float64, device=dev)
    y = torch.empty((4, 2, n), dtype=torch.float64, device=dev)
    x = torch.empty_like(y)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    info2 = torch.empty(1, dtype=torch.int32, device=dev)
    work = api.workspace(n, n, 4, 0, dev)
    stream = torch.cuda.current_stream(dev)
    api.mgs_qr(A, b, Q=Q, R=R, y=y, info=info, work=work)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tq = tb = 0.0
    for _ in range(reps):
        ev[0].record(stream)
        api.mgs_qr(A, b, Q=Q, R=R, y=y, info=info, work=work)
        ev[1].record(stream)
        api.ls_backsolve(R, y, x=x, info=info2)
        ev[2].record(stream)
        torch.cuda.synchronize()
        tq += ev[0].elapsed_time(ev[1]) / reps
        tb += ev[1].elapsed_time(ev[2]) / reps
    out = {"mgs_qr_ms": tq, "backsolve_ms": tb, "solves_per_s": 1e3 / (tq + tb), "info": int(info.item())}
    if QD1024_FLOPS is not None and n == 1024:
        achieved = QD1024_FLOPS / (tq * 1e-3) / 1e12
        out.update(flops_counted=QD1024_FLOPS, achieved_tflops=achieved, frac_fp64_peak=achieved / FP64_PEAK_TFLOPS)
    print("bench: qd %dx%d plain: factorisation %.1f ms, back substitution %.2f ms" % (n, n, tq, tb),
          file=sys.stderr, flush=True)
    return out


def copy_probe(nbytes):
    import torch

    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("bench: copied %d bytes 3 times" % nbytes, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--systems", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-form", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0)
    ap.add_argument("--only-precision-form", action="store_true")
    ap.add_argument("--only-context", action="store_true")
    ap.add_argument("--only-batched", action="store_true")
    ap.add_argument("--only-qd-large", action="store_true")
    ap.add_argument("--only-newton", action="store_true")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.only_context:
        import torch

        from paper_1210_0800_amd import api

        print(json.dumps({"paper_context": paper_context(torch, api), "workloads": workloads(torch, api)}),
              flush=True)
        return
    if args.only_qd_large:
        import torch

        from paper_1210_0800_amd import api

        print(json.dumps({"qd_1024x1024": qd_large(torch, api)}), flush=True)
        return
    if args.only_newton:
        import torch

        from paper_1210_0800_amd import api

        print(json.dumps({"newton": newton_context(torch, api)}), flush=True)
        return
    if args.only_batched:
        import torch

        from paper_1210_0800_amd import api

        print(json.dumps({"batched": batched(torch, api)}), flush=True)
        return
    if args.only_precision_form:
        import torch

        from paper_1210_0800_amd import api

        print(json.dumps({"precision_form": precision_form(torch, api)}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    m = n = 1024
    t_gen = time.perf_counter()
    workers = min(16, len(os.sched_getaffinity(0)))
    host = make_inputs(args.systems, workers)
    t_gen = time.perf_counter() - t_gen
    print("bench: generated %d systems in %.1f s" % (args.systems, t_gen), file=sys.stderr, flush=True)

    import torch

    from paper_1210_0800_amd import api

    dev = torch.device("cuda:0")
    A = [torch.from_numpy(a).to(dev) for a, _ in host]
    B = [torch.from_numpy(b).to(dev) for _, b in host]
    Q = torch.empty_like(A[0])
    R = torch.empty((2, 2, n, n), dtype=torch.float64, device=dev)
    y = torch.empty((2, 2, n), dtype=torch.float64, device=dev)
    rho = torch.empty(2, dtype=torch.float64, device=dev)
    x = torch.empty((2, 2, n), dtype=torch.float64, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    info2 = torch.empty(1, dtype=torch.int32, device=dev)
    work = api.workspace(m, n, 2, 0, dev)
    stream = torch.cuda.current_stream(dev)

    def solve(i, ev=None):
        if ev is not None:
            ev[0].record(stream)
        api.mgs_qr(A[i], B[i], Q=Q, R=R, y=y, rho=rho, info=info, work=work)
        if ev is not None:
            ev[1].record(stream)
        api.ls_backsolve(R, y, x=x, info=info2)
        if ev is not None:
            ev[2].record(stream)

    for _ in range(args.warmup):
        for i in range(args.systems):
            solve(i)
    torch.cuda.synchronize()
    assert int(info.item()) == 0 and int(info2.item()) == 0

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)]
              for _ in range(args.steps * args.systems)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        for i in range(args.systems):
            solve(i, events[s * args.systems + i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print("bench: timed %d steps in %.3f s" % (args.steps, elapsed), file=sys.stderr, flush=True)

    t_qr = np.mean([e[0].elapsed_time(e[1]) for e in events]) * 1e-3
    t_bs = np.mean([e[1].elapsed_time(e[2]) for e in events]) * 1e-3
    f_qr = mgs_flops(m, n, n + 1)
    achieved = f_qr / t_qr / 1e12
    solves = args.steps * args.systems
    out = {
        "metric": METRIC,
        "value": solves / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "dd (2 x f64)",
        "data": "synthetic",
        "config": {
            "workload": "complex double-double MGS least squares (MGS on [A b] + back substitution), "
                        "A 1024x1024 Jacobian-like (N(0,1) entries, columns scaled by 10^U[-12,12]), "
                        "64 systems solved back to back per step",
            "m": m, "n": n, "systems_per_step": args.systems, "prec": "dd",
            "ms_per_solve": elapsed / solves * 1e3,
            "ms_mgs_qr": t_qr * 1e3, "ms_backsolve": t_bs * 1e3,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "mgs_resident_kernel (one cooperative launch per factorisation)",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": traffic_bytes(),
            "flops_per_solve": f_qr,
            "algorithmic_bytes": 16 * 2 * (m * n + m + m * n + n * n + n),
        },
    }
    if not args.no_precision_form:
        out["precision_form"] = precision_form(torch, api)
        out["paper_context"] = paper_context(torch, api)
        out["workloads"] = workloads(torch, api)
        out["batched"] = batched(torch, api)
        out["qd_1024x1024"] = qd_large(torch, api)
        out["newton"] = newton_context(torch, api)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(host[:8])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
