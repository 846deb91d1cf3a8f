"""The oracle's C++ built with AddressSanitizer and UBSan, exercised on
every entry point in a child process (the ASan runtime preloaded): any
out-of-bounds access (the fixed expansion buffers included), leak-free
misuse or undefined behaviour aborts the child and fails the test."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np
import oracle
from paper_1210_0800_amd import inputs
for L in (1, 2, 4):
    p = inputs.random_problem(L, 40, 24, seed=L, config=70)
    o = oracle.mgs(p["A"], p["b"], nthreads=3)
    assert o["info"] == 0
    x, _ = oracle.backsolve(o["R"], o["y"])
    x2, _ = oracle.ls_solve(o["Q"], o["R"], p["b"])
    e = oracle.errors(p["A"], o["Q"], o["R"], nthreads=2)
    T = inputs.table2_matrix(inputs.rng(71, L, 0), 32, L, m=16, n=16)
    ot = oracle.mgs(T)
    eb = oracle.emax_batch(np.stack([T, T]), np.stack([ot["Q"], ot["Q"]]), np.stack([ot["R"], ot["R"]]))
    a = inputs.random_limbs(inputs.rng(72, L, 0), (64,), L)
    for op in ("add", "sub", "mul", "div", "sqrt"):
        oracle.arith(L, op, np.abs(a) if op == "sqrt" else a, a[::-1].copy())
    if L > 1:
        g = inputs.random_complex(inputs.rng(73, L, 3), (24,), L)
        oracle.adjoint(p["A"], p["b"], g, nthreads=2)
        d = inputs.config4(48, cond=1e4)
        A = np.zeros((L, 2, 48, 48)); A[0] = d["A64"][0]
        r = oracle.refine(A, d["b4"][:L].copy(), block=16, nthreads=2)
        assert r["info"] == 0
    Z = p["A"].copy(); Z[:, :, 3] = 0.0
    assert oracle.mgs(Z)["info"] == 4
print("sanitized oracle: all entry points ran clean")
"""


@pytest.mark.slow
def test_oracle_under_asan_and_ubsan(tmp_path):
    so = oracle.build(out=str(tmp_path / "liborc_mgs_asan.so"), sanitize=True)
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["g++", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    env = dict(os.environ)
    env.update(ORC_MGS_LIB=so, LD_PRELOAD=asan + ":" + ubsan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "ran clean" in r.stdout
