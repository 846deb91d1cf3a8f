"""Host-side checks of the C ABI: the library loads, exports every function
declared in include/mgsqr.h, and rejects bad arguments before any launch.

No call here passes argument validation, so no kernel is ever launched.
"""
import ctypes
import os
import re

import pytest

from paper_1210_0800_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgsqr.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_entry_points():
    names = _declared()
    for f in _lib.EXPORTS:
        assert f in names, f
    assert set(names) == set(_lib.EXPORTS), names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert L.mgs_abi_version() == 1


def test_status_strings():
    L = _lib.lib()
    for st in range(0, -7, -1):
        s = L.mgs_status_string(st).decode()
        assert s and s != "unknown status"
    assert L.mgs_status_string(-99).decode() == "unknown status"


def test_workspace_sizes():
    # QR: working copy of b (rounded to 256 bytes) + 1 KiB of sync words,
    # + in dd with m <= 1024 the single launch's hand-off copy of the n
    # columns (2 L m n doubles)
    assert _lib.workspace_size(32, 32, 2, _lib.MGS_OP_QR) == 2 * 2 * 32 * 8 + 1024 + 2 * 2 * 32 * 32 * 8
    assert _lib.workspace_size(1025, 32, 2, _lib.MGS_OP_QR) == 2 * 2 * 1025 * 8 + 1024 + 256 - (2 * 2 * 1025 * 8) % 256
    assert _lib.workspace_size(320, 256, 4, _lib.MGS_OP_QR) == 2 * 4 * 320 * 8 + 1024
    assert _lib.workspace_size(100, 10, 2, _lib.MGS_OP_SOLVE) == 512
    with pytest.raises(_lib.MgsError):
        _lib.workspace_size(10, 11, 2, _lib.MGS_OP_QR)
    with pytest.raises(_lib.MgsError):
        _lib.workspace_size(10, 10, 3, _lib.MGS_OP_QR)
    with pytest.raises(_lib.MgsError):
        _lib.workspace_size(10, 10, 2, 7)
    with pytest.raises(_lib.MgsError):
        _lib.workspace_size(4097, 10, 2, _lib.MGS_OP_QR)
    with pytest.raises(_lib.MgsError):
        _lib.workspace_size(2049, 10, 4, _lib.MGS_OP_QR)


FAKE = 0x10000  # aligned, never dereferenced: every call below fails validation first
ODD = 0x10004 + 1


def _qr(m=8, n=4, prec=2, A=FAKE, lda=8, Q=FAKE + 4096, ldq=8, R=FAKE + 8192, ldr=4, b=None, y=None,
        rho=None, work=FAKE + 20480, wb=1 << 16, info=FAKE + 12288):
    return _lib.lib().mgs_qr(m, n, prec, A, lda, Q, ldq, R, ldr, b, y, rho, work, wb, info, None)


def test_mgs_qr_rejects_bad_arguments():
    assert _qr(prec=3) == -3
    assert _qr(prec=0) == -3
    assert _qr(prec=5) == -3
    assert _qr(m=3, n=4) == -1
    assert _qr(n=0) == -1
    assert _qr(lda=7) == -1
    assert _qr(ldq=7) == -1
    assert _qr(ldr=3) == -1
    assert _qr(m=4097, lda=4097, ldq=4097) == -1
    assert _qr(prec=4, m=2049, lda=2049, ldq=2049) == -1
    assert _qr(A=None) == -2
    assert _qr(A=ODD) == -2
    assert _qr(info=None) == -2
    assert _qr(Q=FAKE, A=FAKE, ldq=9, lda=8) in (-1, -2)
    # the workspace is always required; with b, y too
    assert _qr(work=None) == -2
    assert _qr(wb=8) == -4
    assert _qr(b=FAKE + 16384, y=None, work=FAKE + 20480, wb=1 << 16) == -2
    assert _qr(b=FAKE + 16384, y=FAKE + 24576, work=None, wb=1 << 16) == -2
    assert _qr(b=FAKE + 16384, y=FAKE + 24576, work=FAKE + 20480, wb=8) == -4


def test_ls_solve_and_backsolve_reject_bad_arguments():
    L = _lib.lib()
    assert L.ls_solve(8, 4, 3, FAKE, 8, FAKE, 4, FAKE, FAKE, FAKE, 4096, FAKE, None) == -3
    assert L.ls_solve(3, 4, 2, FAKE, 8, FAKE, 4, FAKE, FAKE, FAKE, 4096, FAKE, None) == -1
    assert L.ls_solve(8, 4, 2, FAKE, 8, FAKE, 4, None, FAKE, FAKE, 4096, FAKE, None) == -2
    assert L.ls_solve(8, 4, 2, FAKE, 8, FAKE, 4, FAKE, FAKE + 64, FAKE + 128, 8, FAKE, None) == -4
    assert L.ls_backsolve(4, 2, FAKE, 3, FAKE, FAKE + 64, FAKE, None) == -1
    assert L.ls_backsolve(0, 2, FAKE, 4, FAKE, FAKE + 64, FAKE, None) == -1
    assert L.ls_backsolve(4, 5, FAKE, 4, FAKE, FAKE + 64, FAKE, None) == -3
    assert L.ls_backsolve(4, 2, FAKE, 4, FAKE, FAKE, FAKE, None) == -2  # x aliases y
    assert L.ls_backsolve(4, 2, None, 4, FAKE, FAKE + 64, FAKE, None) == -2


def test_binding_refuses_cpu_tensors():
    import torch

    from paper_1210_0800_amd import api

    A = torch.zeros(2, 2, 3, 4, dtype=torch.float64)
    with pytest.raises(ValueError):
        api.mgs_qr(A)


def test_ls_adjoint_rejects_bad_arguments():
    L = _lib.lib()
    args = [8, 4, 2, FAKE, 8, FAKE + 64, FAKE + 128, 8, FAKE + 192, 4, FAKE + 256, FAKE + 320, FAKE + 384, 8,
            FAKE + 448, FAKE + 512, 1 << 20, FAKE + 576, None]
    def call(**kw):
        a = list(args)
        names = ["m", "n", "prec", "A", "lda", "b", "Q", "ldq", "R", "ldr", "x", "gx", "gA", "ldga", "gb", "work",
                 "wb", "info", "stream"]
        for k, v in kw.items():
            a[names.index(k)] = v
        return L.ls_adjoint(*a)
    assert call(prec=3) == -3
    assert call(m=3) == -1
    assert call(ldga=7) == -1
    assert call(gA=None) == -2
    assert call(gA=FAKE) == -2        # aliases A
    assert call(gb=FAKE + 64) == -2   # aliases b
    assert call(wb=16) == -4
    # w, z, r, then 2 x (one chunk) x 8 rows of 32-byte dd accumulators
    assert _lib.workspace_size(8, 4, 2, _lib.MGS_OP_ADJOINT) == 3 * 256 + 512


def test_mgs_qr64_rejects_bad_arguments():
    L = _lib.lib()
    names = ["m", "n", "A", "lda", "b", "Q", "ldq", "R", "ldr", "y", "block", "work", "wb", "info", "stream"]
    args = [8, 4, FAKE, 8, FAKE + 128, FAKE + 256, 8, FAKE + 512, 4, FAKE + 1024, 64, FAKE + 2048, 1 << 20,
            FAKE + 4096, None]

    def call(**kw):
        a = list(args)
        for k, v in kw.items():
            a[names.index(k)] = v
        return L.mgs_qr64(*a)
    assert call(block=32) == -3
    assert call(m=3) == -1
    assert call(m=4097, lda=4097, ldq=4097) == -1
    assert call(ldr=3) == -1
    assert call(A=None) == -2
    assert call(y=None) == -2          # b given, y required
    assert call(work=None) == -2
    assert call(wb=64) == -4
    # b == NULL: y may be NULL (fails later on the workspace, not the pointer)
    assert call(b=None, y=None, wb=64) == -4
    # Q64 (8 x 5) and R64 (4 x 5) complex FP64, each rounded up to 256 bytes,
    # then the panel single launch's sync words (1 KiB) and hand-off copy of
    # the panel (2 m min(n, 64) doubles)
    assert _lib.workspace_size(8, 4, 1, _lib.MGS_OP_QR64) == 768 + 512 + 1024 + 512
    # no single launch beyond 2048 rows
    assert _lib.workspace_size(2049, 4, 1, _lib.MGS_OP_QR64) == (2 * 2049 * 5 * 8 + 255) // 256 * 256 + 512
    with pytest.raises(_lib.MgsError):
        _lib.workspace_size(8, 4, 2, _lib.MGS_OP_QR64)


def test_prec1_workspaces_and_refusals():
    # complex double (prec 1): QR and SOLVE only; the adjoint and the
    # precision form stay dd / qd
    # b copy, sync words, and (m <= 2048, at most 32 MiB) the single
    # launch's hand-off copy of the n columns
    assert _lib.workspace_size(32, 32, 1, _lib.MGS_OP_QR) == 2 * 32 * 8 + 1024 + 2 * 32 * 32 * 8
    assert _lib.workspace_size(2048, 1024, 1, _lib.MGS_OP_QR) == 2 * 2048 * 8 + 1024 + 2 * 2048 * 1024 * 8
    assert _lib.workspace_size(2048, 1025, 1, _lib.MGS_OP_QR) == 2 * 2048 * 8 + 1024
    assert _lib.workspace_size(2049, 10, 1, _lib.MGS_OP_QR) == (2 * 2049 * 8 + 255) // 256 * 256 + 1024
    assert _lib.workspace_size(32, 32, 1, _lib.MGS_OP_SOLVE) == 512
    with pytest.raises(_lib.MgsError):
        _lib.workspace_size(32, 32, 1, _lib.MGS_OP_ADJOINT)
    with pytest.raises(_lib.MgsError):
        _lib.workspace_size(32, 32, 1, _lib.MGS_OP_REFINE)
    L = _lib.lib()
    assert L.mgs_refine_solve(8, 4, 1, FAKE, 8, FAKE, FAKE + 64, 64, 0.0, 4, None, None, FAKE, 1 << 20, FAKE,
                              None) == -3


def test_mgs_lstsq_batched_rejects_bad_arguments():
    L = _lib.lib()
    names = ["batch", "m", "n", "prec", "A", "lda", "b", "Q", "ldq", "R", "ldr", "y", "x", "rho", "info", "stream"]
    args = [4, 32, 32, 2, FAKE, 32, FAKE + 4096, FAKE + 8192, 32, FAKE + 12288, 32, None, FAKE + 16384, None,
            FAKE + 20480, None]

    def call(**kw):
        a = list(args)
        for k, v in kw.items():
            a[names.index(k)] = v
        return L.mgs_lstsq_batched(*a)
    assert call(prec=3) == -3
    assert call(batch=-1) == -1
    assert call(n=0) == -1
    assert call(m=31) == -1
    assert call(m=65, lda=65, ldq=65) == -1           # more rows than lanes of a wave
    assert call(m=64, n=64, lda=64, ldq=64, ldr=64) == -1   # 65 columns of [A b]
    assert call(lda=31) == -1
    assert call(ldr=31) == -1
    # qd: the q vectors of a system must fit in LDS (64 m n bytes)
    assert call(prec=4, m=64, n=40, lda=64, ldq=64, ldr=40) == -1
    assert call(A=None) == -2
    assert call(A=ODD) == -2
    assert call(info=None) == -2
    assert call(x=None) == -2                         # b given: y or x required
    assert call(y=FAKE + 16384) == -2                 # x aliases y
    assert call(Q=FAKE, ldq=33, m=32) in (-1, -2)


def test_newton_workspace_and_refusals():
    L = _lib.lib()
    nb = ctypes.c_size_t(0)
    # J, -f, R and the correction, each rounded up to 256 bytes
    assert L.mgs_newton_workspace_size(3, 32, 32, 2, ctypes.byref(nb)) == 0
    r256 = lambda v: (v + 255) // 256 * 256  # noqa: E731
    assert nb.value == r256(3 * 4 * 32 * 32 * 8) + r256(3 * 4 * 32 * 8) + r256(3 * 4 * 32 * 32 * 8) + r256(3 * 4 * 32 * 8)
    # more variables than equations, more than 64 equations, qd q vectors
    # beyond LDS, too many variables, unsupported precision
    for batch, neq, nvar, prec, st in ((1, 31, 32, 2, -1), (1, 65, 32, 2, -1), (1, 64, 63, 4, -1), (1, 64, 64, 2, -1),
                                       (70000, 32, 32, 2, -1), (1, 32, 32, 3, -3)):
        assert L.mgs_newton_workspace_size(batch, neq, nvar, prec, ctypes.byref(nb)) == st, (neq, nvar, prec)
    P = ctypes.c_void_p(64)  # aligned, never dereferenced: refused before any launch
    args = lambda batch, neq, nvar, nmon, nvpm, prec, iters: (  # noqa: E731
        batch, neq, nvar, nmon, nvpm, prec, P, P, P, P, iters, None, P, 1 << 30, P, None)
    assert L.mgs_newton_batched(*args(1, 32, 32, 65, 5, 2, 1)) == -1  # nmon > 64
    assert L.mgs_newton_batched(*args(1, 32, 32, 32, 9, 2, 1)) == -1  # nvpm > 8
    assert L.mgs_newton_batched(*args(1, 32, 32, 32, 5, 2, -1)) == -1
    assert L.mgs_newton_batched(*args(1, 32, 33, 32, 5, 2, 1)) == -1
    assert L.mgs_newton_batched(*args(0, 32, 32, 32, 5, 2, 1)) == 0  # nothing to do
    assert L.mgs_newton_batched(*args(1, 32, 32, 32, 5, 2, 0)) == 0
    a = list(args(1, 32, 32, 32, 5, 2, 1))
    a[13] = 16  # workspace too small
    assert L.mgs_newton_batched(*a) == -4
    a = list(args(1, 32, 32, 32, 5, 2, 1))
    a[6] = None  # vars
    assert L.mgs_newton_batched(*a) == -2
    a = list(args(1, 32, 32, 32, 5, 2, 1))
    a[9] = ctypes.c_void_p(68)  # x misaligned
    assert L.mgs_newton_batched(*a) == -2
    # evaluation: bad sizes and pointers
    ev = lambda batch, neq, nvar, nmon, nvpm, prec: (batch, neq, nvar, nmon, nvpm, prec, P, P, P, P, P, P, None)  # noqa: E731
    assert L.mgs_poly_eval(*ev(1, 32, 64, 32, 5, 2)) == -1
    assert L.mgs_poly_eval(*ev(1, 32, 32, 0, 5, 2)) == -1
    assert L.mgs_poly_eval(*ev(-1, 32, 32, 32, 5, 2)) == -1
    assert L.mgs_poly_eval(*ev(1, 32, 32, 32, 5, 5)) == -3
    assert L.mgs_poly_eval(*ev(0, 32, 32, 32, 5, 2)) == 0
    e = list(ev(1, 32, 32, 32, 5, 2))
    e[10] = None  # J
    assert L.mgs_poly_eval(*e) == -2
