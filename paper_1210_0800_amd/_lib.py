"""ctypes binding of libmgsqr.so (include/mgsqr.h): argument marshalling only.

Every computation runs in the HIP kernels of the library.  PyTorch supplies
device memory and the stream.  Importing this module on a machine where the
library was not built raises immediately: there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libmgsqr.so")

MGS_OK = 0
MGS_OP_QR = 0
MGS_OP_SOLVE = 1
MGS_OP_ADJOINT = 2
MGS_OP_REFINE = 3
MGS_OP_QR64 = 4
MGS_MAX_ROWS = {1: 4096, 2: 4096, 4: 2048}

EXPORTS = ("mgs_abi_version", "mgs_status_string", "mgs_workspace_size", "mgs_qr", "mgs_qr_schedule",
           "ls_solve", "ls_backsolve", "ls_adjoint", "mgs_refine_solve", "mgs_qr64", "mgs_lstsq_batched",
           "mgs_qr_noalloc", "mgs_poly_eval", "mgs_newton_workspace_size", "mgs_newton_batched", "mgs_set_jitter")
SCHEDULES = {"auto": 0, "panel": 1, "resident": 2, "small": 3}

_lib = None


class MgsError(RuntimeError):
    def __init__(self, fn, status):
        msg = lib().mgs_status_string(status).decode()
        super().__init__("%s failed with status %d: %s" % (fn, status, msg))
        self.status = status


def lib():
    """Load libmgsqr.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError("libmgsqr.so is not built (%s); run __graft_entry__.build()" % SO_PATH)
        L = ctypes.CDLL(SO_PATH)
        P, I, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
        L.mgs_abi_version.argtypes = []
        L.mgs_abi_version.restype = I
        L.mgs_status_string.argtypes = [I]
        L.mgs_status_string.restype = ctypes.c_char_p
        L.mgs_workspace_size.argtypes = [I, I, I, I, ctypes.POINTER(S)]
        L.mgs_workspace_size.restype = I
        L.mgs_qr.argtypes = [I, I, I, P, I, P, I, P, I, P, P, P, P, S, P, P]
        L.mgs_qr.restype = I
        L.mgs_qr_schedule.argtypes = [I, I, I, P, I, P, I, P, I, P, P, P, P, S, P, I, P]
        L.mgs_qr_schedule.restype = I
        L.ls_solve.argtypes = [I, I, I, P, I, P, I, P, P, P, S, P, P]
        L.ls_solve.restype = I
        L.ls_backsolve.argtypes = [I, I, P, I, P, P, P, P]
        L.ls_backsolve.restype = I
        L.ls_adjoint.argtypes = [I, I, I, P, I, P, P, I, P, I, P, P, P, I, P, P, S, P, P]
        L.ls_adjoint.restype = I
        L.mgs_refine_solve.argtypes = [I, I, I, P, I, P, P, I, ctypes.c_double, I, P, P, P, S, P, P]
        L.mgs_refine_solve.restype = I
        L.mgs_qr64.argtypes = [I, I, P, I, P, P, I, P, I, P, I, P, S, P, P]
        L.mgs_qr64.restype = I
        L.mgs_lstsq_batched.argtypes = [I, I, I, I, P, I, P, P, I, P, I, P, P, P, P, P]
        L.mgs_lstsq_batched.restype = I
        L.mgs_qr_noalloc.argtypes = [I, I, I, P, I, P, I, P, I, P, P, P, P, P]
        L.mgs_qr_noalloc.restype = I
        L.mgs_poly_eval.argtypes = [I, I, I, I, I, I, P, P, P, P, P, P, P]
        L.mgs_poly_eval.restype = I
        L.mgs_newton_workspace_size.argtypes = [I, I, I, I, ctypes.POINTER(S)]
        L.mgs_newton_workspace_size.restype = I
        L.mgs_newton_batched.argtypes = [I, I, I, I, I, I, P, P, P, P, I, P, P, S, P, P]
        L.mgs_newton_batched.restype = I
        L.mgs_set_jitter.argtypes = [ctypes.c_uint]
        L.mgs_set_jitter.restype = None
        _lib = L
    return _lib


def check(fn, status):
    if status != MGS_OK:
        raise MgsError(fn, status)


def workspace_size(m, n, prec, op):
    out = ctypes.c_size_t(0)
    check("mgs_workspace_size", lib().mgs_workspace_size(m, n, prec, op, ctypes.byref(out)))
    return out.value


def newton_workspace_size(batch, neq, nvar, prec):
    out = ctypes.c_size_t(0)
    check("mgs_newton_workspace_size", lib().mgs_newton_workspace_size(batch, neq, nvar, prec, ctypes.byref(out)))
    return out.value
