"""ctypes loader for libmstrsm.so (the HIP library). No fallback: if the
library is missing or fails to load, every call raises."""
from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmstrsm.so")

_lock = threading.Lock()
_lib = None

MST_OK, MST_EARG, MST_EHIP, MST_ENOMEM, MST_EUNSUPPORTED = 0, -1, -2, -3, -4
SCRATCH_LIMIT = 16 << 20   # MST_SCRATCH_LIMIT: bytes of mstrsm_safe_noalloc's static scratch

# every symbol include/mstrsm.h declares
EXPORTS = ["mstrsm", "mstrsm_safe", "mstrsm_safe_noalloc", "mstrsm_adjoint", "mst_grad_u", "mst_grad_shift",
           "mst_residual", "mst_triang_eig", "mst_lanczos_sigma_min", "mst_lanczos_restart_sigma_min",
           "mstrsm_gen",
           "mstrsm_safe_gen", "mst_gen_triang_eig", "mst_eig_schur", "mst_gen_eig_schur", "mstrsm_op",
           "mstrsm_real", "mstrsm_real_op",
           "mst_status_string",
           "mst_last_bad_arg", "mst_last_error", "mst_version", "mst_profile_start",
           "mst_profile_stop"]

PROF_KINDS = ["gemm_f64", "gemm_f32", "diag", "resid", "aux"]


class MstOpts(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int), ("outer_nb", ctypes.c_int), ("precision", ctypes.c_int),
                ("max_sweeps", ctypes.c_int), ("omega_log2", ctypes.c_int),
                ("force_phase2", ctypes.c_int), ("fuse_blocks", ctypes.c_int),
                ("gemm_staged", ctypes.c_int), ("overlap", ctypes.c_int),
                ("gemm_split", ctypes.c_int), ("refine_tol", ctypes.c_double),
                ("refine_report", ctypes.c_void_p)]


class MstError(RuntimeError):
    def __init__(self, fn: str, code: int, detail: str):
        super().__init__("%s failed with %d: %s" % (fn, code, detail))
        self.code = code


def load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libmstrsm.so is not built (run `python -m paper_1607_01477_amd.build`)")
            lib = ctypes.CDLL(LIB_PATH)
            P, I = ctypes.c_void_p, ctypes.c_int
            OP = ctypes.POINTER(MstOpts)
            sig = {
                "mstrsm": [I, I, P, I, P, P, I, OP, P],
                "mstrsm_safe": [I, I, P, I, P, P, I, P, P, P, OP, P],
                "mstrsm_safe_noalloc": [I, I, P, I, P, P, I, P, P, P, OP, P],
                "mstrsm_adjoint": [I, I, P, I, P, P, I, OP, P],
                "mst_grad_u": [I, I, P, I, P, I, P, I, P],
                "mst_grad_shift": [I, I, P, I, P, I, P, P],
                "mst_residual": [I, I, P, I, P, P, I, P, I, P, I, P],
                "mst_triang_eig": [I, P, I, P, I, P, P, OP, P],
                "mst_lanczos_sigma_min": [I, I, P, I, P, P, I, I, P, P, P, P, OP, P],
                "mst_lanczos_restart_sigma_min": [I, I, P, I, P, P, I, I, I, I, ctypes.c_double, P, P, P,
                                                  P, OP, P],
                "mstrsm_gen": [I, I, P, I, P, I, P, P, I, OP, P],
                "mstrsm_safe_gen": [I, I, P, I, P, I, P, P, I, P, P, P, OP, P],
                "mst_gen_triang_eig": [I, P, I, P, I, P, I, P, P, OP, P],
                "mst_eig_schur": [I, P, I, P, I, P, I, P, P, OP, P],
                "mst_gen_eig_schur": [I, P, I, P, I, P, I, P, I, P, P, OP, P],
                "mstrsm_op": [I, I, I, I, I, P, I, P, P, I, OP, P],
                "mstrsm_real": [I, I, P, I, P, P, I, OP, P],
                "mstrsm_real_op": [I, I, I, I, I, P, I, P, P, I, OP, P],
            }
            for name, args in sig.items():
                f = getattr(lib, name)
                f.argtypes = args
                f.restype = I
            lib.mst_profile_start.restype = I
            lib.mst_profile_stop.argtypes = [P, P, P]
            lib.mst_profile_stop.restype = I
            lib.mst_status_string.argtypes = [I]
            lib.mst_status_string.restype = ctypes.c_char_p
            lib.mst_last_bad_arg.restype = I
            lib.mst_last_error.restype = ctypes.c_char_p
            lib.mst_version.restype = ctypes.c_char_p
            _lib = lib
    return _lib


def check(fn: str, rc: int) -> None:
    if rc == MST_OK:
        return
    lib = load()
    detail = lib.mst_status_string(rc).decode()
    if rc == MST_EARG:
        detail += " (argument %d)" % lib.mst_last_bad_arg()
    elif rc in (MST_EHIP, MST_ENOMEM, MST_EUNSUPPORTED):
        detail += " (%s)" % lib.mst_last_error().decode()
    raise MstError(fn, rc, detail)
