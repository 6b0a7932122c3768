"""ctypes declarations of libcqr.so and libcqr_synth.so (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBDIR = os.path.join(_HERE, "lib")
LIB_PATH = os.path.join(LIBDIR, "libcqr.so")
SYNTH_PATH = os.path.join(LIBDIR, "libcqr_synth.so")

i64, i32, vp, dbl, u64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double, ctypes.c_uint64
szp = ctypes.POINTER(ctypes.c_size_t)
i32p = ctypes.POINTER(ctypes.c_int32)
i64p = ctypes.POINTER(ctypes.c_int64)
dblp = ctypes.POINTER(ctypes.c_double)

# name -> (argtypes, restype); the same names and order as include/cqr.h.
CQR_SIGNATURES = {
    "cqr_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "cqr_version": ([], ctypes.c_char_p),
    "cqr_workspace_size": ([i64, i64, i64, szp], ctypes.c_int),
    "cqr_factor": ([i64, i64, i64, vp, i64, vp, i64, vp, ctypes.c_size_t, vp, vp, vp], ctypes.c_int),
    "cqr_orth": ([i64, i64, vp, i64, vp, i64, vp, ctypes.c_size_t, vp, vp], ctypes.c_int),
    "cqr_orth_against": ([i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, ctypes.c_size_t, vp, vp],
                         ctypes.c_int),
    "cqr_set_wait_limit_us": ([i64], ctypes.c_int),
    "cqr_set_forced_breakdown": ([i64], ctypes.c_int),
    "cqr_solve_workspace_size": ([i64, szp], ctypes.c_int),
    "cqr_solve": ([i64, vp, i64, vp, i64, vp, vp, ctypes.c_size_t, vp, vp], ctypes.c_int),
    "cqr_solve_noalloc": ([i64, vp, i64, vp, i64, vp, vp, vp], ctypes.c_int),
    "cqr_workspace_size_mixed": ([i64, i64, i64, ctypes.c_int, szp], ctypes.c_int),
    "cqr_set_mixed_layout": ([ctypes.c_int], ctypes.c_int),
    "cqr_factor_mixed": ([i64, i64, i64, ctypes.c_int, vp, i64, vp, i64, vp, i64, vp, ctypes.c_size_t, vp, vp, vp],
                         ctypes.c_int),
    "cqr_solve_ir_workspace_size": ([i64, szp], ctypes.c_int),
    "cqr_solve_ir": ([i64, vp, i64, vp, i64, vp, i64, vp, vp, ctypes.c_int32, dbl, i32p, dblp, vp, ctypes.c_size_t, vp],
                     ctypes.c_int),
    "cqr_batched_workspace_size": ([i64, szp], ctypes.c_int),
    "cqr_batched_factor_solve": ([i64, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp],
                                 ctypes.c_int),
    "cqr_batched_solve_backward": ([i64, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
    "cqr_batched_instance": ([ctypes.c_int32, i32p, i32p, i32p, i32p], ctypes.c_int),
    "cqr_batched_plan_get": ([ctypes.c_int, i32p, i32p, i32p], ctypes.c_int),
    "cqr_batched_plan_set": ([ctypes.c_int, ctypes.c_int32, i32p, i32p], ctypes.c_int),
    "cqr_svd_workspace_size": ([ctypes.c_int, i64, i64, i64, i64, szp], ctypes.c_int),
    "cqr_lancsvd": ([i64, i64, vp, i64, i64, i64, ctypes.c_int, vp, i64, vp, i64, vp, vp, i64, vp, vp, ctypes.c_size_t,
                     vp], ctypes.c_int),
    "cqr_randsvd": ([i64, i64, vp, i64, i64, i64, ctypes.c_int, vp, i64, vp, i64, vp, vp, i64, vp, vp, ctypes.c_size_t,
                     vp], ctypes.c_int),
    "cqr_lancsvd_csr": ([i64, i64, i64, vp, vp, vp, vp, vp, vp, i64, i64, ctypes.c_int, vp, i64, vp, i64, vp, vp, i64,
                         vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
    "cqr_randsvd_csr": ([i64, i64, i64, vp, vp, vp, vp, vp, vp, i64, i64, ctypes.c_int, vp, i64, vp, i64, vp, vp, i64,
                         vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
    "cqr_small_svd_workspace_size": ([i64, szp], ctypes.c_int),
    "cqr_small_svd": ([i64, vp, i64, vp, i64, vp, vp, i64, vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
    "cqr_gemm_workspace_size": ([szp], ctypes.c_int),
    "cqr_gemm": ([ctypes.c_int, i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, vp, ctypes.c_size_t, vp],
                 ctypes.c_int),
    "cqr_svd_residuals": ([i64, i64, vp, i64, i64, vp, i64, vp, vp, i64, vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
    "cqr_spmm_workspace_size": ([i64, i64, szp], ctypes.c_int),
    "cqr_spmm": ([ctypes.c_int, i64, i64, i64, vp, vp, vp, i64, vp, i64, vp, i64, vp, ctypes.c_size_t, vp],
                 ctypes.c_int),
    "cqr_csr_transpose_workspace_size": ([i64, szp], ctypes.c_int),
    "cqr_csr_transpose": ([i64, i64, i64, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
    "cqr_prof_enable": ([ctypes.c_int], ctypes.c_int),
    "cqr_prof_reset": ([], ctypes.c_int),
    "cqr_prof_query": ([ctypes.c_char_p, i64p, dblp, dblp, dblp], ctypes.c_int),
    "cqr_prof_name": ([ctypes.c_int], ctypes.c_char_p),
}

SYNTH_SIGNATURES = {
    "cqr_synth_uniform": ([i64, i64, vp, i64, u64, dbl, dbl, vp], ctypes.c_int),
}

_libs: dict = {}


def _open(path: str, sigs: dict):
    if path not in _libs:
        if not os.path.exists(path):
            raise RuntimeError(
                "%s is not built: run `python -c \"import __graft_entry__ as g; g.build()\"` "
                "(there is no fallback implementation)" % path)
        lib = ctypes.CDLL(path)
        for name, (args, res) in sigs.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _libs[path] = lib
    return _libs[path]


def lib():
    return _open(LIB_PATH, CQR_SIGNATURES)


def synth_lib():
    return _open(SYNTH_PATH, SYNTH_SIGNATURES)


class CqrError(RuntimeError):
    pass


def check(code: int, what: str) -> None:
    if code != 0:
        msg = lib().cqr_status_string(code).decode()
        raise CqrError("%s failed with status %d: %s" % (what, code, msg))
