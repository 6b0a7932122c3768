"""CPU FP64 oracle for the paper's block Gram-Schmidt QR (arXiv 2403.06218, Sec. 3).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the HIP library and its
binding never do, and the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, IEEE double); this module only
marshals numpy arrays through ctypes.  Functions:

* ``householder_qr(Y)``      O-def: the unique thin QR with diag(R) > 0 by
                              textbook Householder reflections.
* ``cgs_qr(Y, b, ...)``       O-alg: Algorithm 3 (CGS-QR) with Algorithm 4
                              (CholeskyQR2) on block 1, Algorithm 5 (CGS-CQR2) on
                              the later blocks, and the CGS2 breakdown fallback.
* ``cholqr2(Q)``             Algorithm 4 alone.
* ``cgs_cqr2(Q, P)``         Algorithm 5 alone.
* ``chol(W)``, ``trsm_rlt``  the POTRF / TRSM building blocks of Table 1.
* ``qr_solve``, ``qr_solve_grad``  x = R^{-1} Q^T b and its adjoint.
* ``orth_against_fb``        Algorithm 5 (or 4) with the CGS2 fallback.
* ``check_invariants``       the loop invariants I1-I4 of Algorithm 3.

``oracle.svd`` holds the truncated-SVD drivers (RandSVD, LancSVD) built on these.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

VARIANT_PRINTED_R = 1   # Alg. 4 S7 / Alg. 5 S11 as printed: R = L^T Lbar^T
VARIANT_PRINTED_H = 2   # Alg. 5 S12 as printed: H = H + Hbar


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, i32, dp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        sig = {
            "ora_chol": ([i64, dp, i64], i32),
            "ora_trsm_rlt": ([i64, i64, dp, i64, dp, i64], None),
            "ora_cholqr2": ([i64, i64, dp, i64, dp, i64, i32], i32),
            "ora_cgs_cqr2": ([i64, i64, i64, dp, i64, dp, i64, dp, i64, dp, i64, i32], i32),
            "ora_cgs_qr": ([i64, i64, i64, dp, i64, dp, i64, i32, dp, dp, dp], i32),
            "ora_householder_qr": ([i64, i64, dp, i64, dp, i64, dp, i64], i32),
            "ora_qr_solve": ([i64, dp, i64, dp, i64, dp, dp], i32),
            "ora_qr_solve_grad": ([i64, dp, i64, dp, i64, dp, dp, dp, i64, dp], i32),
            "ora_check_invariants": ([i64, i64, i64, dp, i64, dp, i64, dp, i64, dp], None),
            "ora_orth_against_fb": ([i64, i64, i64, dp, i64, dp, i64, dp, i64], i32),
            "ora_num_threads": ([], i32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    """Column-major float64 copy (leading dimension = number of rows)."""
    return np.array(a, dtype=np.float64, order="F", copy=True)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().ora_num_threads())


def chol(W):
    """Lower Cholesky factor of W (POTRF).  Returns (L, rc); rc = j+1 on a breakdown at pivot j."""
    L = _f64(W)
    n = L.shape[0]
    rc = _load().ora_chol(n, _p(L), max(n, 1))
    return L, int(rc)


def trsm_rlt(Q, L):
    """Q L^{-T} by row-wise forward substitution (TRSM, right, lower, transposed)."""
    Q = _f64(Q)
    L = _f64(L)
    q, b = Q.shape
    _load().ora_trsm_rlt(q, b, _p(Q), max(q, 1), _p(L), max(b, 1))
    return Q


def cholqr2(Q, variant: int = 0):
    """Algorithm 4.  Returns (Q, R, rc)."""
    Q = _f64(Q)
    q, b = Q.shape
    R = np.zeros((b, b), order="F")
    rc = _load().ora_cholqr2(q, b, _p(Q), max(q, 1), _p(R), max(b, 1), variant)
    return Q, R, int(rc)


def cgs_cqr2(Q, P, variant: int = 0):
    """Algorithm 5.  Returns (Q, H, R, rc)."""
    Q = _f64(Q)
    P = _f64(P)
    q, b = Q.shape
    s = P.shape[1]
    H = np.zeros((max(s, 1), b), order="F")
    R = np.zeros((b, b), order="F")
    rc = _load().ora_cgs_cqr2(q, b, s, _p(Q), max(q, 1), _p(P), max(q, 1), _p(H), max(s, 1), _p(R),
                              max(b, 1), variant)
    return Q, H[:s], R, int(rc)


def cgs_qr(Y, b: int, variant: int = 0, check_invariants: bool = False):
    """Algorithm 3 (CGS-QR).

    Returns a dict with Q, R, info (0 or first fallback block, 1-based),
    block_flags (bit 0 fallback, bit 1 exactly dependent column) and, when
    ``check_invariants`` is set, ``inv`` = worst [I1, I2, I3, I4] over all blocks.
    """
    Q = _f64(Y)
    q, r = Q.shape
    R = np.zeros((r, r), order="F")
    k = -(-r // b) if r > 0 else 0
    flags = np.zeros(max(k, 1), dtype=np.int32)
    info = np.zeros(1, dtype=np.int32)
    inv = np.zeros(4) if check_invariants else None
    rc = _load().ora_cgs_qr(q, r, b, _p(Q), max(q, 1), _p(R), max(r, 1), variant, _p(flags), _p(info),
                            _p(inv) if inv is not None else None)
    if rc != 0:
        raise ValueError("ora_cgs_qr: invalid argument %d" % (-rc))
    out = {"Q": Q, "R": R, "info": int(info[0]), "block_flags": flags[:k].copy()}
    if inv is not None:
        out["inv"] = inv
    return out


def orth_against_fb(Q, P=None):
    """Algorithm 5 (Algorithm 4 when P is None or empty) with the CGS2
    breakdown fallback.  Returns (Q, H, R, rc): rc 0, 1 (fallback) or 3
    (fallback with an exactly dependent column)."""
    Q = np.asarray(Q, dtype=np.float64)
    q, w = Q.shape
    s = 0 if P is None else P.shape[1]
    X = np.zeros((q, s + w), order="F")
    if s:
        X[:, :s] = P
    X[:, s:] = Q
    H = np.zeros((max(s, 1), w), order="F")
    R = np.zeros((w, w), order="F")
    rc = _load().ora_orth_against_fb(q, s, w, _p(X), max(q, 1), _p(H), max(s, 1), _p(R), max(w, 1))
    return np.asfortranarray(X[:, s:]), H[:s], R, int(rc)


def check_invariants(Y0, Q, R, J: int):
    """Loop invariants of Algorithm 3 with J finished columns: returns
    [I1, I2, I3, I4] = [||Q_J^T Q_J - I||_F / (q eps),
    ||Y_J - Q_J R_J||_F / (q eps ||Y_J||_F), 1 if R_J is not upper triangular
    with a non-negative diagonal, 1 if a column at or after J differs from Y0
    in any bit]."""
    Y0 = _f64(Y0)
    Q = _f64(Q)
    R = _f64(R)
    q, r = Q.shape
    out = np.zeros(4)
    _load().ora_check_invariants(q, r, J, _p(Y0), max(q, 1), _p(Q), max(q, 1), _p(R), max(r, 1), _p(out))
    return out


def householder_qr(Y):
    """O-def: thin QR with diag(R) >= 0 by Householder reflections.  Returns (Q, R)."""
    Y = _f64(Y)
    q, r = Y.shape
    Q = np.zeros((q, r), order="F")
    R = np.zeros((r, r), order="F")
    rc = _load().ora_householder_qr(q, r, _p(Y), max(q, 1), _p(Q), max(q, 1), _p(R), max(r, 1))
    if rc != 0:
        raise ValueError("ora_householder_qr: invalid argument %d" % (-rc))
    return Q, R


def qr_solve(Q, R, b):
    """x = R^{-1} (Q^T b).  Returns (x, rc)."""
    Q = _f64(Q)
    R = _f64(R)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = Q.shape[0]
    x = np.zeros(n)
    rc = _load().ora_qr_solve(n, _p(Q), max(n, 1), _p(R), max(n, 1), _p(b), _p(x))
    return x, int(rc)


def qr_solve_grad(Q, R, x, w):
    """Adjoint of x = (QR)^{-1} b for dL/dx = w.  Returns (dA, db, rc)."""
    Q = _f64(Q)
    R = _f64(R)
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = Q.shape[0]
    dA = np.zeros((n, n), order="F")
    db = np.zeros(n)
    rc = _load().ora_qr_solve_grad(n, _p(Q), max(n, 1), _p(R), max(n, 1), _p(x), _p(w), _p(dA), max(n, 1),
                                   _p(db))
    return dA, db, int(rc)
