"""Truncated SVD (RandSVD, Algorithm 1; LancSVD, Algorithm 2) on the library's
kernels: argument marshalling into ``libcqr.so`` only.  Matrices are
column-major float64 device tensors (``colmajor``); a sparse A is a ``Csr``
(CSR arrays of A and of its transpose on the device).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _native, colmajor

LANCZOS = 0
RANDOMIZED = 1
SPARSE = 2


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ld(t: torch.Tensor) -> int:
    rows, cols = t.shape
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("expected a float64 GPU tensor")
    if rows > 1 and t.stride(0) != 1:
        raise ValueError("expected a column-major tensor (stride(0) == 1)")
    return max(t.stride(1) if cols > 1 else rows, rows, 1)


def workspace_size(method: int, m: int, n: int, r: int, b: int) -> int:
    nb = ctypes.c_size_t(0)
    _native.check(_native.lib().cqr_svd_workspace_size(method, m, n, r, b, ctypes.byref(nb)), "cqr_svd_workspace_size")
    return int(nb.value)


class Csr:
    """A sparse m x n matrix on the device: CSR of A and CSR of A^T (built by
    the library's transpose kernel)."""

    def __init__(self, m: int, n: int, rowptr, col, val, device="cuda"):
        self.m, self.n = int(m), int(n)
        self.rowptr = torch.as_tensor(np.asarray(rowptr, dtype=np.int32)).to(device)
        self.col = torch.as_tensor(np.asarray(col, dtype=np.int32)).to(device)
        self.val = torch.as_tensor(np.asarray(val, dtype=np.float64)).to(device)
        self.nnz = int(self.col.numel())
        self.trowptr = torch.empty(self.n + 1, dtype=torch.int32, device=device)
        self.tcol = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=device)
        self.tval = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=device)
        nb = ctypes.c_size_t(0)
        lib = _native.lib()
        _native.check(lib.cqr_csr_transpose_workspace_size(self.n, ctypes.byref(nb)), "cqr_csr_transpose_workspace_size")
        work = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=device)
        rc = lib.cqr_csr_transpose(self.m, self.n, self.nnz, _ptr(self.rowptr), _ptr(self.col), _ptr(self.val),
                                   _ptr(self.trowptr), _ptr(self.tcol), _ptr(self.tval), _ptr(work), work.numel(),
                                   _stream())
        _native.check(rc, "cqr_csr_transpose")
        self._work = work  # kept alive until the stream has used it

    def spmm(self, X: torch.Tensor, trans: bool = False, C: torch.Tensor | None = None) -> torch.Tensor:
        """C = A X (X n x w) or C = A^T X (X m x w)."""
        rows, inner = (self.n, self.m) if trans else (self.m, self.n)
        w = X.shape[1]
        if X.shape[0] != inner:
            raise ValueError("X has %d rows, expected %d" % (X.shape[0], inner))
        if C is None:
            C = colmajor(rows, w, device=X.device)
        nb = ctypes.c_size_t(0)
        lib = _native.lib()
        _native.check(lib.cqr_spmm_workspace_size(self.m, self.n, ctypes.byref(nb)), "cqr_spmm_workspace_size")
        work = torch.empty(nb.value, dtype=torch.uint8, device=X.device)
        if trans:
            ptrs = (self.trowptr, self.tcol, self.tval)
        else:
            ptrs = (self.rowptr, self.col, self.val)
        rc = lib.cqr_spmm(1 if trans else 0, self.m, self.n, self.nnz, _ptr(ptrs[0]), _ptr(ptrs[1]), _ptr(ptrs[2]), w,
                          _ptr(X), _ld(X), _ptr(C), _ld(C), _ptr(work), work.numel(), _stream())
        _native.check(rc, "cqr_spmm")
        return C


def _outputs(m, n, r, device):
    return colmajor(m, r, device=device), torch.empty(r, dtype=torch.float64, device=device), colmajor(n, r, device=device)


def lancsvd(A, r: int, b: int, p: int, Q1: torch.Tensor, work: torch.Tensor | None = None, sync: bool = True):
    """LancSVD of A (dense column-major tensor or Csr) from the m x b start
    block Q1.  Returns (U, sigma, V, info): info the number of
    orthogonalisations that took the CGS2 fallback (int with sync=True, else
    an int32 device tensor)."""
    sparse = isinstance(A, Csr)
    m, n = (A.m, A.n) if sparse else A.shape
    dev = Q1.device
    U, s, V = _outputs(m, n, r, dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    need = workspace_size(LANCZOS | (SPARSE if sparse else 0), m, n, r, b)
    if work is None or work.numel() < need:
        work = torch.empty(need, dtype=torch.uint8, device=dev)
    lib = _native.lib()
    if sparse:
        rc = lib.cqr_lancsvd_csr(m, n, A.nnz, _ptr(A.rowptr), _ptr(A.col), _ptr(A.val), _ptr(A.trowptr), _ptr(A.tcol),
                                 _ptr(A.tval), r, b, p, _ptr(Q1), _ld(Q1), _ptr(U), _ld(U), _ptr(s), _ptr(V), _ld(V),
                                 _ptr(info), _ptr(work), work.numel(), _stream())
        _native.check(rc, "cqr_lancsvd_csr")
    else:
        rc = lib.cqr_lancsvd(m, n, _ptr(A), _ld(A), r, b, p, _ptr(Q1), _ld(Q1), _ptr(U), _ld(U), _ptr(s), _ptr(V),
                             _ld(V), _ptr(info), _ptr(work), work.numel(), _stream())
        _native.check(rc, "cqr_lancsvd")
    return U, s, V, (int(info[0].item()) if sync else info)


def randsvd(A, r: int, b: int, p: int, Q0: torch.Tensor, work: torch.Tensor | None = None, sync: bool = True):
    """RandSVD of A (dense column-major tensor or Csr) from the n x r start
    block Q0.  Returns (U, sigma, V, info) as lancsvd."""
    sparse = isinstance(A, Csr)
    m, n = (A.m, A.n) if sparse else A.shape
    dev = Q0.device
    U, s, V = _outputs(m, n, r, dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    need = workspace_size(RANDOMIZED | (SPARSE if sparse else 0), m, n, r, b)
    if work is None or work.numel() < need:
        work = torch.empty(need, dtype=torch.uint8, device=dev)
    lib = _native.lib()
    if sparse:
        rc = lib.cqr_randsvd_csr(m, n, A.nnz, _ptr(A.rowptr), _ptr(A.col), _ptr(A.val), _ptr(A.trowptr), _ptr(A.tcol),
                                 _ptr(A.tval), r, b, p, _ptr(Q0), _ld(Q0), _ptr(U), _ld(U), _ptr(s), _ptr(V), _ld(V),
                                 _ptr(info), _ptr(work), work.numel(), _stream())
        _native.check(rc, "cqr_randsvd_csr")
    else:
        rc = lib.cqr_randsvd(m, n, _ptr(A), _ld(A), r, b, p, _ptr(Q0), _ld(Q0), _ptr(U), _ld(U), _ptr(s), _ptr(V),
                             _ld(V), _ptr(info), _ptr(work), work.numel(), _stream())
        _native.check(rc, "cqr_randsvd")
    return U, s, V, (int(info[0].item()) if sync else info)


def small_svd(B: torch.Tensor):
    """One-sided Jacobi SVD of a small square B (r <= 256).  Returns (U, sigma, V, sweeps)."""
    r = B.shape[0]
    U, s, V = _outputs(r, r, r, B.device)
    sw = torch.zeros(1, dtype=torch.int32, device=B.device)
    nb = ctypes.c_size_t(0)
    lib = _native.lib()
    _native.check(lib.cqr_small_svd_workspace_size(r, ctypes.byref(nb)), "cqr_small_svd_workspace_size")
    work = torch.empty(nb.value, dtype=torch.uint8, device=B.device)
    rc = lib.cqr_small_svd(r, _ptr(B), _ld(B), _ptr(U), _ld(U), _ptr(s), _ptr(V), _ld(V), _ptr(sw), _ptr(work),
                           work.numel(), _stream())
    _native.check(rc, "cqr_small_svd")
    return U, s, V, int(sw[0].item())


def gemm(A: torch.Tensor, B: torch.Tensor, trans_a: bool = False, C: torch.Tensor | None = None,
         alpha: float = 1.0, beta: float = 0.0, work: torch.Tensor | None = None) -> torch.Tensor:
    """C = alpha op(A) B + beta C with op(A) = A^T (trans_a) or A, on the library's FP64 MFMA kernels."""
    K, N = B.shape
    M = A.shape[1] if trans_a else A.shape[0]
    if C is None:
        C = colmajor(M, N, device=B.device)
    if work is None:
        nb = ctypes.c_size_t(0)
        _native.check(_native.lib().cqr_gemm_workspace_size(ctypes.byref(nb)), "cqr_gemm_workspace_size")
        work = torch.empty(nb.value, dtype=torch.uint8, device=B.device)
    rc = _native.lib().cqr_gemm(1 if trans_a else 0, M, N, K, float(alpha), _ptr(A), _ld(A), _ptr(B), _ld(B),
                                float(beta), _ptr(C), _ld(C), _ptr(work), work.numel(), _stream())
    _native.check(rc, "cqr_gemm")
    return C


def residuals(A: torch.Tensor, U: torch.Tensor, s: torch.Tensor, V: torch.Tensor, count: int) -> torch.Tensor:
    """||A v_j - sigma_j u_j||_2 / sigma_j for the first ``count`` triplets (dense A)."""
    m, n = A.shape
    res = torch.empty(count, dtype=torch.float64, device=A.device)
    work = torch.empty(m * count * 8, dtype=torch.uint8, device=A.device)
    rc = _native.lib().cqr_svd_residuals(m, n, _ptr(A), _ld(A), count, _ptr(U), _ld(U), _ptr(s), _ptr(V), _ld(V),
                                         _ptr(res), _ptr(work), work.numel(), _stream())
    _native.check(rc, "cqr_svd_residuals")
    return res
