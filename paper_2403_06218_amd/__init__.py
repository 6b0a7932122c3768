"""MI355X-native block Gram-Schmidt QR (CGS-QR with CholeskyQR2 / CGS-CQR2) and solve.

The compute path is the HIP library ``lib/libcqr.so`` (C ABI declared in
``include/cqr.h``); this package only marshals torch device tensors into it:
pointers, sizes, leading dimensions, workspace and the current stream.  The
native library is loaded on first use and its absence is an error -- there is
no fallback implementation.

Matrices are column-major: a q x r matrix is a torch tensor of shape (q, r)
with strides (1, ld), ld >= q, e.g. ``colmajor(q, r)``.
"""
from __future__ import annotations

import ctypes

import torch

from . import _native
from ._native import CqrError

FLAG_FALLBACK = 1
FLAG_ZERO_COL = 2
PREC_BF16 = 1
PREC_FP8 = 2

__all__ = ["colmajor", "workspace_size", "qr", "qr_async", "orth", "orth_against", "solve", "solve_noalloc", "solve_workspace_size",
           "set_wait_limit_us", "set_forced_breakdown", "set_mixed_layout", "qr_mixed", "qr_mixed_async", "solve_ir",
           "synth_uniform",
           "prof_enable", "prof_reset", "prof_query", "prof_names", "CqrError", "version"]


def version() -> str:
    return _native.lib().cqr_version().decode()


def colmajor(rows: int, cols: int, device="cuda", dtype=torch.float64, ld: int | None = None) -> torch.Tensor:
    """Uninitialised column-major (rows x cols) tensor with leading dimension ld."""
    ld = rows if ld is None else ld
    base = torch.empty((cols, ld), device=device, dtype=dtype)
    return base.t()[:rows, :]


def _ld(t: torch.Tensor, name: str) -> int:
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if not t.is_cuda:
        raise TypeError("%s must be a GPU tensor" % name)
    if t.dim() == 1:
        if t.stride(0) != 1:
            raise ValueError("%s must be contiguous" % name)
        return max(1, t.shape[0])
    rows, cols = t.shape
    if cols <= 1 and rows <= 1:
        return 1
    if t.stride(0) != 1 and rows > 1:
        raise ValueError("%s must be column-major (stride(0) == 1); use colmajor()" % name)
    return max(t.stride(1) if cols > 1 else rows, rows, 1)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def workspace_size(q: int, r: int, b: int) -> int:
    n = ctypes.c_size_t(0)
    _native.check(_native.lib().cqr_workspace_size(q, r, b, ctypes.byref(n)), "cqr_workspace_size")
    return int(n.value)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def _status(n: int, device) -> torch.Tensor:
    return torch.zeros(max(n, 1), dtype=torch.int32, device=device)


def qr_async(Y: torch.Tensor, b: int, R: torch.Tensor | None = None, work: torch.Tensor | None = None,
             info: torch.Tensor | None = None, flags: torch.Tensor | None = None):
    """CGS-QR of column-major Y (q x r) in place, enqueued on the current
    stream with no host synchronisation (capturable).  Returns (Q, R, info,
    flags) with info (1 entry) and flags (one per block) int32 device tensors
    that the kernels fill."""
    q, r = Y.shape
    ldy = _ld(Y, "Y")
    if R is None:
        R = colmajor(r, r, device=Y.device)
    ldr = _ld(R, "R")
    need = workspace_size(q, r, b)
    if work is None:
        work = _workspace(need, Y.device)
    k = -(-r // b) if r else 0
    info = _status(1, Y.device) if info is None else info
    flags = _status(k, Y.device) if flags is None else flags
    rc = _native.lib().cqr_factor(q, r, b, _ptr(Y), ldy, _ptr(R), ldr, _ptr(work), work.numel(), _ptr(info),
                                  _ptr(flags), _stream())
    _native.check(rc, "cqr_factor")
    return Y, R, info, flags


def qr(Y: torch.Tensor, b: int, R: torch.Tensor | None = None, work: torch.Tensor | None = None):
    """CGS-QR of column-major Y (q x r) in place.  Returns (Q, R, info,
    block_flags) with info and the flags read back to the host (this waits for
    the stream).  Q is Y itself; R is r x r upper triangular (column-major)."""
    r = Y.shape[1]
    k = -(-r // b) if r else 0
    Q, R, info, flags = qr_async(Y, b, R, work)
    return Q, R, int(info[0].item()), [int(v) for v in flags[:k].tolist()]


def orth(Q: torch.Tensor, R: torch.Tensor | None = None, work: torch.Tensor | None = None, sync: bool = True):
    """CholeskyQR2 of column-major Q (q x b) in place.  Returns (Q, R, info):
    info an int (sync=True, waits for the stream) or an int32 device tensor."""
    q, b = Q.shape
    if R is None:
        R = colmajor(b, b, device=Q.device)
    if work is None:
        work = _workspace(workspace_size(q, b, b), Q.device)
    info = _status(1, Q.device)
    rc = _native.lib().cqr_orth(q, b, _ptr(Q), _ld(Q, "Q"), _ptr(R), _ld(R, "R"), _ptr(work), work.numel(),
                                _ptr(info), _stream())
    _native.check(rc, "cqr_orth")
    return Q, R, (int(info[0].item()) if sync else info)


def orth_against(Q: torch.Tensor, P: torch.Tensor, H: torch.Tensor | None = None, R: torch.Tensor | None = None,
                 work: torch.Tensor | None = None, sync: bool = True):
    """CGS-CQR2: orthogonalise Q (q x b) against P (q x s) in place.  Returns
    (Q, H, R, info): info an int (sync=True) or an int32 device tensor."""
    q, b = Q.shape
    s = P.shape[1]
    if H is None:
        H = colmajor(max(s, 1), b, device=Q.device)[:s]
    if R is None:
        R = colmajor(b, b, device=Q.device)
    if work is None:
        work = _workspace(workspace_size(q, s + b, b), Q.device)
    ldh = max(1, H.stride(1)) if s > 0 else 1
    info = _status(1, Q.device)
    rc = _native.lib().cqr_orth_against(q, b, s, _ptr(Q), _ld(Q, "Q"), _ptr(P), _ld(P, "P") if s else max(q, 1),
                                        _ptr(H) if s else ctypes.c_void_p(0), ldh, _ptr(R), _ld(R, "R"),
                                        _ptr(work), work.numel(), _ptr(info), _stream())
    _native.check(rc, "cqr_orth_against")
    return Q, H, R, (int(info[0].item()) if sync else info)


def set_wait_limit_us(us: int) -> None:
    """Bound of the library's bounded device-side waits (microseconds)."""
    _native.check(_native.lib().cqr_set_wait_limit_us(int(us)), "cqr_set_wait_limit_us")


def solve_workspace_size(n: int) -> int:
    """Bytes of device workspace solve() needs for order n."""
    nb = ctypes.c_size_t(0)
    _native.check(_native.lib().cqr_solve_workspace_size(n, ctypes.byref(nb)), "cqr_solve_workspace_size")
    return int(nb.value)


def solve(Q: torch.Tensor, R: torch.Tensor, rhs: torch.Tensor, work: torch.Tensor | None = None,
          status: torch.Tensor | None = None) -> torch.Tensor:
    """x = R^{-1} Q^T rhs (asynchronous on the current stream).  rhs is not
    modified.  status (optional int32 device tensor) receives 0, or 1 if the
    back substitution abandoned a bounded wait (x is then not valid)."""
    n = Q.shape[0]
    x = rhs.clone().contiguous()
    if work is None:
        work = _workspace(solve_workspace_size(n), Q.device)
    rc = _native.lib().cqr_solve(n, _ptr(Q), _ld(Q, "Q"), _ptr(R), _ld(R, "R"), _ptr(x), _ptr(work), work.numel(),
                                 _ptr(status), _stream())
    _native.check(rc, "cqr_solve")
    return x


def solve_noalloc(Q: torch.Tensor, R: torch.Tensor, rhs: torch.Tensor, status: torch.Tensor | None = None,
                  x: torch.Tensor | None = None) -> torch.Tensor:
    """solve() through the entry point that allocates nothing on the device
    (its workspace is the library's fixed per-GPU array; n <= 65536).  Only
    the output x is allocated here, and not even that when x is given."""
    n = Q.shape[0]
    if x is None:
        x = rhs.clone().contiguous()
    elif x.data_ptr() != rhs.data_ptr():
        x.copy_(rhs)
    rc = _native.lib().cqr_solve_noalloc(n, _ptr(Q), _ld(Q, "Q"), _ptr(R), _ld(R, "R"), _ptr(x), _ptr(status),
                                         _stream())
    _native.check(rc, "cqr_solve_noalloc")
    return x


def qr_mixed_async(Y: torch.Tensor, b: int, prec: int = PREC_BF16, Q: torch.Tensor | None = None,
                   R: torch.Tensor | None = None, work: torch.Tensor | None = None,
                   info: torch.Tensor | None = None, flags: torch.Tensor | None = None):
    """Low-precision CGS-QR of column-major FP64 Y (not modified): BF16
    (prec=PREC_BF16) or FP8 E4M3 (prec=PREC_FP8) MFMA projections/updates, FP64
    panel, enqueued with no host synchronisation.  Returns (Q (FP32), R (FP32),
    info, flags) with info and flags int32 device tensors."""
    q, r = Y.shape
    if Q is None:
        Q = colmajor(q, r, device=Y.device, dtype=torch.float32)
    if R is None:
        R = colmajor(r, r, device=Y.device, dtype=torch.float32)
    n = ctypes.c_size_t(0)
    _native.check(_native.lib().cqr_workspace_size_mixed(q, r, b, prec, ctypes.byref(n)), "cqr_workspace_size_mixed")
    if work is None:
        work = _workspace(int(n.value), Y.device)
    k = -(-r // b) if r else 0
    info = _status(1, Y.device) if info is None else info
    flags = _status(k, Y.device) if flags is None else flags
    rc = _native.lib().cqr_factor_mixed(q, r, b, prec, _ptr(Y), _ld(Y, "Y"), _ptr(Q), _ld32(Q, "Q"), _ptr(R),
                                        _ld32(R, "R"), _ptr(work), work.numel(), _ptr(info), _ptr(flags), _stream())
    _native.check(rc, "cqr_factor_mixed")
    return Q, R, info, flags


def qr_mixed(Y: torch.Tensor, b: int, prec: int = PREC_BF16, Q: torch.Tensor | None = None,
             R: torch.Tensor | None = None, work: torch.Tensor | None = None):
    """qr_mixed_async, then info read back to the host (waits for the
    stream).  Returns (Q (FP32), R (FP32), info)."""
    Q, R, info, _ = qr_mixed_async(Y, b, prec, Q, R, work)
    return Q, R, int(info[0].item())


def set_mixed_layout(tiled: bool = True) -> None:
    """Testing aid: tiled (default) or column-major storage of the finished
    low-precision columns of the mixed factorisation (same results)."""
    _native.check(_native.lib().cqr_set_mixed_layout(1 if tiled else 0), "cqr_set_mixed_layout")


def set_forced_breakdown(blk: int) -> None:
    """Testing aid: treat block blk (0-based) of later factorisations as broken
    down (the CGS2 fallback redoes it); -1 turns it off."""
    _native.check(_native.lib().cqr_set_forced_breakdown(int(blk)), "cqr_set_forced_breakdown")


def solve_ir(Y: torch.Tensor, Q: torch.Tensor, R: torch.Tensor, rhs: torch.Tensor, maxiter: int = 50,
             tol: float = 16.0, work: torch.Tensor | None = None):
    """FP64 iterative refinement with the low-precision factors.  Returns (x, iters, scaled_residual)."""
    n = Y.shape[0]
    x = torch.empty(n, dtype=torch.float64, device=Y.device)
    nb = ctypes.c_size_t(0)
    _native.check(_native.lib().cqr_solve_ir_workspace_size(n, ctypes.byref(nb)), "cqr_solve_ir_workspace_size")
    if work is None:
        work = _workspace(int(nb.value), Y.device)
    rhs = rhs.contiguous()
    it = ctypes.c_int32(0)
    res = ctypes.c_double(0)
    rc = _native.lib().cqr_solve_ir(n, _ptr(Y), _ld(Y, "Y"), _ptr(Q), _ld32(Q, "Q"), _ptr(R), _ld32(R, "R"), _ptr(rhs),
                                    _ptr(x), maxiter, tol, ctypes.byref(it), ctypes.byref(res), _ptr(work),
                                    work.numel(), _stream())
    _native.check(rc, "cqr_solve_ir")
    return x, int(it.value), float(res.value)


def _ld32(t: torch.Tensor, name: str) -> int:
    if t.dtype != torch.float32:
        raise TypeError("%s must be float32" % name)
    if not t.is_cuda:
        raise TypeError("%s must be a GPU tensor" % name)
    rows, cols = t.shape
    if t.stride(0) != 1 and rows > 1:
        raise ValueError("%s must be column-major (stride(0) == 1); use colmajor()" % name)
    return max(t.stride(1) if cols > 1 else rows, rows, 1)


def synth_uniform(A: torch.Tensor, seed: int, lo: float = -1.0, hi: float = 1.0) -> torch.Tensor:
    """Fill column-major A in place with the seeded U[lo, hi) stream (see inputs.py)."""
    rows, cols = A.shape if A.dim() == 2 else (A.shape[0], 1)
    rc = _native.synth_lib().cqr_synth_uniform(rows, cols, _ptr(A), _ld(A, "A"), seed & 0xFFFFFFFFFFFFFFFF,
                                               float(lo), float(hi), _stream())
    if rc != 0:
        raise CqrError("cqr_synth_uniform failed with status %d" % rc)
    return A


def prof_enable(on: bool = True) -> None:
    _native.lib().cqr_prof_enable(1 if on else 0)


def prof_reset() -> None:
    _native.lib().cqr_prof_reset()


def prof_names() -> list[str]:
    out, i = [], 0
    while True:
        p = _native.lib().cqr_prof_name(i)
        if not p:
            return out
        out.append(p.decode())
        i += 1


def prof_query(name: str) -> dict:
    n = ctypes.c_int64(0)
    ms, fl, by = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
    rc = _native.lib().cqr_prof_query(name.encode(), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl),
                                      ctypes.byref(by))
    _native.check(rc, "cqr_prof_query")
    return {"launches": int(n.value), "ms": ms.value, "flops": fl.value, "bytes": by.value}
