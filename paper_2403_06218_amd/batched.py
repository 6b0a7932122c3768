"""Batched form: many independent square systems of uneven size (n <= 512).

``PackedBatch`` stores a batch in three flat device buffers (A then Q, R, and
the right-hand sides then the solutions), each matrix column-major with leading
dimension n_i, together with the device arrays of sizes, leading dimensions and
element pointers that ``cqr_batched_factor_solve`` takes.  ``factor_solve``
marshals them into the library; every step of the factorisation and the solve
runs in its kernels.

``tune`` is the autotuner of the batched form: for each size bucket it times
every kernel instance that can serve the bucket on a synthetic batch of that
bucket's sizes and installs the fastest per bucket as the library's plan.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import _native
from ._native import CqrError

F64 = 0
F32 = 1
_DT = {torch.float64: F64, torch.float32: F32}
NMAX = 512


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _vp(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


class PackedBatch:
    """A batch of square systems in packed column-major storage on one device."""

    def __init__(self, sizes, dtype=torch.float64, device="cuda", rhs: bool = True):
        sizes = np.asarray(sizes, dtype=np.int64)
        if dtype not in _DT:
            raise TypeError("dtype must be float64 or float32")
        self.sizes = sizes
        self.dtype = dtype
        self.count = int(sizes.size)
        self.offsets = np.zeros(self.count + 1, dtype=np.int64)
        np.cumsum(sizes * sizes, out=self.offsets[1:])
        self.voffsets = np.zeros(self.count + 1, dtype=np.int64)
        np.cumsum(sizes, out=self.voffsets[1:])
        total = int(self.offsets[-1])
        self.A = torch.zeros(max(total, 1), dtype=dtype, device=device)
        self.R = torch.zeros(max(total, 1), dtype=dtype, device=device)
        self.B = torch.zeros(max(int(self.voffsets[-1]), 1), dtype=dtype, device=device) if rhs else None
        es = self.A.element_size()
        n32 = torch.from_numpy(sizes.astype(np.int32))
        self.n_dev = n32.to(device)
        self.lda_dev = n32.to(device)
        self.ldr_dev = n32.to(device)
        off = torch.from_numpy(self.offsets[:-1].copy())
        self.a_ptrs = (off * es + self.A.data_ptr()).to(device)
        self.r_ptrs = (off * es + self.R.data_ptr()).to(device)
        if rhs:
            voff = torch.from_numpy(self.voffsets[:-1].copy())
            self.b_ptrs = (voff * es + self.B.data_ptr()).to(device)
        else:
            self.b_ptrs = None
        # Byte offsets of every matrix / vector, for building pointer arrays of
        # other buffers with the same packing on the device (no host copy, so
        # that calls stay capturable).
        self.moff_bytes = (off * es).to(device)
        self.voff_bytes = (torch.from_numpy(self.voffsets[:-1].copy()) * es).to(device)
        self.info = torch.zeros(max(self.count, 1), dtype=torch.int32, device=device)
        self.flags = torch.zeros(max(self.count, 1), dtype=torch.int32, device=device)

    # Column-major views of matrix i.
    def _view(self, flat: torch.Tensor, i: int) -> torch.Tensor:
        n = int(self.sizes[i])
        o = int(self.offsets[i])
        return flat[o:o + n * n].view(n, n).t()

    def a(self, i: int) -> torch.Tensor:
        return self._view(self.A, i)

    def r(self, i: int) -> torch.Tensor:
        return self._view(self.R, i)

    def b(self, i: int) -> torch.Tensor:
        o = int(self.voffsets[i])
        return self.B[o:o + int(self.sizes[i])]


def workspace_size(count: int) -> int:
    nb = ctypes.c_size_t(0)
    _native.check(_native.lib().cqr_batched_workspace_size(count, ctypes.byref(nb)), "cqr_batched_workspace_size")
    return nb.value


def factor_solve(batch: PackedBatch, work: torch.Tensor | None = None, solve: bool = True) -> PackedBatch:
    """CGS-QR of every A_i in place (A_i := Q_i, R_i) and, with solve, B_i := x_i.

    Runs on the current stream without synchronising; ``batch.info`` /
    ``batch.flags`` receive the per-matrix breakdown reports.
    """
    nbytes = workspace_size(batch.count)
    if work is None or work.numel() < nbytes:
        work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=batch.A.device)
    b_ptrs = batch.b_ptrs if (solve and batch.b_ptrs is not None) else None
    rc = _native.lib().cqr_batched_factor_solve(
        batch.count, _DT[batch.dtype], _vp(batch.n_dev), _vp(batch.a_ptrs), _vp(batch.lda_dev), _vp(batch.r_ptrs),
        _vp(batch.ldr_dev), _vp(b_ptrs), _vp(batch.info), _vp(batch.flags), _vp(work), ctypes.c_size_t(nbytes),
        _stream())
    _native.check(rc, "cqr_batched_factor_solve")
    return batch


def instances() -> list[dict]:
    out = []
    i = 0
    while True:
        dt, nm, bw, wv = (ctypes.c_int32() for _ in range(4))
        rc = _native.lib().cqr_batched_instance(i, ctypes.byref(dt), ctypes.byref(nm), ctypes.byref(bw),
                                                ctypes.byref(wv))
        if rc != 0:
            return out
        out.append({"id": i, "dtype": dt.value, "nmax": nm.value, "bw": bw.value, "waves": wv.value})
        i += 1


def get_plan(dtype=torch.float64) -> dict:
    nb = ctypes.c_int32()
    hi = (ctypes.c_int32 * 8)()
    inst = (ctypes.c_int32 * 8)()
    _native.check(_native.lib().cqr_batched_plan_get(_DT[dtype], ctypes.byref(nb), hi, inst), "cqr_batched_plan_get")
    return {"hi": list(hi[:nb.value]), "inst": list(inst[:nb.value])}


def set_plan(dtype, hi, inst) -> None:
    n = len(hi)
    h = (ctypes.c_int32 * max(n, 1))(*hi)
    s = (ctypes.c_int32 * max(n, 1))(*inst)
    _native.check(_native.lib().cqr_batched_plan_set(_DT[dtype], n, h, s), "cqr_batched_plan_set")


def block_width(n: int, dtype=torch.float64) -> int:
    """Block width the current plan uses for a matrix of size n."""
    plan = get_plan(dtype)
    insts = instances()
    for h, i in zip(plan["hi"], plan["inst"]):
        if n <= h:
            return insts[i]["bw"]
    raise ValueError("n = %d is above the plan's largest size %d" % (n, plan["hi"][-1]))


def _fill(batch: PackedBatch, seed: int) -> None:
    """Synthetic U[-1, 1) entries and right-hand sides (GPU generator)."""
    from . import synth_uniform
    if batch.dtype == torch.float64:
        synth_uniform(batch.A.view(-1, 1), seed)
        if batch.B is not None:
            synth_uniform(batch.B.view(-1, 1), seed + 1)
    else:
        tmp = torch.empty(batch.A.numel(), dtype=torch.float64, device=batch.A.device)
        synth_uniform(tmp.view(-1, 1), seed)
        batch.A.copy_(tmp)
        if batch.B is not None:
            tb = torch.empty(batch.B.numel(), dtype=torch.float64, device=batch.A.device)
            synth_uniform(tb.view(-1, 1), seed + 1)
            batch.B.copy_(tb)


def tune(dtype=torch.float64, buckets=((0, 64), (64, 256), (256, 512)), count: int = 1024, reps: int = 3,
         seed: int = 12345, verbose: bool = False) -> dict:
    """Times every instance able to serve each bucket and installs the fastest.

    Each bucket (lo, hi] is timed on ``count`` matrices with sizes uniform in
    it (fewer for the largest sizes), entries U[-1, 1).  Returns the plan and
    the timings (ms per batch) of every candidate.
    """
    from .inputs import batch_sizes
    dt = _DT[dtype]
    insts = [i for i in instances() if i["dtype"] == dt]
    old = get_plan(dtype)
    his, chosen, table = [], [], {}
    try:
        for (lo, hi) in buckets:
            cnt = count if hi <= 256 else max(64, count // 4)
            sizes = batch_sizes(cnt, lo + 1, hi, seed + hi)
            batch = PackedBatch(sizes, dtype=dtype)
            a0 = torch.empty_like(batch.A)
            b0 = torch.empty_like(batch.B)
            _fill(batch, seed)
            a0.copy_(batch.A)
            b0.copy_(batch.B)
            best, best_ms = None, None
            for ins in insts:
                if ins["nmax"] < hi:
                    continue
                if lo > 0:
                    filler = next(i["id"] for i in insts if i["nmax"] >= lo)
                    set_plan(dtype, [lo, hi], [filler, ins["id"]])
                else:
                    set_plan(dtype, [hi], [ins["id"]])
                times = []
                for _ in range(reps + 1):
                    batch.A.copy_(a0)
                    batch.B.copy_(b0)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    factor_solve(batch)
                    torch.cuda.synchronize()
                    times.append((time.perf_counter() - t0) * 1e3)
                ms = float(np.median(times[1:]))
                table["%d-%d:%d" % (lo, hi, ins["id"])] = ms
                if verbose:
                    print("bucket (%d, %d] instance %s: %.3f ms" % (lo, hi, ins, ms), flush=True)
                if best_ms is None or ms < best_ms:
                    best, best_ms = ins["id"], ms
            if best is None:
                raise CqrError("no instance serves sizes up to %d" % hi)
            his.append(hi)
            chosen.append(best)
    except Exception:
        set_plan(dtype, old["hi"], old["inst"])
        raise
    set_plan(dtype, his, chosen)
    return {"hi": his, "inst": chosen, "timings_ms": table}


def solve_backward(batch: PackedBatch, g: torch.Tensor, dA: torch.Tensor, db: torch.Tensor) -> None:
    """Adjoint of ``factor_solve``: with batch.A holding Q, batch.R holding R and
    batch.B holding x, writes dA (flat, packed like batch.A) = -lambda x^T and
    db (flat, packed like batch.B) = lambda for lambda = A^{-T} g (g packed like
    batch.B).  Asynchronous on the current stream."""
    for t, ref, name in ((g, batch.B, "g"), (db, batch.B, "db"), (dA, batch.A, "dA")):
        if t.dtype != batch.dtype or not t.is_cuda or t.numel() < ref.numel() or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s GPU tensor of at least %d elements"
                             % (name, batch.dtype, ref.numel()))
    g_ptrs = batch.voff_bytes + g.data_ptr()
    db_ptrs = batch.voff_bytes + db.data_ptr()
    da_ptrs = batch.moff_bytes + dA.data_ptr()
    rc = _native.lib().cqr_batched_solve_backward(
        batch.count, _DT[batch.dtype], _vp(batch.n_dev), _vp(batch.a_ptrs), _vp(batch.lda_dev), _vp(batch.r_ptrs),
        _vp(batch.ldr_dev), _vp(batch.b_ptrs), _vp(g_ptrs), _vp(da_ptrs), _vp(batch.lda_dev), _vp(db_ptrs),
        _stream())
    _native.check(rc, "cqr_batched_solve_backward")


class QRSolve(torch.autograd.Function):
    """x = A^{-1} b for a batch of square systems A (..., n, n), b (..., n),
    n <= 512, through the batched CGS-QR factorisation and solve; the backward
    pass is the library's adjoint kernel (lambda = A^{-T} g from the stored
    factors, dA = -lambda x^T, db = lambda).  ``n`` above the batched plan's
    largest size raises ValueError.  A block that breaks down is redone by the
    column-by-column fallback inside the kernel; the per-matrix ``info`` of
    the batch (nonzero on a fallback) stays on the device and is not read."""

    @staticmethod
    def forward(ctx, A, b):
        single = A.dim() == 2
        A3 = A.unsqueeze(0) if single else A
        b2 = b.unsqueeze(0) if single else b
        nb, n, n2 = A3.shape
        if n != n2 or b2.shape != (nb, n):
            raise ValueError("A must be (..., n, n) and b (..., n)")
        # The kernels skip a matrix above the plan's largest size (info = -1,
        # x left as b); refuse it here instead of returning that silently.
        top = get_plan(A.dtype)["hi"][-1]
        if n > top:
            raise ValueError("n = %d is above the batched plan's largest size %d" % (n, top))
        batch = PackedBatch([n] * nb, dtype=A.dtype, device=A.device)
        # Column-major storage of A_i is row-major storage of A_i^T.
        batch.A.view(nb, n, n).copy_(A3.detach().transpose(1, 2))
        batch.B.view(nb, n).copy_(b2.detach())
        factor_solve(batch)
        ctx.batch = batch
        ctx.single = single
        x = batch.B.view(nb, n).clone()
        return x[0] if single else x

    @staticmethod
    def backward(ctx, gx):
        batch = ctx.batch
        nb, n = batch.count, int(batch.sizes[0])
        g = (gx.unsqueeze(0) if ctx.single else gx).to(batch.dtype).contiguous().view(-1)
        dA = torch.empty_like(batch.A)
        db = torch.empty_like(batch.B)
        solve_backward(batch, g, dA, db)
        dA3 = dA.view(nb, n, n).transpose(1, 2)
        db2 = db.view(nb, n)
        if ctx.single:
            return dA3[0], db2[0]
        return dA3, db2


def qr_solve(A: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Differentiable batched solve x = A^{-1} b (see QRSolve)."""
    return QRSolve.apply(A, b)
