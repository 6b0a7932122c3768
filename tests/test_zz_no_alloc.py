"""cqr_solve_noalloc (the solve for callers that cannot allocate device
memory; its workspace is the library's fixed per-GPU array) against cqr_solve
with a caller workspace, through the C ABI: the same kernels on the same
inputs, so the same bits.  Two calls in a row, the second with a smaller n,
so the second runs over what the first left in the shared array; the size
limit is rejected on the host before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2403_06218_amd as cqr
from paper_2403_06218_amd import _native, inputs

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

TOO_LARGE = -102


def _factors(n, seed):
    Y = inputs.uniform_matrix(n, n, seed=seed)
    Yd = cqr.colmajor(n, n)
    Yd.copy_(torch.from_numpy(Y))
    Q, R, info, _ = cqr.qr(Yd, 64)
    assert info == 0
    return Y, Q, R


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def _call_both(Q, R, rhs):
    """x from cqr_solve (caller workspace) and from cqr_solve_noalloc, both
    through the C ABI on the current stream, and their status words."""
    lib = _native.lib()
    n = Q.shape[0]
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    x_ref = rhs.clone()
    x_na = rhs.clone()
    s_ref = torch.full((1,), -9, dtype=torch.int32, device="cuda")
    s_na = torch.full((1,), -9, dtype=torch.int32, device="cuda")
    work = torch.empty(cqr.solve_workspace_size(n), dtype=torch.uint8, device="cuda")
    assert lib.cqr_solve(n, _ptr(Q), Q.stride(1), _ptr(R), R.stride(1), _ptr(x_ref), _ptr(work), work.numel(),
                         _ptr(s_ref), st) == 0
    assert lib.cqr_solve_noalloc(n, _ptr(Q), Q.stride(1), _ptr(R), R.stride(1), _ptr(x_na), _ptr(s_na), st) == 0
    torch.cuda.synchronize()
    return x_ref, x_na, int(s_ref[0]), int(s_na[0])


def test_noalloc_solve_matches_solve_twice_then_smaller():
    for n, seed in ((3000, 41), (1000, 42)):
        print("cqr_solve_noalloc vs cqr_solve: n=%d seed=%d" % (n, seed), flush=True)
        Y, Q, R = _factors(n, seed)
        rhs = torch.from_numpy(inputs.uniform_vector(n, seed + 100)).cuda()
        x_ref, x_na, s_ref, s_na = _call_both(Q, R, rhs)
        assert s_ref == 0 and s_na == 0
        assert torch.equal(x_ref, x_na), "no-allocation solve differs from cqr_solve (n=%d)" % n
        xh = x_na.cpu().numpy()
        hpl = np.abs(Y @ xh - rhs.cpu().numpy()).max() / (np.abs(Y).sum(axis=1).max() * np.abs(xh).max() * n
                                                          * 2.0 ** -52)
        assert hpl < 16, hpl
        ref = oracle.cgs_qr(Y, 64)
        xo, _ = oracle.qr_solve(ref["Q"], ref["R"], rhs.cpu().numpy())
        tol = 8 * np.linalg.cond(Y) * n * 2.0 ** -52
        assert np.abs(xh - xo).max() <= tol * np.abs(xo).max()


def test_noalloc_rejects_sizes_above_its_scratch():
    lib = _native.lib()
    v = ctypes.c_void_p(0x1000)  # never dereferenced: the size check fails first
    assert lib.cqr_solve_noalloc(65537, v, 65537, v, 65537, v, None, None) == TOO_LARGE
    assert b"65536" in lib.cqr_status_string(TOO_LARGE)
    Q = cqr.colmajor(65537, 1)
    with pytest.raises(_native.CqrError, match="65536"):
        cqr.solve_noalloc(Q, Q, torch.zeros(65537, dtype=torch.float64, device="cuda"))
