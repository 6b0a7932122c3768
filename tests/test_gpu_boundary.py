"""The asynchronous boundary of the FP64 path, through the C ABI: cqr_factor
decides and runs the breakdown fallback (Section 3) on the device, writes info
and the block flags to device memory and never synchronises, so the whole
factorisation can be captured in a hipGraph; the bounded waits of the
fallback's grid barriers and of the back substitution report an abandoned
wait instead of hanging or returning a silently wrong result; block widths
above 128 factor their Gram matrix as a 2 x 2 block.

The abandoned-wait cases force the condition from the host by setting the
wait bound to zero: every kernel still runs to its end (all accesses stay in
bounds, every wait is bounded), only the reported status changes.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2403_06218_amd as cqr
from paper_2403_06218_amd import inputs
from gpu_util import EPS, hpl_ratio, orth_ratio, recon_ratio, to_dev, to_host

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

INFO_WAIT_ABANDONED = -2
DEFAULT_WAIT_US = 10 * 1000 * 1000


def _hilbert_case(q, w, nblk, bad, seed):
    Y = inputs.uniform_matrix(q, nblk * w, seed=seed)
    i, j = np.arange(q), np.arange(w)
    Y[:, bad * w:(bad + 1) * w] = 1.0 / (i[:, None] + j[None, :] + 1.0)
    return Y


def test_factor_is_asynchronous_and_reports_on_device():
    """info and flags arrive in device tensors; the host learns them only by
    reading those tensors (a Hilbert block forces the fallback in block 2)."""
    Y = _hilbert_case(300, 16, 4, 1, seed=31)
    Yd = to_dev(Y)
    Q, R, info, flags = cqr.qr_async(Yd, 16)
    assert info.is_cuda and flags.is_cuda
    torch.cuda.synchronize()
    ref = oracle.cgs_qr(Y, 16)
    assert int(info[0]) == ref["info"] == 2
    assert flags.cpu().tolist() == list(ref["block_flags"]) == [0, 1, 0, 0]
    Qg, Rg = to_host(Q), to_host(R)
    assert np.linalg.norm(Y - Qg @ Rg) < 1e-13 * np.linalg.norm(Y)
    assert orth_ratio(Qg) < 16


def test_factor_graph_replay_with_fallback_matches_eager():
    """The whole factorisation, the fallback of a Hilbert block included,
    captured in a hipGraph: every replay (eager calls in between) gives the
    eager call's bits, info and flags."""
    q, w = 2000, 32
    Y = _hilbert_case(q, w, 5, 2, seed=32)
    src = to_dev(Y)
    Yw = cqr.colmajor(q, Y.shape[1])
    R = cqr.colmajor(Y.shape[1], Y.shape[1])
    work = torch.empty(cqr.workspace_size(q, Y.shape[1], w), dtype=torch.uint8, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    flags = torch.zeros(5, dtype=torch.int32, device="cuda")
    Yw.copy_(src)
    cqr.qr_async(Yw, w, R=R, work=work, info=info, flags=flags)
    torch.cuda.synchronize()
    Qe, Re, ie, fe = Yw.clone(), R.clone(), info.clone(), flags.clone()
    assert int(ie[0]) == 3 and fe.cpu().tolist() == [0, 0, 1, 0, 0]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        Yw.copy_(src)
        cqr.qr_async(Yw, w, R=R, work=work, info=info, flags=flags)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        Yw.copy_(src)
        cqr.qr_async(Yw, w, R=R, work=work, info=info, flags=flags)
    for _ in range(3):
        # eager work between replays, on other buffers
        Z = to_dev(inputs.uniform_matrix(500, 64, seed=33))
        cqr.qr(Z, 16)
        Yw.fill_(float("nan"))
        R.fill_(float("nan"))
        info.fill_(-9)
        flags.fill_(-9)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Yw, Qe) and torch.equal(R, Re)
        assert torch.equal(info, ie) and torch.equal(flags, fe)


@pytest.mark.parametrize("q,r,b", [(1000, 600, 256), (700, 700, 200), (3000, 512, 256), (600, 300, 160)])
def test_wide_blocks_match_oracle(q, r, b):
    """Block widths 129..256: 2 x 2 block Cholesky of the Gram matrix."""
    Y = inputs.uniform_matrix(q, r, seed=q + r + b)
    Yd = to_dev(Y)
    Q, R, info, flags = cqr.qr(Yd, b)
    Qg, Rg = to_host(Q), to_host(R)
    ref = oracle.cgs_qr(Y, b)
    assert info == ref["info"] == 0 and list(flags) == list(ref["block_flags"])
    tol = 8 * np.linalg.cond(Y) * q * EPS
    np.testing.assert_allclose(Qg, ref["Q"], rtol=0, atol=tol)
    np.testing.assert_allclose(Rg, ref["R"], rtol=0, atol=tol * np.linalg.norm(Y, 2))
    assert recon_ratio(Y, Qg, Rg) < 16 and orth_ratio(Qg) < 16


def _graded_case(q, w, nblk, bad, seed, kappa=1e10):
    """U[-1, 1] columns with block `bad` replaced by U diag(s) V^T, s graded
    from 1 to 1/kappa: the block's Gram has condition kappa^2 = 1e20, so its
    Cholesky factorisation breaks down, while CGS2 still orthogonalises it
    (a block that is numerically rank deficient, such as a wide Hilbert block,
    is beyond CGS2: its noise-level remainders lose orthogonality in the oracle
    as in any CGS2)."""
    Y = inputs.uniform_matrix(q, nblk * w, seed=seed)
    U, _ = np.linalg.qr(inputs.normal_matrix(q, w, seed=seed + 1))
    V, _ = np.linalg.qr(inputs.normal_matrix(w, w, seed=seed + 2))
    Y[:, bad * w:(bad + 1) * w] = (U * np.logspace(0, -np.log10(kappa), w)) @ V.T
    return Y


def test_wide_block_fallback():
    """A width-192 block of condition 1e10 breaks the 2 x 2 block Cholesky;
    the block falls back to CGS2 with the oracle's info/flags, and the result
    meets the backward-error bars."""
    Y = _graded_case(1500, 192, 3, 1, seed=34)
    Yd = to_dev(Y)
    Q, R, info, flags = cqr.qr(Yd, 192)
    ref = oracle.cgs_qr(Y, 192)
    assert info == ref["info"] == 2
    assert list(flags) == list(ref["block_flags"]) == [0, 1, 0]
    Qg, Rg = to_host(Q), to_host(R)
    assert recon_ratio(Y, Qg, Rg) < 16
    assert orth_ratio(Qg) < 16
    assert recon_ratio(Y, ref["Q"], ref["R"]) < 16


def test_solve_reports_abandoned_wait():
    """With the wait bound at zero the back substitution gives up on its
    first wait: it still ends, reports status 1 and poisons x with NaN.  With
    the default bound the same solve is exact again."""
    n = 8192
    Rh = np.triu(inputs.uniform_matrix(n, n, 35))
    np.fill_diagonal(Rh, 1.0 + np.abs(Rh).sum(axis=1))
    Rd = to_dev(Rh)
    Qd = cqr.colmajor(n, n)
    Qd.zero_()
    Qd.diagonal().fill_(1.0)
    c = torch.from_numpy(inputs.uniform_vector(n, 36)).cuda()
    st = torch.full((1,), -9, dtype=torch.int32, device="cuda")
    try:
        cqr.set_wait_limit_us(0)
        x = cqr.solve(Qd, Rd, c, status=st)
        torch.cuda.synchronize()
    finally:
        cqr.set_wait_limit_us(DEFAULT_WAIT_US)
    assert int(st[0]) == 1
    assert torch.isnan(x).any()
    x = cqr.solve(Qd, Rd, c, status=st)
    torch.cuda.synchronize()
    assert int(st[0]) == 0
    assert not torch.isnan(x).any()


def test_fallback_reports_abandoned_wait():
    """The fallback's grid barriers with a zero wait bound: the launch still
    ends and info reports the abandoned wait; the default bound restores the
    oracle's info.  A zero first column makes the block's first pivot exactly
    0, so the fallback is certain to run (on 256 workgroups at q = 65536)."""
    Y = inputs.uniform_matrix(65536, 16, seed=37)
    Y[:, 8] = 0.0
    try:
        cqr.set_wait_limit_us(0)
        _, _, info, _ = cqr.qr(to_dev(Y), 8)
    finally:
        cqr.set_wait_limit_us(DEFAULT_WAIT_US)
    assert info == INFO_WAIT_ABANDONED
    _, _, info, flags = cqr.qr(to_dev(Y), 8)
    ref = oracle.cgs_qr(Y, 8)
    assert info == ref["info"] == 2 and flags == list(ref["block_flags"]) == [0, 3]


def _forced(blk):
    cqr.set_forced_breakdown(blk)


@pytest.mark.parametrize("q,r,b,blk", [(600, 600, 64, 3), (1000, 700, 256, 1), (20000, 64, 16, 2)])
def test_forced_breakdown_matches_unique_qr(q, r, b, blk):
    """A breakdown forced from the host in block blk: the block is redone by
    the CGS2 fallback.  The thin QR with positive diagonal is unique, so the
    result still matches the oracle's factorisation of the same input; info
    and the flags report the fallback.  (q = 20000, b = 16 takes the
    row-streaming path, which then keeps a copy of the block.)"""
    Y = inputs.uniform_matrix(q, r, seed=q + blk)
    try:
        _forced(blk)
        Q, R, info, flags = cqr.qr(to_dev(Y), b)
    finally:
        _forced(-1)
    ref = oracle.cgs_qr(Y, b)
    assert ref["info"] == 0
    assert info == blk + 1
    want = [0] * len(flags)
    want[blk] = 1
    assert flags == want
    Qg, Rg = to_host(Q), to_host(R)
    tol = 8 * np.linalg.cond(Y) * q * EPS
    np.testing.assert_allclose(Qg, ref["Q"], rtol=0, atol=tol)
    np.testing.assert_allclose(Rg, ref["R"], rtol=0, atol=tol * np.linalg.norm(Y, 2))
    assert recon_ratio(Y, Qg, Rg) < 16 and orth_ratio(Qg) < 16


@pytest.mark.parametrize("prec", [cqr.PREC_BF16, cqr.PREC_FP8])
def test_mixed_forced_breakdown_refines_to_oracle_solution(prec):
    """The precision form's fallback: a breakdown forced in block 5 of a
    diagonally dominant n = 2048 matrix (b = 128) is redone by CGS2 in FP64
    against the FP32 finished columns; info/flags report it on the device;
    the refinement still reaches the FP64 HPL bar and the oracle's x."""
    n, b, blk = 2048, 128, 5
    Y = inputs.diag_dominant(n, seed=51)
    rhs = inputs.uniform_vector(n, seed=52)
    Yd = to_dev(Y)
    try:
        _forced(blk)
        Q, R, info, flags = cqr.qr_mixed_async(Yd, b, prec=prec)
        torch.cuda.synchronize()
    finally:
        _forced(-1)
    assert int(info[0]) == blk + 1
    fl = flags.cpu().tolist()
    assert fl[blk] == 1 and sum(fl) == 1
    x, iters, res = cqr.solve_ir(Yd, Q, R, torch.from_numpy(rhs).cuda(), maxiter=30, tol=16.0)
    xh = x.cpu().numpy()
    assert res < 16 and hpl_ratio(Y, xh, rhs) < 16
    ref = oracle.cgs_qr(Y, b)
    xo, _ = oracle.qr_solve(ref["Q"], ref["R"], rhs)
    assert np.abs(xh - xo).max() <= 16 * np.linalg.cond(Y) * n * EPS * np.abs(xo).max()
    # The redone block is orthonormal to FP32 accuracy and orthogonal to the earlier columns.
    Qh = np.asfortranarray(Q.t().cpu().numpy().T).astype(np.float64)
    blkQ = Qh[:, blk * b:(blk + 1) * b]
    assert np.abs(blkQ.T @ blkQ - np.eye(b)).max() < 1e-5
    assert np.abs(Qh[:, :blk * b].T @ blkQ).max() < 1e-2


def test_mixed_factor_graph_replay_matches_eager():
    """cqr_factor_mixed is kernels only: captured in a hipGraph (with a forced
    fallback block), every replay gives the eager call's bits and info."""
    n, b = 1024, 128
    Yd = to_dev(inputs.diag_dominant(n, seed=53))
    Q = cqr.colmajor(n, n, dtype=torch.float32)
    R = cqr.colmajor(n, n, dtype=torch.float32)
    import ctypes
    nb = ctypes.c_size_t(0)
    cqr._native.lib().cqr_workspace_size_mixed(n, n, b, cqr.PREC_BF16, ctypes.byref(nb))
    work = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    flags = torch.zeros(n // b, dtype=torch.int32, device="cuda")
    try:
        _forced(2)
        cqr.qr_mixed_async(Yd, b, Q=Q, R=R, work=work, info=info, flags=flags)
        torch.cuda.synchronize()
        Qe, Re, ie, fe = Q.clone(), R.clone(), info.clone(), flags.clone()
        assert int(ie[0]) == 3
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            cqr.qr_mixed_async(Yd, b, Q=Q, R=R, work=work, info=info, flags=flags)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            cqr.qr_mixed_async(Yd, b, Q=Q, R=R, work=work, info=info, flags=flags)
    finally:
        _forced(-1)
    for _ in range(3):
        cqr.qr(to_dev(inputs.uniform_matrix(300, 64, seed=54)), 16)
        Q.fill_(float("nan"))
        R.fill_(float("nan"))
        info.fill_(-9)
        flags.fill_(-9)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Q, Qe) and torch.equal(R, Re)
        assert torch.equal(info, ie) and torch.equal(flags, fe)
