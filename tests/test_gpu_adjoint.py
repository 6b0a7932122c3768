"""Adjoint of the batched solve (lambda = A^{-T} g from the stored factors,
dA = -lambda x^T, db = lambda) and the torch.autograd.Function around it.

References: the oracle's gradient (FP64, from its own factors) and central
finite differences of the GPU forward with h = 1e-6.  Tolerances: the adjoint
is two backward-stable solves, so lambda and x each carry a relative error of
at most about kappa n eps, and |dA - dA_oracle| <= 16 kappa n eps max|dA|.
Finite differences carry O(h^2) truncation plus the forward's rounding divided
by h; they are held to 1e-4 relative to max|dA| (resp. max|db|).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2403_06218_amd import batched, inputs
from gpu_util import EPS

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

EPS32 = 2.0 ** -23


def _c5(count, n, seed, dtype=torch.float64):
    """U[-1, 1) entries + 4 I, right-hand sides and loss weights U[-1, 1)."""
    A = np.stack([inputs.uniform_matrix(n, n, seed + i) + 4.0 * np.eye(n) for i in range(count)])
    b = np.stack([inputs.uniform_vector(n, seed + 1000 + i) for i in range(count)])
    w = np.stack([inputs.uniform_vector(n, seed + 2000 + i) for i in range(count)])
    if dtype == torch.float32:
        A, b, w = (t.astype(np.float32).astype(np.float64) for t in (A, b, w))
    return A, b, w


def _oracle_grad(A, b, w, bw):
    ref = oracle.cgs_qr(np.asfortranarray(A), bw)
    x, rc = oracle.qr_solve(ref["Q"], ref["R"], b)
    assert rc == 0
    dA, db, rc = oracle.qr_solve_grad(ref["Q"], ref["R"], x, w)
    assert rc == 0
    return x, dA, db


@pytest.mark.parametrize("sizes", [[1, 17, 64, 100, 256, 512], [33, 300]])
def test_batched_backward_matches_oracle_gradient(sizes):
    count = len(sizes)
    batch = batched.PackedBatch(sizes)
    mats = [inputs.packed_matrix(sizes, i, 11) + 4.0 * np.eye(n) for i, n in enumerate(sizes)]
    rhs = [inputs.packed_vector(sizes, i, 12) for i in range(count)]
    ws = [inputs.packed_vector(sizes, i, 13) for i in range(count)]
    batch.A.copy_(torch.from_numpy(np.concatenate([m.ravel(order="F") for m in mats])))
    batch.B.copy_(torch.from_numpy(np.concatenate(rhs)))
    batched.factor_solve(batch)
    g = torch.from_numpy(np.concatenate(ws)).cuda()
    dA = torch.empty_like(batch.A)
    db = torch.empty_like(batch.B)
    batched.solve_backward(batch, g, dA, db)
    torch.cuda.synchronize()
    for i, n in enumerate(sizes):
        _, dAo, dbo = _oracle_grad(mats[i], rhs[i], ws[i], batched.block_width(n))
        o, vo = int(batch.offsets[i]), int(batch.voffsets[i])
        dAg = dA[o:o + n * n].view(n, n).t().cpu().numpy()
        dbg = db[vo:vo + n].cpu().numpy()
        tol = 16 * np.linalg.cond(mats[i]) * n * EPS
        np.testing.assert_allclose(dbg, dbo, rtol=0, atol=tol * np.abs(dbo).max(), err_msg="db n=%d" % n)
        np.testing.assert_allclose(dAg, dAo, rtol=0, atol=tol * np.abs(dAo).max(), err_msg="dA n=%d" % n)


def test_autograd_c5_fp64_against_oracle_and_finite_differences():
    """Batch of 4 matrices n = 512 (U[-1, 1) + 4 I), loss = sum(w * x)."""
    count, n, h = 4, 512, 1e-6
    A, b, w = _c5(count, n, seed=500)
    At = torch.from_numpy(A).cuda().requires_grad_(True)
    bt = torch.from_numpy(b).cuda().requires_grad_(True)
    wt = torch.from_numpy(w).cuda()
    x = batched.qr_solve(At, bt)
    (wt * x).sum().backward()
    dA = At.grad.cpu().numpy()
    db = bt.grad.cpu().numpy()
    bw = batched.block_width(n)
    for k in range(count):
        xo, dAo, dbo = _oracle_grad(A[k], b[k], w[k], bw)
        tol = 16 * np.linalg.cond(A[k]) * n * EPS
        np.testing.assert_allclose(x[k].detach().cpu().numpy(), xo, rtol=0, atol=tol * np.abs(xo).max())
        np.testing.assert_allclose(db[k], dbo, rtol=0, atol=tol * np.abs(dbo).max())
        np.testing.assert_allclose(dA[k], dAo, rtol=0, atol=tol * np.abs(dAo).max())
    # Central differences on 64 sampled entries per matrix, all perturbations
    # in one batched forward call.
    rng = np.random.default_rng(5)
    picks = [rng.choice(n * n, 64, replace=False) for _ in range(count)]
    pert = np.empty((count * 128, n, n))
    rhs = np.empty((count * 128, n))
    for k in range(count):
        for t, e in enumerate(picks[k]):
            i, j = e % n, e // n
            for sgn, slot in ((1.0, 2 * t), (-1.0, 2 * t + 1)):
                P = A[k].copy()
                P[i, j] += sgn * h
                pert[k * 128 + slot] = P
                rhs[k * 128 + slot] = b[k]
    with torch.no_grad():
        xp = batched.qr_solve(torch.from_numpy(pert).cuda(), torch.from_numpy(rhs).cuda()).cpu().numpy()
    for k in range(count):
        loss = xp[k * 128:(k + 1) * 128] @ w[k]
        fd = (loss[0::2] - loss[1::2]) / (2 * h)
        got = np.array([dA[k][e % n, e // n] for e in picks[k]])
        np.testing.assert_allclose(got, fd, rtol=0, atol=1e-4 * np.abs(dA[k]).max())
    # db by central differences on every entry of one matrix's right-hand side.
    k = 0
    pb = np.repeat(b[k][None, :], 2 * n, axis=0)
    pb[np.arange(n) * 2, np.arange(n)] += h
    pb[np.arange(n) * 2 + 1, np.arange(n)] -= h
    with torch.no_grad():
        xb = batched.qr_solve(torch.from_numpy(np.repeat(A[k][None], 2 * n, axis=0)).cuda(),
                              torch.from_numpy(pb).cuda()).cpu().numpy()
    lb = xb @ w[k]
    np.testing.assert_allclose(db[k], (lb[0::2] - lb[1::2]) / (2 * h), rtol=0, atol=1e-4 * np.abs(db[k]).max())


def test_autograd_c5_fp32():
    """FP32 path: lambda solves A^T lambda = w to FP32 backward error, and dA is
    exactly the FP32 outer product -lambda x^T."""
    count, n = 4, 512
    A, b, w = _c5(count, n, seed=600, dtype=torch.float32)
    At = torch.from_numpy(A).float().cuda().requires_grad_(True)
    bt = torch.from_numpy(b).float().cuda().requires_grad_(True)
    x = batched.qr_solve(At, bt)
    (torch.from_numpy(w).float().cuda() * x).sum().backward()
    lam = bt.grad.double().cpu().numpy()
    xs = x.detach().double().cpu().numpy()
    dA = At.grad.cpu().numpy()
    for k in range(count):
        r = np.abs(A[k].T @ lam[k] - w[k]).max() / (np.abs(A[k]).sum(axis=0).max() * np.abs(lam[k]).max() * n * EPS32)
        assert r < 16, r
        outer = -(lam[k].astype(np.float32)[:, None] * xs[k].astype(np.float32)[None, :])
        assert np.array_equal(dA[k], outer)
        hpl = np.abs(A[k] @ xs[k] - b[k]).max() / (np.abs(A[k]).sum(axis=1).max() * np.abs(xs[k]).max() * n * EPS32)
        assert hpl < 16, hpl


def test_single_matrix_autograd():
    n = 96
    A = inputs.uniform_matrix(n, n, 7) + 4.0 * np.eye(n)
    b = inputs.uniform_vector(n, 8)
    w = inputs.uniform_vector(n, 9)
    At = torch.from_numpy(A).cuda().requires_grad_(True)
    bt = torch.from_numpy(b).cuda().requires_grad_(True)
    x = batched.qr_solve(At, bt)
    assert x.shape == (n,)
    (torch.from_numpy(w).cuda() * x).sum().backward()
    _, dAo, dbo = _oracle_grad(A, b, w, batched.block_width(n))
    tol = 16 * np.linalg.cond(A) * n * EPS
    np.testing.assert_allclose(At.grad.cpu().numpy(), dAo, rtol=0, atol=tol * np.abs(dAo).max())
    np.testing.assert_allclose(bt.grad.cpu().numpy(), dbo, rtol=0, atol=tol * np.abs(dbo).max())


def test_backward_graph_replay_matches_eager():
    """The adjoint call captured in a hipGraph replays to the eager bits."""
    sizes = [64, 200, 512, 31]
    batch = batched.PackedBatch(sizes)
    mats = [inputs.packed_matrix(sizes, i, 21) + 4.0 * np.eye(n) for i, n in enumerate(sizes)]
    batch.A.copy_(torch.from_numpy(np.concatenate([m.ravel(order="F") for m in mats])))
    batch.B.copy_(torch.from_numpy(np.concatenate([inputs.packed_vector(sizes, i, 22) for i in range(4)])))
    batched.factor_solve(batch)
    g = torch.from_numpy(np.concatenate([inputs.packed_vector(sizes, i, 23) for i in range(4)])).cuda()
    dA = torch.empty_like(batch.A)
    db = torch.empty_like(batch.B)
    batched.solve_backward(batch, g, dA, db)
    torch.cuda.synchronize()
    refA, refb = dA.clone(), db.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batched.solve_backward(batch, g, dA, db)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batched.solve_backward(batch, g, dA, db)
    for _ in range(3):
        dA.fill_(float("nan"))
        db.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(dA, refA) and torch.equal(db, refb)
