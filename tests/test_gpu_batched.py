"""Batched form (many square systems of uneven size, one persistent launch per
size bucket) through the C ABI, against the CPU oracle.

Each matrix is compared with the oracle's CGS-QR at the block width the plan
uses for its size.  Tolerances as in the single-matrix parity tests:
|dQ| <= 8 kappa q eps, |dR| <= 8 kappa q eps ||Y||_2, backward-error bars
< 16 (reconstruction, orthogonality, HPL residual), info and flags exact on the
FP64 path.  The FP32 path is held to the same bars with eps = 2^-23 against
the FP64 oracle run on the FP32-rounded inputs; its info may differ from the
FP64 oracle's (FP32 Cholesky breaks down earlier), and its factors must stay
valid either way.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2403_06218_amd import batched, inputs
from gpu_util import EPS, hpl_ratio

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

EPS32 = 2.0 ** -23
EDGE = [1, 2, 7, 8, 15, 16, 17, 31, 32, 33, 47, 63, 64, 65, 96, 127, 128, 129, 200, 255, 256, 257, 300, 384,
        511, 512]


def _make(sizes, dtype, seed, edit=None):
    sizes = np.asarray(sizes, dtype=np.int64)
    batch = batched.PackedBatch(sizes, dtype=dtype)
    mats = [inputs.packed_matrix(sizes, i, seed) for i in range(sizes.size)]
    rhs = [inputs.packed_vector(sizes, i, seed + 1) for i in range(sizes.size)]
    if edit is not None:
        edit(mats)
    flat = np.concatenate([m.ravel(order="F") for m in mats])
    batch.A.copy_(torch.from_numpy(flat).to(dtype))
    batch.B.copy_(torch.from_numpy(np.concatenate(rhs)).to(dtype))
    if dtype == torch.float32:
        mats = [m.astype(np.float32).astype(np.float64) for m in mats]
        rhs = [v.astype(np.float32).astype(np.float64) for v in rhs]
    return batch, mats, rhs


def _host(batch, i):
    return (batch.a(i).cpu().numpy().astype(np.float64), batch.r(i).cpu().numpy().astype(np.float64),
            batch.b(i).cpu().numpy().astype(np.float64))


def _check_one(batch, i, Y, rhs, eps, exact_info):
    n = Y.shape[0]
    b = batched.block_width(n, batch.dtype)
    Qg, Rg, xg = _host(batch, i)
    info = int(batch.info[i])
    flags = int(batch.flags[i])
    ref = oracle.cgs_qr(Y, b)
    if exact_info:
        assert info == ref["info"], (n, info, ref["info"])
        assert flags == int(np.bitwise_or.reduce(np.asarray(ref["block_flags"], dtype=np.int64))), (n, flags)
    kappa = np.linalg.cond(Y)
    tol = 8 * kappa * n * eps
    if tol < 0.5:
        np.testing.assert_allclose(Qg, ref["Q"], rtol=0, atol=tol, err_msg="Q, n=%d" % n)
        np.testing.assert_allclose(Rg, ref["R"], rtol=0, atol=tol * np.linalg.norm(Y, 2), err_msg="R, n=%d" % n)
    assert np.array_equal(np.tril(Rg, -1), np.zeros_like(Rg)), n
    assert (np.diag(Rg) > 0).all(), n
    assert np.linalg.norm(Y - Qg @ Rg) / (n * eps * np.linalg.norm(Y)) < 16, n
    assert np.linalg.norm(Qg.T @ Qg - np.eye(n)) / (n * eps) < 16, n
    hpl = np.abs(Y @ xg - rhs).max() / (np.abs(Y).sum(axis=1).max() * np.abs(xg).max() * n * eps)
    assert hpl < 16, (n, hpl)
    if tol < 0.5:
        xo, rc = oracle.qr_solve(ref["Q"], ref["R"], rhs)
        assert rc == 0
        assert np.abs(xg - xo).max() <= 8 * kappa * n * eps * np.abs(xo).max(), n


def test_fp64_edge_and_random_sizes():
    sizes = EDGE + list(inputs.batch_sizes(100, 8, 256, seed=3))
    batch, mats, rhs = _make(sizes, torch.float64, seed=21)
    batched.factor_solve(batch)
    torch.cuda.synchronize()
    for i in range(len(sizes)):
        _check_one(batch, i, mats[i], rhs[i], EPS, exact_info=True)


def test_fp32_edge_and_random_sizes():
    sizes = EDGE + list(inputs.batch_sizes(60, 8, 256, seed=4))
    batch, mats, rhs = _make(sizes, torch.float32, seed=22)
    batched.factor_solve(batch)
    torch.cuda.synchronize()
    assert (batch.info.cpu().numpy() >= 0).all()
    for i in range(len(sizes)):
        _check_one(batch, i, mats[i], rhs[i], EPS32, exact_info=False)


@pytest.mark.parametrize("inst", [i["id"] for i in batched.instances()])
def test_every_instance(inst):
    """Each kernel instance, installed as the only bucket, on sizes up to its nmax."""
    meta = batched.instances()[inst]
    dtype = torch.float64 if meta["dtype"] == batched.F64 else torch.float32
    old = batched.get_plan(dtype)
    batched.set_plan(dtype, [meta["nmax"]], [inst])
    try:
        sizes = sorted({n for n in (1, 16, 17, 33, 100, meta["nmax"] // 2 + 3, meta["nmax"]) if n <= meta["nmax"]})
        batch, mats, rhs = _make(sizes, dtype, seed=30 + inst)
        batched.factor_solve(batch)
        torch.cuda.synchronize()
        for i in range(len(sizes)):
            _check_one(batch, i, mats[i], rhs[i], EPS if dtype == torch.float64 else EPS32,
                       exact_info=dtype == torch.float64)
    finally:
        batched.set_plan(dtype, old["hi"], old["inst"])


def test_fallback_and_zero_column_in_batch():
    """A Hilbert block (second block) and an exactly zero column (first block)
    among ordinary matrices: the same info and flags as the oracle."""
    sizes = [48, 40, 100, 48]

    def edit(mats):
        i, j = np.arange(48), np.arange(16)
        mats[0][:, 16:32] = 1.0 / (i[:, None] + j[None, :] + 1.0)
        mats[1][:, 5] = 0.0

    batch, mats, rhs = _make(sizes, torch.float64, seed=40, edit=edit)
    assert batched.block_width(48) == 16 and batched.block_width(40) == 16
    batched.factor_solve(batch)
    torch.cuda.synchronize()
    info = batch.info.cpu().numpy()
    flags = batch.flags.cpu().numpy()
    ref0 = oracle.cgs_qr(mats[0], 16)
    ref1 = oracle.cgs_qr(mats[1], 16)
    assert info[0] == ref0["info"] == 2 and flags[0] == 1
    assert info[1] == ref1["info"] == 1 and flags[1] == 3
    Q0, R0, _ = _host(batch, 0)
    assert np.linalg.norm(mats[0] - Q0 @ R0) < 1e-14 * np.linalg.norm(mats[0])
    assert np.linalg.norm(Q0.T @ Q0 - np.eye(48)) / (48 * EPS) < 16
    Q1, R1, _ = _host(batch, 1)
    assert R1[5, 5] == 0.0 and not Q1[:, 5].any()
    np.testing.assert_allclose(Q1 @ R1, mats[1], atol=1e-13)
    keep = [c for c in range(40) if c != 5]
    np.testing.assert_allclose(Q1[:, keep], ref1["Q"][:, keep], atol=1e-12)
    np.testing.assert_allclose(R1, ref1["R"], atol=1e-12)
    for i in (2, 3):
        _check_one(batch, i, mats[i], rhs[i], EPS, exact_info=True)


def test_invalid_entries_reported_and_untouched():
    sizes = [20, 30, 25]
    batch, mats, rhs = _make(sizes, torch.float64, seed=50)
    lda = batch.lda_dev.clone()
    lda[1] = 29  # lda < n
    batch.lda_dev.copy_(lda)
    a1 = batch.a(1).clone()
    batched.factor_solve(batch)
    torch.cuda.synchronize()
    info = batch.info.cpu().numpy()
    assert info[1] == -1 and info[0] == 0 and info[2] == 0
    assert torch.equal(batch.a(1), a1)
    for i in (0, 2):
        _check_one(batch, i, mats[i], rhs[i], EPS, exact_info=True)


def test_graph_replay_matches_eager():
    """The whole batched call captured in a hipGraph and replayed three times,
    with eager work between replays, gives the eager bits every time."""
    sizes = list(inputs.batch_sizes(300, 8, 256, seed=6))
    batch, _, _ = _make(sizes, torch.float64, seed=60)
    a0, b0 = batch.A.clone(), batch.B.clone()
    work = torch.empty(max(batched.workspace_size(batch.count), 1), dtype=torch.uint8, device="cuda")
    batched.factor_solve(batch, work)
    torch.cuda.synchronize()
    refA, refR, refB = batch.A.clone(), batch.R.clone(), batch.B.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.A.copy_(a0)
        batch.B.copy_(b0)
        batched.factor_solve(batch, work)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        batch.A.copy_(a0)
        batch.B.copy_(b0)
        batch.R.zero_()
        batched.factor_solve(batch, work)
    for _ in range(3):
        batch.A.fill_(float("nan"))
        batch.R.fill_(float("nan"))
        batch.B.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(batch.A, refA) and torch.equal(batch.R, refR) and torch.equal(batch.B, refB)


def test_repeated_runs_bit_identical():
    sizes = list(inputs.batch_sizes(200, 8, 256, seed=7))
    b1, _, _ = _make(sizes, torch.float64, seed=70)
    b2, _, _ = _make(sizes, torch.float64, seed=70)
    batched.factor_solve(b1)
    batched.factor_solve(b2)
    torch.cuda.synchronize()
    assert torch.equal(b1.A, b2.A) and torch.equal(b1.R, b2.R) and torch.equal(b1.B, b2.B)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_ten_thousand_uneven_sizes(dtype):
    """The benchmark batch: 10,000 matrices, n uniform in [8, 256], U[-1, 1]
    entries from the GPU generator.  Sampled matrices against the oracle, every
    matrix against the HPL bar (residual computed by torch on the GPU)."""
    sizes = inputs.batch_sizes(10000, 8, 256, seed=0)
    batch = batched.PackedBatch(sizes, dtype=dtype)
    batched._fill(batch, seed=100)
    a0, b0 = batch.A.clone(), batch.B.clone()
    batched.factor_solve(batch)
    torch.cuda.synchronize()
    assert (batch.info.cpu().numpy() >= 0).all()
    eps = EPS if dtype == torch.float64 else EPS32
    worst = 0.0
    for i in range(batch.count):
        n = int(sizes[i])
        o = int(batch.offsets[i])
        Y = a0[o:o + n * n].view(n, n).t().double()
        x = batch.b(i).double()
        rhs = b0[int(batch.voffsets[i]):int(batch.voffsets[i]) + n].double()
        r = (Y @ x - rhs).abs().max() / (Y.abs().sum(dim=1).max() * x.abs().max() * n * eps)
        worst = max(worst, float(r))
    assert worst < 16, worst
    rng = np.random.default_rng(1)
    for i in rng.choice(batch.count, 12, replace=False):
        Y = inputs.packed_matrix(sizes, int(i), 100)
        rhs = inputs.packed_vector(sizes, int(i), 101)
        if dtype == torch.float32:
            Y = Y.astype(np.float32).astype(np.float64)
            rhs = rhs.astype(np.float32).astype(np.float64)
        _check_one(batch, int(i), Y, rhs, eps, exact_info=dtype == torch.float64)
