"""The low-precision form (BF16 MFMA projections/updates, FP64 panel) and the
FP64 iterative refinement, through the C ABI, against the CPU oracle.

Tolerances.  The BF16 products round each input to 8 significand bits
(u = 2^-8) and accumulate in FP32, so the mixed factors agree with the FP64
QR to O(u) relative to ||Y|| (bounds below use 8u * sqrt(b) scaled by
kappa); they are only a preconditioner.  The refined solution must satisfy the
FP64 HPL bar ||Yx - b||_inf / (||Y||_inf ||x||_inf n eps) < 16, and then agrees
with the oracle's FP64 solution to 16 kappa n eps relative (forward error of a
backward-stable solve).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2403_06218_amd as cqr
from paper_2403_06218_amd import inputs
from gpu_util import EPS, hpl_ratio, to_dev, to_host

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

U_BF16 = 2.0 ** -8


def _host32(T):
    return np.asfortranarray(T.t().cpu().numpy().T).astype(np.float64)


@pytest.mark.parametrize("n,b", [(512, 64), (512, 128), (1000, 64), (2048, 128), (1024, 256), (1000, 256),
                                 (700, 256), (600, 144), (4096, 256)])
def test_mixed_factor_against_oracle(n, b):
    """Diagonally dominant input (off-diagonal U[-0.5, 0.5], diagonal = row sum + 1)."""
    Y = inputs.diag_dominant(n, seed=n)
    Yd = to_dev(Y)
    Q, R, info = cqr.qr_mixed(Yd, b)
    torch.cuda.synchronize()
    assert info == 0
    Qh, Rh = _host32(Q), _host32(R)
    # Y is read only.
    assert np.array_equal(to_host(Yd), Y)
    assert np.array_equal(np.tril(Rh, -1), np.zeros_like(Rh))
    assert (np.diag(Rh) > 0).all()
    kappa = np.linalg.cond(Y)
    bound = 8 * U_BF16 * np.sqrt(b) * kappa
    ref = oracle.cgs_qr(Y, b)
    Qo, Ro = ref["Q"], ref["R"]
    assert np.abs(Qh - Qo).max() < bound
    assert np.abs(Rh - Ro).max() < bound * np.abs(Ro).max()
    assert np.linalg.norm(Y - Qh @ Rh) / np.linalg.norm(Y) < bound
    assert np.abs(Qh.T @ Qh - np.eye(n)).max() < bound


@pytest.mark.parametrize("n,b", [(512, 64), (2048, 128), (4096, 128), (4096, 256)])
def test_mixed_ir_solve_reaches_fp64_residual(n, b):
    Y = inputs.diag_dominant(n, seed=7 + n)
    rhs = inputs.uniform_vector(n, seed=8 + n)
    Yd = to_dev(Y)
    Q, R, info = cqr.qr_mixed(Yd, b)
    assert info == 0
    x, iters, res = cqr.solve_ir(Yd, Q, R, torch.from_numpy(rhs).cuda(), maxiter=50, tol=16.0)
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    assert res < 16 and 1 <= iters < 50
    assert hpl_ratio(Y, xh, rhs) < 16
    ref = oracle.cgs_qr(Y, b)
    xo, rc = oracle.qr_solve(ref["Q"], ref["R"], rhs)
    assert rc == 0
    kappa = np.linalg.cond(Y)
    assert np.abs(xh - xo).max() < 16 * kappa * n * EPS * np.abs(xo).max()


def test_mixed_ragged_and_small_blocks():
    """r not a multiple of b, b = 16, q > r (tall)."""
    Y = inputs.diag_dominant(300, seed=3)[:, :200].copy(order="F")
    Q, R, info = cqr.qr_mixed(to_dev(Y), 48)
    torch.cuda.synchronize()
    assert info == 0
    Qh, Rh = _host32(Q), _host32(R)
    assert np.linalg.norm(Y - Qh @ Rh) / np.linalg.norm(Y) < 8 * U_BF16 * np.sqrt(48) * np.linalg.cond(Y)
    Q2, R2, info2 = cqr.qr_mixed(to_dev(Y), 16)
    assert info2 == 0
    np.testing.assert_allclose(_host32(R2), Rh, atol=8 * U_BF16 * np.abs(Rh).max())


def test_mixed_rejects_unsupported_block():
    Y = to_dev(inputs.diag_dominant(64, seed=1))
    with pytest.raises(cqr.CqrError):
        cqr.qr_mixed(Y, 100)
    with pytest.raises(cqr.CqrError):
        cqr.qr_mixed(to_dev(inputs.diag_dominant(512, seed=1)), 272)


U_FP8 = 2.0 ** -4


@pytest.mark.parametrize("n,b", [(512, 64), (1000, 256), (2048, 256)])
def test_fp8_factor_backward_error(n, b):
    """FP8 (E4M3, per-column power-of-two scales) projections/updates: the
    factors reconstruct Y to a small multiple of u = 2^-4 and stay close to
    orthonormal; the triangle is exact upper with a positive diagonal."""
    Y = inputs.diag_dominant(n, seed=n + 1)
    Q, R, info = cqr.qr_mixed(to_dev(Y), b, prec=cqr.PREC_FP8)
    torch.cuda.synchronize()
    assert info == 0
    Qh, Rh = _host32(Q), _host32(R)
    assert np.array_equal(np.tril(Rh, -1), np.zeros_like(Rh))
    assert (np.diag(Rh) > 0).all()
    rec = np.linalg.norm(Y - Qh @ Rh) / np.linalg.norm(Y)
    orth = np.abs(Qh.T @ Qh - np.eye(n)).max()
    assert rec < 2 * U_FP8, rec
    assert orth < 4 * U_FP8, orth


@pytest.mark.parametrize("n,b", [(2048, 256), (1024, 64)])
def test_fp8_factor_against_oracle(n, b):
    """FP8 factors element by element against the oracle's FP64 factors.
    With E = Y - Q R and F = I - Q^T Q measured on the FP8 result, first-order
    QR perturbation theory (exact orthonormal factors of Y + E) bounds
    ||dQ||_F by sqrt(2) kappa_2(Y) ||E||_F / ||Y||_2, and the departure of Q
    from orthonormality adds at most ||F||_F; twice that sum allows for the
    second-order terms.  R is bounded the same way relative to ||Y||_2."""
    Y = inputs.diag_dominant(n, seed=n + 5)
    Q, R, info = cqr.qr_mixed(to_dev(Y), b, prec=cqr.PREC_FP8)
    torch.cuda.synchronize()
    assert info == 0
    Qh, Rh = _host32(Q), _host32(R)
    ref = oracle.cgs_qr(Y, b)
    n2 = np.linalg.norm(Y, 2)
    kappa = np.linalg.cond(Y)
    e = np.linalg.norm(Y - Qh @ Rh) / n2
    f = np.linalg.norm(Qh.T @ Qh - np.eye(n))
    assert e < 2 * U_FP8 and np.abs(Qh.T @ Qh - np.eye(n)).max() < 4 * U_FP8
    bound = 2 * (np.sqrt(2) * kappa * e + f)
    assert np.abs(Qh - ref["Q"]).max() < bound
    assert np.abs(Rh - ref["R"]).max() < bound * n2


@pytest.mark.parametrize("n,b", [(512, 64), (4096, 256)])
def test_fp8_ir_solve_reaches_fp64_residual(n, b):
    Y = inputs.diag_dominant(n, seed=17 + n)
    rhs = inputs.uniform_vector(n, seed=18 + n)
    Yd = to_dev(Y)
    Q, R, info = cqr.qr_mixed(Yd, b, prec=cqr.PREC_FP8)
    assert info == 0
    x, iters, res = cqr.solve_ir(Yd, Q, R, torch.from_numpy(rhs).cuda(), maxiter=50, tol=16.0)
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    assert res < 16 and 1 <= iters < 50
    assert hpl_ratio(Y, xh, rhs) < 16
    ref = oracle.cgs_qr(Y, 64)
    xo, rc = oracle.qr_solve(ref["Q"], ref["R"], rhs)
    assert rc == 0
    assert np.abs(xh - xo).max() < 16 * np.linalg.cond(Y) * n * EPS * np.abs(xo).max()


@pytest.mark.parametrize("prec", [cqr.PREC_BF16, cqr.PREC_FP8])
def test_large_factor_and_refinement_properties(prec):
    """n = 16384, b = 256: the later projections have at least 12288 rows of
    output and take the 256-row tile.  Properties that hold at any size (the
    oracle would take minutes): reconstruction and orthogonality within the
    precision's bounds, an exact upper triangle with a positive diagonal, and
    the refined solution under the FP64 HPL bar (residual recomputed here)."""
    n, b = 16384, 256
    u = U_BF16 if prec == cqr.PREC_BF16 else U_FP8
    Y = cqr.colmajor(n, n)
    cqr.synth_uniform(Y, 77, -0.5, 0.5)
    Y.diagonal().zero_()
    Y.diagonal().copy_(Y.abs().sum(dim=1) + 1.0)
    rhs = torch.empty(n, dtype=torch.float64, device="cuda")
    cqr.synth_uniform(rhs.view(n, 1), 78)
    Q, R, info = cqr.qr_mixed(Y, b, prec=prec)
    torch.cuda.synchronize()
    assert info == 0
    assert not torch.tril(R, -1).any()
    assert (R.diagonal() > 0).all()
    Qd, Rd = Q.double(), R.double()
    rec = float(torch.linalg.norm(Y - Qd @ Rd) / torch.linalg.norm(Y))
    assert rec < 2 * u, rec
    G = Qd.t().contiguous() @ Qd
    G.diagonal().sub_(1.0)
    orth = float(G.abs().max())
    assert orth < 4 * u, orth
    del Qd, Rd, G
    x, iters, res = cqr.solve_ir(Y, Q, R, rhs, maxiter=50, tol=16.0)
    assert res < 16 and iters <= 10, (res, iters)
    r = (Y @ x - rhs).abs().max()
    hpl = float(r / (Y.abs().sum(dim=1).max() * x.abs().max() * n * EPS))
    assert hpl < 16, hpl


@pytest.mark.parametrize("prec", [cqr.PREC_BF16, cqr.PREC_FP8])
@pytest.mark.parametrize("n,b", [(1024, 256), (512, 64)])
def test_mixed_permutation_bit_exact(prec, n, b):
    """Permutation input: 0/1 entries are exact in BF16 and FP8, every
    projection P^T Y_j is exactly 0 (a product that paired A and B entries of
    different k would make some 1) and every Gram exactly I, so Q = Y and
    R = I to the bit in both low-precision forms, wide and narrow tiles."""
    Y = np.asfortranarray(np.eye(n)[:, np.random.default_rng(n + b).permutation(n)])
    Q, R, info = cqr.qr_mixed(to_dev(Y), b, prec=prec)
    torch.cuda.synchronize()
    assert info == 0
    assert np.array_equal(_host32(Q), Y)
    assert np.array_equal(_host32(R), np.eye(n))


@pytest.mark.parametrize("prec", [cqr.PREC_BF16, cqr.PREC_FP8])
def test_c3_n65536_properties(prec):
    """The largest mixed-precision workload, n = 65536 (b = 256, Y 34 GB):
    size-independent checks only.  Freivalds probes of the reconstruction
    ||Y z - Q (R z)|| / (||Y||_F ||z||) for 4 Gaussian z, orthogonality of 64
    sampled columns of Q, the exact upper triangle with a positive diagonal
    (sampled rows), and the refined solution under the FP64 HPL bar with the
    residual recomputed here."""
    n, b = 65536, 256
    u = U_BF16 if prec == cqr.PREC_BF16 else U_FP8
    Y = cqr.colmajor(n, n)
    cqr.synth_uniform(Y, 91, -0.5, 0.5)
    Y.diagonal().zero_()
    rs = torch.zeros(n, dtype=torch.float64, device="cuda")
    for j in range(0, n, 4096):
        rs += Y[:, j:j + 4096].abs().sum(dim=1)
    Y.diagonal().copy_(rs + 1.0)
    rhs = torch.empty(n, dtype=torch.float64, device="cuda")
    cqr.synth_uniform(rhs.view(n, 1), 92)
    Q, R, info, flags = cqr.qr_mixed_async(Y, b, prec=prec)
    torch.cuda.synchronize()
    assert int(info[0]) == 0 and not flags.any()
    g = torch.Generator(device="cuda").manual_seed(93)
    Z = torch.randn(n, 4, dtype=torch.float64, device="cuda", generator=g)
    ynorm = float(torch.linalg.norm(Y))
    RZ = torch.zeros(n, 4, dtype=torch.float64, device="cuda")
    QRZ = torch.zeros(n, 4, dtype=torch.float64, device="cuda")
    for j in range(0, n, 8192):  # R Z and Q (R Z) in column slabs (FP64 accumulation)
        RZ += R[:, j:j + 8192].double() @ Z[j:j + 8192]
    for j in range(0, n, 8192):
        QRZ += Q[:, j:j + 8192].double() @ RZ[j:j + 8192]
    rec = float(torch.linalg.norm(Y @ Z - QRZ) / (ynorm * torch.linalg.norm(Z)))
    assert rec < 2 * u, rec
    cols = torch.from_numpy(np.sort(np.random.default_rng(94).choice(n, 64, replace=False))).cuda()
    Qc = Q[:, cols].double()
    G = Qc.t() @ Qc
    G.diagonal().sub_(1.0)
    assert float(G.abs().max()) < 4 * u
    rows = cols
    Rr = R[rows].double()
    jj = torch.arange(n, device="cuda")
    assert not (Rr * (jj[None, :] < rows[:, None])).any()
    assert (R.diagonal()[rows] > 0).all()
    del Qc, G, Rr, RZ, QRZ
    x, iters, res = cqr.solve_ir(Y, Q, R, rhs, maxiter=50, tol=16.0)
    assert res < 16 and iters <= 10, (res, iters)
    r = (Y @ x - rhs).abs().max()
    hpl = float(r / ((rs + Y.diagonal().abs()).max() * x.abs().max() * n * EPS))
    assert hpl < 16, hpl


@pytest.mark.parametrize("prec,n,b", [(cqr.PREC_BF16, 2048, 256), (cqr.PREC_BF16, 1000, 256),
                                      (cqr.PREC_FP8, 2048, 256), (cqr.PREC_FP8, 776, 128)])
def test_tiled_column_storage_is_bit_identical(prec, n, b):
    """The tiled storage of the finished low-precision columns changes only
    where the products read their operand from, not the order of any sum:
    Q, R and info are the same bits as with column-major storage (ragged
    sizes and block widths that are not multiples of the 128-column blocks
    included; block widths whose products all take the wide GEMM tile, as the
    tiled storage does)."""
    Yd = to_dev(inputs.diag_dominant(n, seed=71 + n))
    out = []
    try:
        for tiled in (False, True):
            cqr.set_mixed_layout(tiled)
            Q, R, info = cqr.qr_mixed(Yd, b, prec=prec)
            torch.cuda.synchronize()
            assert info == 0
            out.append((Q.clone(), R.clone()))
    finally:
        cqr.set_mixed_layout(True)
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
