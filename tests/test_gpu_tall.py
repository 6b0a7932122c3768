"""Narrow blocks of tall matrices (q >= 16384 rows, block width <= 16, at most
128 earlier columns): the row-streaming form of Algorithms 4 and 5, against
the CPU oracle.  Bars as in the parity tests: |dQ| <= 8 kappa q eps,
|dR| <= 8 kappa q eps ||Y||_2, backward-error ratios < 16, info and per-block
flags exact.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2403_06218_amd as cqr
from paper_2403_06218_amd import inputs
from gpu_util import EPS, orth_ratio, recon_ratio, to_dev, to_host

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def _check(Y, b, ld=None):
    Yd = to_dev(Y, ld)
    Q, R, info, flags = cqr.qr(Yd, b)
    torch.cuda.synchronize()
    Qg, Rg = to_host(Q), to_host(R)
    ref = oracle.cgs_qr(Y, b)
    q = Y.shape[0]
    kappa = np.linalg.cond(Y)
    tol = 8 * kappa * q * EPS
    assert info == ref["info"]
    assert list(flags) == list(ref["block_flags"])
    np.testing.assert_allclose(Qg, ref["Q"], rtol=0, atol=tol)
    np.testing.assert_allclose(Rg, ref["R"], rtol=0, atol=tol * np.linalg.norm(Y, 2))
    assert np.array_equal(np.tril(Rg, -1), np.zeros_like(Rg))
    assert recon_ratio(Y, Qg, Rg) < 16
    assert orth_ratio(Qg) < 16
    return Qg, Rg


@pytest.mark.parametrize("q,r,b", [(20000, 64, 16), (16384, 56, 16), (17001, 40, 8), (30000, 16, 16),
                                   (20000, 37, 12), (16500, 160, 16)])
def test_tall_shapes_against_oracle(q, r, b):
    """Ragged last blocks, widths below 16, row counts off the tile grid, and
    (r = 160) bases past 128 columns, where the last blocks take the GEMM path."""
    Y = inputs.normal_matrix(q, r, seed=q + r + b)
    _check(Y, b)


def test_tall_padded_leading_dimension():
    Y = inputs.uniform_matrix(18000, 48, seed=5)
    _check(Y, 16, ld=18007)


def test_tall_fallback_block():
    """A block whose columns are nearly dependent on earlier ones breaks the
    Cholesky factorisation: the same fallback and flags as the oracle."""
    q, w = 20000, 16
    Y = inputs.uniform_matrix(q, 3 * w, seed=11)
    i, j = np.arange(q), np.arange(w)
    Y[:, w:2 * w] = 1.0 / (i[:, None] + j[None, :] + 1.0)
    Yd = to_dev(Y)
    Q, R, info, flags = cqr.qr(Yd, w)
    torch.cuda.synchronize()
    ref = oracle.cgs_qr(Y, w)
    assert info == ref["info"] == 2
    assert list(flags) == list(ref["block_flags"])
    Qg, Rg = to_host(Q), to_host(R)
    assert np.linalg.norm(Y - Qg @ Rg) < 1e-13 * np.linalg.norm(Y)
    assert orth_ratio(Qg) < 16


def test_tall_orth_against():
    """Algorithm 5 alone on a tall block: Q_in = P H + Q R, P^T Q = 0."""
    q = 25000
    Y = inputs.normal_matrix(q, 64, seed=6)
    P, _ = np.linalg.qr(Y[:, :48])
    Qin = Y[:, 48:]
    Qd, Hd, Rd, info = cqr.orth_against(to_dev(Qin), to_dev(P))
    torch.cuda.synchronize()
    Qo, Ho, Ro, rc = oracle.cgs_cqr2(Qin, P)
    assert info == 0 and rc == 0
    kappa = np.linalg.cond(np.hstack([P, Qin]))
    tol = 8 * kappa * q * EPS
    np.testing.assert_allclose(to_host(Qd), Qo, rtol=0, atol=tol)
    np.testing.assert_allclose(to_host(Hd), Ho, rtol=0, atol=tol * np.linalg.norm(Qin, 2))
    np.testing.assert_allclose(to_host(Rd), Ro, rtol=0, atol=tol * np.linalg.norm(Qin, 2))


def test_tall_repeated_runs_bit_identical():
    Y = inputs.normal_matrix(40000, 64, seed=7)
    Q1, R1, _, _ = cqr.qr(to_dev(Y), 16)
    Q2, R2, _, _ = cqr.qr(to_dev(Y), 16)
    torch.cuda.synchronize()
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2)
