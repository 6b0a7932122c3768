"""Pins of the truncated-SVD oracle (RandSVD, Algorithm 1; LancSVD,
Algorithm 2) against what the mathematics fixes, independent of the oracle's
own code: singular values known by construction (the paper's dense test
matrices, Sec. 4), LAPACK's full SVD when the subspace is the whole space,
the block Golub-Kahan-Lanczos relations of Sec. 2.2, orthonormality, and the
printed-vs-corrected reading of S8."""
import numpy as np
import pytest

import oracle
from oracle import svd
from paper_2403_06218_amd import inputs

EPS = 2.0 ** -52


def _start(rows, cols, seed):
    return inputs.normal_matrix(rows, cols, seed)


def test_dense_test_matrix_has_the_constructed_singular_values():
    A, sig = inputs.svd_test_matrix(2000, 200, seed=3)
    s = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(s[:100], sig[:100], rtol=1e-12, atol=1e-13)
    assert sig[0] == 10.0 and sig[99] == pytest.approx(10.0 ** (15 / 100 - 14)) and sig[-1] == 1e-14


@pytest.mark.parametrize("n,b", [(32, 4), (48, 8)])
def test_lancsvd_full_subspace_is_the_exact_svd(n, b):
    """Square A with r = n: both Krylov bases span the whole space, the
    remainder Qbar_{k+1} R_k is rounding noise, and B_k carries all singular
    values of A (brute force against LAPACK's SVD)."""
    m = n
    A = inputs.uniform_matrix(m, n, seed=m + n)
    out = svd.lancsvd(A, n, 1, b, _start(m, b, 1))
    s = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(out["sigma"], s, rtol=0, atol=1e3 * EPS * s[0])
    U, V = out["U"], out["V"]
    np.testing.assert_allclose(A @ V, U * out["sigma"], atol=1e4 * EPS * s[0])


def test_randsvd_full_subspace_is_the_exact_svd():
    m, n, b = 70, 40, 8
    A = inputs.uniform_matrix(m, n, seed=5)
    U, s, V, infos = svd.randsvd(A, n, 1, b, _start(n, n, 2))
    ref = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(s, ref, rtol=0, atol=1e3 * EPS * ref[0])
    np.testing.assert_allclose(A @ V, U * s, atol=1e4 * EPS * ref[0])
    np.testing.assert_allclose(U.T @ U, np.eye(n), atol=1e3 * EPS)


def test_lancsvd_relations_of_the_block_bidiagonalisation():
    """After one restart cycle (p = 1): A P_k = Pbar_k B_k + Qbar_{k+1} R_k E_k^T,
    A^T Pbar_k = P_k B_k^T, orthonormal bases, Pbar_k^T Qbar_{k+1} = 0 (the
    readings of the relations printed garbled in Sec. 2.2), and B_k lower
    triangular with b diagonals below the main one."""
    m, n, r, b = 400, 120, 48, 8
    A = inputs.uniform_matrix(m, n, 9)
    out = svd.lancsvd(A, r, 1, b, _start(m, b, 4), keep_last=True)
    P, Pb, Qn, Rk, B = out["P"], out["Pbar"], out["Qnext"], out["Rk"], out["B"]
    nA = np.linalg.norm(A, 2)
    Ek = np.zeros((r, b))
    Ek[-b:, :] = np.eye(b)
    np.testing.assert_allclose(A @ P, Pb @ B + Qn @ Rk @ Ek.T, atol=1e3 * EPS * nA)
    np.testing.assert_allclose(A.T @ Pb, P @ B.T, atol=1e3 * EPS * nA)
    np.testing.assert_allclose(P.T @ P, np.eye(r), atol=1e3 * EPS)
    np.testing.assert_allclose(Pb.T @ Pb, np.eye(r), atol=1e3 * EPS)
    assert np.abs(Pb.T @ Qn).max() < 1e3 * EPS
    assert np.array_equal(np.triu(B, 1), np.zeros_like(B))
    assert np.array_equal(np.tril(B, -(b + 1)), np.zeros_like(B))


def test_lancsvd_converges_to_the_constructed_singular_values():
    """The paper's dense experiment scaled down (m = 3000, n = 300, b = 16,
    r = 64, the 10 largest triplets).  At this n the constructed spectrum
    decays by 10^(-15/150) per index, so one cycle already reaches rounding
    accuracy; p = 4 restarts keep it there."""
    m, n, r, b = 3000, 300, 64, 16
    A, sig = inputs.svd_test_matrix(m, n, seed=11)
    start = _start(m, b, 12)
    for p in (1, 4):
        out = svd.lancsvd(A, r, p, b, start)
        err = np.abs(out["sigma"][:10] - sig[:10]).max() / sig[0]
        res = svd.residuals(A, out["U"], out["sigma"], out["V"], 10)
        assert err < 1e-13 and res.max() < 1e-12, (p, err, res)


def _clustered(m, n, seed):
    rng = np.random.default_rng(seed)
    X, _ = np.linalg.qr(rng.standard_normal((m, n)))
    Y, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sig = np.linspace(1.0, 0.2, n)
    return (X * sig) @ Y.T, sig


def test_restarts_improve_a_clustered_spectrum():
    """Clustered singular values (1 down to 0.2, evenly spaced): each restart
    of LancSVD and each subspace iteration of RandSVD reduces the error of the
    leading values (the roles of p in Sec. 2), and for the same number of
    products with A LancSVD is the more accurate (Sec. 4, dense problems)."""
    m, n = 2000, 200
    A, sig = _clustered(m, n, 1)
    start = _start(m, 8, 12)
    le = [np.abs(svd.lancsvd(A, 32, p, 8, start)["sigma"][:8] - sig[:8]).max() for p in (1, 2, 4, 8)]
    assert le[0] > le[1] > le[2] > le[3] and le[3] < 1e-4, le
    Q0 = _start(n, 16, 3)
    re = [np.abs(svd.randsvd(A, 16, p, 8, Q0)[1][:8] - sig[:8]).max() for p in (1, 4, 16)]
    assert re[0] > re[1] > re[2], re
    # The same number of products with A (32; LancSVD's are half as wide):
    # LancSVD p = 4 is more accurate than RandSVD p = 16.
    assert le[2] < re[2]


def test_S8_S9_reading_satisfies_the_adjoint_relation():
    """With U = Pbar_k Ubar (S9) and V = P_k Vbar (the reading of S8),
    A^T U = V Sigma holds to rounding for every triplet, at any p (from
    A^T Pbar_k = P_k B_k^T).  S8 as printed (P_k Vbar^T) violates it."""
    m, n = 2000, 200
    A, sig = _clustered(m, n, 2)
    out = svd.lancsvd(A, 32, 1, 8, _start(m, 8, 16), keep_last=True)
    U, s, V = out["U"], out["sigma"], out["V"]
    nA = np.linalg.norm(A, 2)
    assert np.abs(A.T @ U - V * s).max() < 1e3 * EPS * nA
    Vbt = np.linalg.svd(out["B"])[2]
    printed = out["P"] @ Vbt
    assert np.abs(A.T @ U - printed * s).max() > 1e-2 * nA


def test_orth_against_fallback_matches_cgs2():
    """Algorithm 5 with its fallback: a block whose Gram matrix breaks the
    Cholesky factorisation is redone by CGS2 and still satisfies the output
    contract Q_in = P H + Q R, P^T Q = 0, Q^T Q = I."""
    rng = np.random.default_rng(3)
    P, _ = np.linalg.qr(rng.standard_normal((200, 10)))
    U, _ = np.linalg.qr(rng.standard_normal((200, 12)))
    Qin = (U * np.logspace(0, -10, 12)) @ np.linalg.qr(rng.standard_normal((12, 12)))[0]
    Q, H, R, rc = oracle.orth_against_fb(Qin, P)
    assert rc == 1
    assert np.linalg.norm(Qin - P @ H - Q @ R) < 1e-14 * np.linalg.norm(Qin)
    assert np.abs(P.T @ Q).max() < 1e-14 and np.abs(Q.T @ Q - np.eye(12)).max() < 1e-13
    assert np.array_equal(np.tril(R, -1), np.zeros_like(R))
    Q2, H2, R2, rc2 = oracle.orth_against_fb(U, P)
    assert rc2 == 0
