"""Truncated SVD on the GPU (RandSVD, Algorithm 1; LancSVD, Algorithm 2; the
small SVD of S5/S6; the products with A; the sparse products and transpose)
through the C ABI, against the CPU oracle, LAPACK (numpy) and scipy.sparse.

Tolerances.  Every step of both drivers is backward stable in FP64, so the GPU
run and the oracle's run are exact runs for matrices within
||dA|| <= (number of steps) * m * eps * ||A||_2 of A; the singular values of
the two runs then differ by at most twice that (Weyl), and a singular vector
whose value is separated from the others by `gap` by at most that over gap
(Wedin's sin-theta bound), compared up to sign.  The small SVD is held to the
LAPACK bars 16 r eps ||B|| (values, reconstruction) and 16 r eps
(orthogonality); the products with A to the standard elementwise bound
K eps (|A| |X|); integer outputs (the transposed sparsity pattern) bit for
bit.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2403_06218_amd as cqr
from oracle import svd as osvd
from paper_2403_06218_amd import inputs, svd
from gpu_util import EPS, to_dev, to_host

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def _h(t):
    return to_host(t) if t.dim() == 2 else t.cpu().numpy()


def _graded_bidiagonal(r, b, seed):
    """A block lower bidiagonal r x r matrix (the shape of B_k) with singular
    values spread over 15 decades."""
    rng = np.random.default_rng(seed)
    B = np.zeros((r, r))
    for i in range(0, r, b):
        B[i:i + b, i:i + b] = np.tril(rng.standard_normal((b, b)))
        if i + b < r:
            B[i + b:i + 2 * b, i:i + b] = np.triu(rng.standard_normal((b, b)))
    U, _, Vt = np.linalg.svd(B)
    return (U * np.logspace(1, -14, r)) @ Vt


@pytest.mark.parametrize("r,kind", [(1, "u"), (2, "u"), (7, "u"), (64, "u"), (65, "u"), (128, "u"), (256, "u"),
                                    (64, "graded"), (256, "graded")])
def test_small_svd_matches_lapack(r, kind):
    B = inputs.uniform_matrix(r, r, seed=r) if kind == "u" else _graded_bidiagonal(r, 16, seed=r)
    U, s, V, sweeps = svd.small_svd(to_dev(B))
    Ug, sg, Vg = _h(U), _h(s), _h(V)
    ref = np.linalg.svd(B, compute_uv=False)
    nb = np.linalg.norm(B, 2)
    assert sweeps > 0 if r > 1 else sweeps == 0  # a 1 x 1 matrix needs no rotation
    assert (np.diff(sg) <= 0).all()
    np.testing.assert_allclose(sg, ref, rtol=0, atol=16 * r * EPS * nb)
    assert np.linalg.norm(B - (Ug * sg) @ Vg.T) <= 16 * r * EPS * np.linalg.norm(B)
    assert np.abs(Vg.T @ Vg - np.eye(r)).max() <= 16 * r * EPS
    keep = sg > 1e3 * r * EPS * nb  # columns of U are accurate where sigma is not at rounding level
    assert np.abs(Ug[:, keep].T @ Ug[:, keep] - np.eye(keep.sum())).max() <= 16 * r * EPS * nb / sg[keep].min()


@pytest.mark.parametrize("trans,M,N,K", [(True, 3000, 16, 200000), (False, 200000, 16, 3000), (True, 1000, 64, 50000),
                                         (False, 50000, 64, 1000), (True, 77, 16, 10000), (False, 1001, 13, 333)])
def test_products_with_A(trans, M, N, K):
    """C = A^T X and C = A X on the FP64 MFMA kernels (the skinny shapes of
    LancSVD's S2/S4 and RandSVD's S1/S3), elementwise within K eps |A||X|."""
    A = inputs.uniform_matrix(K, M, seed=M + K) if trans else inputs.uniform_matrix(M, K, seed=M + K)
    X = inputs.uniform_matrix(K, N, seed=N)
    C = svd.gemm(to_dev(A), to_dev(X), trans_a=trans)
    ref = (A.T @ X) if trans else (A @ X)
    bound = K * EPS * ((np.abs(A).T @ np.abs(X)) if trans else (np.abs(A) @ np.abs(X)))
    assert (np.abs(_h(C) - ref) <= bound).all()


def _weyl(nsteps, m, nA):
    return 2.0 * nsteps * m * EPS * nA


def _compare_triplets(Ug, sg, Vg, Uo, so, Vo, tol, idx):
    """Triplets idx of the GPU run against the oracle's: values within the
    Weyl bound, vectors (up to sign) within Wedin's bound where separated."""
    idx = list(idx)
    np.testing.assert_allclose(sg[idx], so[idx], rtol=0, atol=tol)
    for j in idx:
        gap = min([abs(so[j] - so[i]) for i in range(len(so)) if i != j] + [so[j]])
        if gap < 1e3 * tol:
            continue
        bound = 2.0 * tol / gap
        for G, O in ((Ug, Uo), (Vg, Vo)):
            d = min(np.abs(G[:, j] - O[:, j]).max(), np.abs(G[:, j] + O[:, j]).max())
            assert d <= bound, (j, d, bound)


def _check_rayleigh_ritz(A, Ug, sg, Vg, r):
    """Properties of any correct Rayleigh-Ritz output, converged or not:
    U and V orthonormal and U^T A V = diag(sigma) (the bases are exact
    projections, P_k-bar^T A P_k = B_k), each to a small multiple of r eps
    (||A||).  The oracle's own runs stay below 5 r eps."""
    nA = sg[0]
    assert np.abs(Ug.T @ Ug - np.eye(r)).max() <= 64 * r * EPS
    assert np.abs(Vg.T @ Vg - np.eye(r)).max() <= 64 * r * EPS
    assert np.abs(Ug.T @ (A @ Vg) - np.diag(sg)).max() <= 64 * r * EPS * nA


def _converged(A, ref, thresh=1e-8):
    """Indices of the oracle's triplets whose residual is below thresh: only
    these are determined by A and the start block; the unconverged Ritz
    values of a Krylov run on a graded spectrum depend on rounding (two
    correct runs agree on them only loosely)."""
    res = osvd.residuals(A, ref["U"], ref["sigma"], ref["V"])
    return np.nonzero(res < thresh)[0], res


@pytest.mark.parametrize("p", [1, 3])
def test_lancsvd_matches_oracle(p):
    """The paper's dense test matrix (Sec. 4) scaled down: m = 4000, n = 400,
    b = 16, r = 64."""
    m, n, r, b = 4000, 400, 64, 16
    A, sig = inputs.svd_test_matrix(m, n, seed=5)
    Q1 = inputs.normal_matrix(m, b, seed=6)
    U, s, V, info = svd.lancsvd(to_dev(A), r, b, p, to_dev(Q1))
    Ug, sg, Vg = _h(U), _h(s), _h(V)
    ref = osvd.lancsvd(A, r, p, b, Q1)
    assert info == sum(1 for c in ref["codes"] if c != 0) == 0
    k = r // b
    tol = _weyl(p * (4 * k + 2) + 2, m, sig[0])
    conv, ref_res = _converged(A, ref)
    assert len(conv) >= 10 and (conv[:10] == np.arange(10)).all()
    _compare_triplets(Ug, sg, Vg, ref["U"], ref["sigma"], ref["V"], tol, conv)
    _check_rayleigh_ritz(A, Ug, sg, Vg, r)
    # The 10 leading values reach rounding level (constructed spectrum) and
    # their residuals follow the oracle's.
    assert np.abs(sg[:10] - sig[:10]).max() < 1e-13 * sig[0]
    res = _h(svd.residuals(to_dev(A), U, s, V, 10))
    np.testing.assert_allclose(res, osvd.residuals(A, Ug, sg, Vg, 10), rtol=1e-6, atol=1e-15)
    np.testing.assert_allclose(res, ref_res[:10], rtol=1e-2, atol=1e-13)
    assert res.max() < (1e-12 if p > 1 else 1e-10)


def test_randsvd_matches_oracle():
    m, n, r, b, p = 4000, 400, 64, 16, 2
    A, sig = inputs.svd_test_matrix(m, n, seed=7)
    Q0 = inputs.normal_matrix(n, r, seed=8)
    U, s, V, info = svd.randsvd(to_dev(A), r, b, p, to_dev(Q0))
    Ug, sg, Vg = _h(U), _h(s), _h(V)
    Uo, so, Vo, infos = osvd.randsvd(A, r, p, b, Q0)
    assert info == sum(1 for c in infos if c != 0) == 0
    tol = _weyl(p * 4 + 3, m, sig[0])
    _compare_triplets(Ug, sg, Vg, Uo, so, Vo, tol, range(r))


def test_lancsvd_tall_paper_shape():
    """m = 1e5 x n = 1e3 (the paper's m/n aspect, n scaled down), b = 16,
    r = 64, p = 2: against the constructed singular values and the oracle's."""
    m, n, r, b, p = 100000, 1000, 64, 16, 2
    A, sig = inputs.svd_test_matrix(m, n, seed=9)
    Q1 = inputs.normal_matrix(m, b, seed=10)
    Ad = to_dev(A)
    U, s, V, info = svd.lancsvd(Ad, r, b, p, to_dev(Q1))
    Ug, sg, Vg = _h(U), _h(s), _h(V)
    ref = osvd.lancsvd(A, r, p, b, Q1)
    assert info == 0
    conv, _ = _converged(A, ref)
    assert len(conv) >= 10
    _compare_triplets(Ug, sg, Vg, ref["U"], ref["sigma"], ref["V"], _weyl(p * 18 + 2, m, sig[0]), conv)
    _check_rayleigh_ritz(A, Ug, sg, Vg, r)
    assert np.abs(sg[:10] - sig[:10]).max() < 1e-13 * sig[0]


def _sparse(m, n, nnz, seed):
    rowptr, col, val = inputs.sparse_matrix(m, n, nnz, seed)
    import scipy.sparse as sp
    S = sp.csr_matrix((val, col, rowptr), shape=(m, n))
    return S, svd.Csr(m, n, rowptr, col, val)


def test_csr_transpose_is_exact():
    S, G = _sparse(5000, 3000, 60000, seed=11)
    T = S.T.tocsr()
    T.sort_indices()
    torch.cuda.synchronize()
    assert np.array_equal(G.trowptr.cpu().numpy(), T.indptr.astype(np.int32))
    assert np.array_equal(G.tcol[:G.nnz].cpu().numpy(), T.indices.astype(np.int32))
    assert np.array_equal(G.tval[:G.nnz].cpu().numpy(), T.data)


@pytest.mark.parametrize("w", [1, 16, 20, 64, 100])
@pytest.mark.parametrize("trans", [False, True])
def test_spmm_matches_scipy(w, trans):
    S, G = _sparse(5000, 3000, 60000, seed=12)
    inner = 5000 if trans else 3000
    X = inputs.uniform_matrix(inner, w, seed=w)
    C = _h(G.spmm(to_dev(X), trans=trans))
    M = S.T if trans else S
    ref = M @ X
    absM = abs(M)
    nz = np.diff(M.tocsr().indptr).max()
    assert (np.abs(C - ref) <= nz * EPS * (absM @ np.abs(X))).all()
    C2 = _h(G.spmm(to_dev(X), trans=trans))
    assert np.array_equal(C, C2)  # reproducible bit for bit


def test_lancsvd_and_randsvd_csr_match_oracle():
    """Sparse A (synthetic, heavy-tailed row lengths): both drivers against
    the oracle run on the dense copy of A."""
    m, n = 6000, 2000
    S, G = _sparse(m, n, 40000, seed=13)
    A = S.toarray()
    nA = np.linalg.norm(A, 2)
    r, b = 32, 16
    Q1 = inputs.normal_matrix(m, b, seed=14)
    U, s, V, info = svd.lancsvd(G, r, b, 2, to_dev(Q1))
    ref = osvd.lancsvd(A, r, 2, b, Q1)
    assert info == 0
    np.testing.assert_allclose(_h(s), ref["sigma"], rtol=0, atol=_weyl(2 * 10 + 2, m, nA))
    Q0 = inputs.normal_matrix(n, r, seed=15)
    U, s, V, info = svd.randsvd(G, r, b, 3, to_dev(Q0))
    Uo, so, Vo, _ = osvd.randsvd(A, r, 3, b, Q0)
    assert info == 0
    np.testing.assert_allclose(_h(s), so, rtol=0, atol=_weyl(3 * 4 + 3, m, nA))


def test_paper_dense_shape_matches_stored_oracle():
    """The paper's dense experiment at full size, m = 1e5, n = 1e4 (Sec. 4:
    b = 16, r = 64 for LancSVD, r = 16 for RandSVD, p in {1, 4}): sigma_1..10
    and the residuals of the 10 leading triplets against the oracle's, stored
    in tests/golden/lancsvd_dense_m100000_n10000.json by
    tests/golden/make_lancsvd_dense.py (the oracle takes minutes there).  A is
    built on the GPU from the same random ingredients (the same matrix up to
    rounding), so values agree to 1e-9 relative and residuals to 1e-6
    relative (they are differences of nearly equal vectors)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "lancsvd_dense_m100000_n10000.json")))
    m, n, seed = gold["m"], gold["n"], gold["seed"]
    A, sig = inputs.svd_test_matrix_device(m, n, seed)
    np.testing.assert_allclose(sig[:10], gold["sigma_exact_1_10"], rtol=1e-15)
    for name, run in gold["runs"].items():
        rows = m if name.startswith("lanc") else n
        width = run["b"] if name.startswith("lanc") else run["r"]
        Q1 = torch.from_numpy(np.ascontiguousarray(inputs.normal_matrix(rows, width, seed + 1).T)).cuda().t()
        fn = svd.lancsvd if name.startswith("lanc") else svd.randsvd
        U, s, V, info = fn(A, run["r"], run["b"], run["p"], Q1)
        assert info == 0, name
        sg = s.cpu().numpy()
        res = svd.residuals(A, U, s, V, 10).cpu().numpy()
        np.testing.assert_allclose(sg[:10], run["sigma_1_10"], rtol=1e-9, err_msg=name)
        np.testing.assert_allclose(res, run["residual_1_10"], rtol=1e-6, err_msg=name)
        del U, s, V
