"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

The oracle (``oracle/``) is checked here against things other than itself:
hand-worked factorizations, exact special cases, LAPACK (through numpy) on
random inputs, numpy's LU-based determinant, a textbook CGS2 written from its
definition, the loop invariants of Algorithm 3, and backward-error bounds.
None of these tests touch a GPU.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2403_06218_amd import inputs

EPS = 2.0 ** -52
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    """Parse a golden fixture: '# ' comment lines, then 'KEY' blocks of rows."""
    blocks, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.isalpha() and line.isupper():
                cur = line
                blocks[cur] = []
            else:
                blocks[cur].append([float(eval(t, {"sqrt": math.sqrt})) for t in line.split()])
    return {k: np.array(v) for k, v in blocks.items()}


def _recon(Y, Q, R):
    return np.linalg.norm(Y - Q @ R) / (Y.shape[0] * EPS * np.linalg.norm(Y))


def _orth(Q):
    return np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])) / (Q.shape[0] * EPS)


def _lapack_qr(Y):
    """Thin QR from LAPACK (numpy), sign-normalised so that diag(R) >= 0."""
    Q, R = np.linalg.qr(Y)
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * s, (R.T * s).T


# --------------------------------------------------------------------------
# Hand-worked cases (tests/golden/*.txt, derivations in the fixture headers)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["qr_2x2.txt", "qr_3x3.txt"])
def test_hand_worked_cases(name):
    g = _read_golden(name)
    Y, Qx, Rx = g["Y"], g["Q"], g["R"]
    n = Y.shape[1]
    Qd, Rd = oracle.householder_qr(Y)
    np.testing.assert_allclose(Qd, Qx, atol=4 * EPS * n)
    np.testing.assert_allclose(Rd, Rx, atol=4 * EPS * n * 4)
    for b in range(1, n + 1):
        out = oracle.cgs_qr(Y, b, check_invariants=True)
        np.testing.assert_allclose(out["Q"], Qx, atol=8 * EPS * n)
        np.testing.assert_allclose(out["R"], Rx, atol=8 * EPS * n * 4)
        assert out["info"] == 0
        # |det Y| equals the product of the diagonal of R (fixture's DET line).
        assert abs(np.prod(np.diag(out["R"])) - g["DET"][0, 0]) < 1e-13


# --------------------------------------------------------------------------
# Exact special cases
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,b", [(7, 3), (16, 4), (33, 8), (64, 64)])
def test_permutation_is_bit_exact(n, b):
    """A permutation matrix is orthogonal: Q = Y and R = I with no rounding at all
    (every Gram is exactly I, every projection exactly 0, chol(I) = I)."""
    rng = np.random.default_rng(n)
    Y = np.eye(n)[:, rng.permutation(n)]
    out = oracle.cgs_qr(Y, b)
    assert np.array_equal(out["Q"], Y)
    assert np.array_equal(out["R"], np.eye(n))
    Qd, Rd = oracle.householder_qr(Y)
    np.testing.assert_allclose(Qd, Y, atol=1e-15)
    np.testing.assert_allclose(Rd, np.eye(n), atol=1e-15)


@pytest.mark.parametrize("b", [1, 2, 5])
def test_diagonal_small_integers_bit_exact(b):
    """Y = D (integer entries, any signs): Q = sign(D), R = |D| exactly."""
    d = np.array([3.0, -5.0, 2.0, -1.0, 7.0, 4.0, -6.0])
    Y = np.diag(d)
    out = oracle.cgs_qr(Y, b)
    assert np.array_equal(out["Q"], np.diag(np.sign(d)))
    assert np.array_equal(out["R"], np.diag(np.abs(d)))


@pytest.mark.parametrize("n,b", [(12, 4), (20, 7)])
def test_upper_triangular_positive_diag(n, b):
    """Y upper triangular with diag > 0 is already its own R: Q = I[:, :n]."""
    rng = np.random.default_rng(3)
    Y = np.triu(rng.uniform(-1, 1, (n, n))) + 2.0 * np.eye(n)
    out = oracle.cgs_qr(Y, b)
    np.testing.assert_allclose(out["Q"], np.eye(n), atol=64 * EPS)
    np.testing.assert_allclose(out["R"], Y, atol=64 * EPS * np.abs(Y).max())


@pytest.mark.parametrize("n,b", [(16, 4), (32, 32), (64, 16)])
def test_hadamard_orthonormal(n, b):
    """A normalised Hadamard matrix is orthogonal: Q = Y, R = I to rounding,
    and |det Y| = 1 = prod r_ii."""
    H = np.array([[1.0]])
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    Y = H / math.sqrt(n)
    out = oracle.cgs_qr(Y, b)
    np.testing.assert_allclose(out["Q"], Y, atol=16 * n * EPS)
    np.testing.assert_allclose(out["R"], np.eye(n), atol=16 * n * EPS)
    assert abs(np.sum(np.log(np.diag(out["R"])))) < 16 * n * EPS


def test_power_of_two_column_scaling_is_exact():
    """Y D with D a positive power-of-two diagonal factors as (Q, R D) bit for bit."""
    Y = inputs.uniform_matrix(40, 24, seed=11)
    D = 2.0 ** np.array([(-1) ** j * (j % 5) for j in range(24)], dtype=float)
    a = oracle.cgs_qr(Y, 8)
    c = oracle.cgs_qr(Y * D, 8)
    assert np.array_equal(c["Q"], a["Q"])
    assert np.array_equal(c["R"], a["R"] * D)


def test_row_permutation_invariance():
    """U Y with U a permutation factors as (U Q, R) up to rounding."""
    Y = inputs.uniform_matrix(50, 30, seed=12)
    perm = np.random.default_rng(0).permutation(50)
    a = oracle.cgs_qr(Y, 8)
    c = oracle.cgs_qr(Y[perm], 8)
    np.testing.assert_allclose(c["Q"], a["Q"][perm], atol=1e-12)
    np.testing.assert_allclose(c["R"], a["R"], atol=1e-12)


# --------------------------------------------------------------------------
# Independent routines: LAPACK, LU determinant, textbook CGS2
# --------------------------------------------------------------------------

@pytest.mark.parametrize("q,r,seed", [(30, 30, 0), (64, 40, 1), (100, 17, 2)])
def test_householder_matches_lapack(q, r, seed):
    Y = inputs.uniform_matrix(q, r, seed)
    Qd, Rd = oracle.householder_qr(Y)
    Ql, Rl = _lapack_qr(Y)
    kappa = np.linalg.cond(Y)
    tol = 64 * kappa * q * EPS
    np.testing.assert_allclose(Qd, Ql, atol=tol)
    np.testing.assert_allclose(Rd, Rl, atol=tol * np.abs(Rl).max())


@pytest.mark.parametrize("n,b,seed", [(48, 8, 0), (96, 32, 1), (128, 24, 2), (128, 128, 3)])
def test_cgs_qr_matches_lapack_and_householder(n, b, seed):
    """Thin QR with diag(R) > 0 is unique: Algorithm 3 must reach the same factors
    as Householder QR (oracle and LAPACK) within kappa * n * eps."""
    Y = inputs.uniform_matrix(n, n, seed)
    out = oracle.cgs_qr(Y, b)
    Qd, Rd = oracle.householder_qr(Y)
    Ql, Rl = _lapack_qr(Y)
    kappa = np.linalg.cond(Y)
    tol = 64 * kappa * n * EPS
    for Qx, Rx in ((Qd, Rd), (Ql, Rl)):
        np.testing.assert_allclose(out["Q"], Qx, atol=tol)
        np.testing.assert_allclose(out["R"], Rx, atol=tol * np.abs(Rx).max())
    assert out["info"] == 0 and not out["block_flags"].any()


@pytest.mark.parametrize("n,seed", [(20, 0), (64, 1), (200, 2)])
def test_det_equals_prod_diag(n, seed):
    """|det Y| = prod r_ii, compared as log sums with numpy's LU slogdet."""
    Y = inputs.uniform_matrix(n, n, seed)
    out = oracle.cgs_qr(Y, 8)
    sign, logdet = np.linalg.slogdet(Y)
    assert sign != 0
    assert abs(np.sum(np.log(np.diag(out["R"]))) - logdet) < 1e-9 * max(1.0, abs(logdet))


def _textbook_cgs2(Y):
    """Classical Gram-Schmidt, each column projected twice (Giraud et al. 2005):
    v = y - Q Q^T y; v = v - Q Q^T v; r = both projections, r_jj = ||v||."""
    q, r = Y.shape
    Q = np.zeros((q, r))
    R = np.zeros((r, r))
    for j in range(r):
        v = Y[:, j].copy()
        h1 = Q[:, :j].T @ v
        v = v - Q[:, :j] @ h1
        n1 = np.linalg.norm(v)
        v = v / n1
        h2 = Q[:, :j].T @ v
        v = v - Q[:, :j] @ h2
        n2 = np.linalg.norm(v)
        Q[:, j] = v / n2
        R[:j, j] = h1 + h2 * n1
        R[j, j] = n1 * n2
    return Q, R


@pytest.mark.parametrize("q,r,seed", [(40, 40, 4), (90, 33, 5)])
def test_block_width_one_is_cgs2(q, r, seed):
    """With b = 1, Algorithm 3 reduces to classical Gram-Schmidt with
    re-orthogonalisation, column by column."""
    Y = inputs.uniform_matrix(q, r, seed)
    out = oracle.cgs_qr(Y, 1)
    Qc, Rc = _textbook_cgs2(Y)
    np.testing.assert_allclose(out["Q"], Qc, atol=1e-13)
    np.testing.assert_allclose(out["R"], Rc, atol=1e-13)


# --------------------------------------------------------------------------
# Brute force on tiny integer inputs + loop invariants I1..I4
# --------------------------------------------------------------------------

def test_brute_force_tiny_integer_inputs():
    rng = np.random.default_rng(2024)
    checked = 0
    while checked < 300:
        q = int(rng.integers(1, 7))
        r = int(rng.integers(1, q + 1))
        Y = rng.integers(-3, 4, size=(q, r)).astype(float)
        if np.linalg.matrix_rank(Y) < r or np.linalg.cond(Y) > 1e3:
            continue
        Ql, Rl = _lapack_qr(Y)
        Qd, Rd = oracle.householder_qr(Y)
        np.testing.assert_allclose(Qd, Ql, atol=1e-12)
        np.testing.assert_allclose(Rd, Rl, atol=1e-12)
        for b in range(1, r + 1):
            out = oracle.cgs_qr(Y, b, check_invariants=True)
            np.testing.assert_allclose(out["Q"], Ql, atol=1e-11)
            np.testing.assert_allclose(out["R"], Rl, atol=1e-11)
            i1, i2, i3, i4 = out["inv"]
            assert i1 < 16 and i2 < 16 and i3 == 0 and i4 == 0
        checked += 1


@pytest.mark.parametrize("q,r,b,seed", [(64, 64, 8, 0), (64, 50, 16, 1), (60, 45, 7, 2), (33, 33, 32, 3)])
def test_loop_invariants_every_block(q, r, b, seed):
    """After every column block: I1 orthogonality, I2 reconstruction of the
    finished columns, I3 R upper triangular with diag >= 0, I4 later columns
    untouched (bit for bit)."""
    Y = inputs.uniform_matrix(q, r, seed)
    out = oracle.cgs_qr(Y, b, check_invariants=True)
    i1, i2, i3, i4 = out["inv"]
    assert i1 < 16, i1
    assert i2 < 16, i2
    assert i3 == 0 and i4 == 0


def _clean_partial(q=24, r=20, b=4, blocks=3, seed=5):
    """A factorization stopped after `blocks` column blocks of Algorithm 3:
    the first J = blocks*b columns of Q and R finished, the rest of Q still Y."""
    Y = inputs.uniform_matrix(q, r, seed)
    J = blocks * b
    out = oracle.cgs_qr(Y[:, :J], b)
    Q = Y.copy(order="F")
    Q[:, :J] = out["Q"]
    R = np.zeros((r, r), order="F")
    R[:J, :J] = out["R"]
    return Y, Q, R, J


def test_invariant_check_clean_partial_factorization():
    Y, Q, R, J = _clean_partial()
    i1, i2, i3, i4 = oracle.check_invariants(Y, Q, R, J)
    assert i1 < 16 and i2 < 16 and i3 == 0 and i4 == 0


def test_invariant_check_detects_planted_error():
    """Each invariant fires on a violation planted (on the CPU) in an otherwise
    clean partial factorization, and only that one: I1 a non-orthogonal
    column, I2 a Q R that misses Y, I3 a sub-diagonal entry or a negative
    diagonal of R, I4 one flipped bit in a column not yet reached."""
    Y, Q, R, J = _clean_partial()
    # I1: column 1 of Q and row 1 of R rescaled together (Q R unchanged).
    Q1, R1 = Q.copy(order="F"), R.copy(order="F")
    Q1[:, 1] *= 1.0 + 1e-9
    R1[1, :] /= 1.0 + 1e-9
    inv = oracle.check_invariants(Y, Q1, R1, J)
    assert inv[0] > 1e3 and inv[1] < 16 and inv[2] == 0 and inv[3] == 0, inv
    # I2: one off-diagonal entry of R moved (Q still orthonormal).
    R2 = R.copy(order="F")
    R2[2, J - 1] += 1e-9
    inv = oracle.check_invariants(Y, Q, R2, J)
    assert inv[0] < 16 and inv[1] > 1e3 and inv[2] == 0 and inv[3] == 0, inv
    # I3: a tiny nonzero below the diagonal (Q R moves by far less than eps).
    R3 = R.copy(order="F")
    R3[J - 1, 2] = 1e-300
    inv = oracle.check_invariants(Y, Q, R3, J)
    assert inv[0] < 16 and inv[1] < 16 and inv[2] == 1 and inv[3] == 0, inv
    # I3: a negative diagonal entry, with the Q column negated (Q R unchanged).
    Q4, R4 = Q.copy(order="F"), R.copy(order="F")
    Q4[:, 3] = -Q4[:, 3]
    R4[3, :] = -R4[3, :]
    inv = oracle.check_invariants(Y, Q4, R4, J)
    assert inv[0] < 16 and inv[1] < 16 and inv[2] == 1 and inv[3] == 0, inv
    # I4: the lowest bit of one entry of a later column flipped.
    Q5 = Q.copy(order="F")
    col = Q5[:, J + 2].copy()
    col.view(np.uint64)[7] ^= np.uint64(1)
    Q5[:, J + 2] = col
    inv = oracle.check_invariants(Y, Q5, R, J)
    assert inv[0] < 16 and inv[1] < 16 and inv[2] == 0 and inv[3] == 1, inv


def test_invariants_hold_through_the_fallback():
    """A rank-deficient block forces the CGS2 fallback; the invariants still hold
    after every block (the dependent column is zero with R_jj = 0)."""
    Y = inputs.uniform_matrix(20, 20, 5)
    Y2 = Y.copy()
    Y2[:, 9] = Y2[:, 8]
    out2 = oracle.cgs_qr(Y2, 4, check_invariants=True)
    assert out2["info"] == 3 and out2["block_flags"][2] & 1
    assert out2["inv"][2] == 0 and out2["inv"][3] == 0


# --------------------------------------------------------------------------
# Backward error at the small benchmark size (n = 512, uniform[-1, 1])
# --------------------------------------------------------------------------

@pytest.mark.parametrize("b", [32, 64, 128])
def test_backward_error_n512(b):
    Y = inputs.uniform_matrix(512, 512, seed=0)
    out = oracle.cgs_qr(Y, b)
    assert _recon(Y, out["Q"], out["R"]) < 16
    assert _orth(out["Q"]) < 16
    rhs = inputs.uniform_vector(512, seed=1)
    x, rc = oracle.qr_solve(out["Q"], out["R"], rhs)
    assert rc == 0
    hpl = np.abs(Y @ x - rhs).max() / (np.abs(Y).sum(axis=1).max() * np.abs(x).max() * 512 * EPS)
    assert hpl < 16
    np.testing.assert_allclose(x, np.linalg.solve(Y, rhs), rtol=0, atol=1e-9 * np.abs(x).max())


# --------------------------------------------------------------------------
# The readings of the paper: corrected R and H updates
# --------------------------------------------------------------------------

def _graded(q, r, kappa, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((q, r)))
    V, _ = np.linalg.qr(rng.standard_normal((r, r)))
    s = np.logspace(0, -math.log10(kappa), r)
    return (U * s) @ V.T


def test_printed_S7_order_loses_reconstruction():
    """Algorithm 4 S7 as printed (R = L^T Lbar^T) differs from the algebra of
    S3/S6 (R = Lbar^T L^T); on an ill-conditioned block only the corrected
    order reconstructs Y to working accuracy."""
    Y = _graded(200, 8, 1e6, 0)
    Qc, Rc, rc = oracle.cholqr2(Y)
    Qp, Rp, rp = oracle.cholqr2(Y, variant=oracle.VARIANT_PRINTED_R)
    assert rc == 0 and rp == 0
    rel_c = np.linalg.norm(Y - Qc @ Rc) / np.linalg.norm(Y)
    rel_p = np.linalg.norm(Y - Qp @ Rp) / np.linalg.norm(Y)
    assert rel_c < 1e-13
    assert rel_p > 1e3 * rel_c


def test_printed_S12_loses_reconstruction():
    """Algorithm 5 S12 as printed (H = H + Hbar) omits the factor L^T of the
    second projection; the corrected update reconstructs, the printed one does not."""
    rng = np.random.default_rng(1)
    P, _ = np.linalg.qr(rng.standard_normal((300, 16)))
    Qin = P @ rng.standard_normal((16, 8)) * 1e3 + _graded(300, 8, 1e3, 2)
    Qc, Hc, Rc, rc = oracle.cgs_cqr2(Qin, P)
    Qp, Hp, Rp, rp = oracle.cgs_cqr2(Qin, P, variant=oracle.VARIANT_PRINTED_H)
    assert rc == 0 and rp == 0
    rel_c = np.linalg.norm(Qin - P @ Hc - Qc @ Rc) / np.linalg.norm(Qin)
    rel_p = np.linalg.norm(Qin - P @ Hp - Qp @ Rp) / np.linalg.norm(Qin)
    assert rel_c < 1e-13
    assert rel_p > 10 * rel_c


def test_cgs_cqr2_outputs_contract():
    """Algorithm 5 contract: Q_in = P H + Q R, P^T Q = 0, Q^T Q = I, R upper."""
    rng = np.random.default_rng(7)
    P, _ = np.linalg.qr(rng.standard_normal((120, 24)))
    Qin = rng.standard_normal((120, 10))
    Q, H, R, rc = oracle.cgs_cqr2(Qin, P)
    assert rc == 0
    assert np.linalg.norm(Qin - P @ H - Q @ R) < 1e-13 * np.linalg.norm(Qin)
    assert np.abs(P.T @ Q).max() < 1e-14
    assert np.abs(Q.T @ Q - np.eye(10)).max() < 1e-14
    assert np.array_equal(np.tril(R, -1), np.zeros((10, 10)))
    assert (np.diag(R) > 0).all()


# --------------------------------------------------------------------------
# Building blocks: POTRF and TRSM against their definitions
# --------------------------------------------------------------------------

def test_chol_and_trsm_definitions():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((30, 12))
    W = A.T @ A
    L, rc = oracle.chol(W)
    assert rc == 0
    assert np.array_equal(np.triu(L, 1), np.zeros_like(L))
    np.testing.assert_allclose(L @ L.T, W, atol=1e-12 * np.abs(W).max())
    np.testing.assert_allclose(L, np.linalg.cholesky(W), atol=1e-12)
    X = oracle.trsm_rlt(A, L)
    np.testing.assert_allclose(X @ L.T, A, atol=1e-13)


def test_chol_breakdown_rule():
    """A pivot that is not > 0 is a breakdown (zero, negative and NaN)."""
    _, rc = oracle.chol(np.array([[4.0, 2.0], [2.0, 1.0]]))   # singular: second pivot 0
    assert rc == 2
    _, rc = oracle.chol(np.array([[1.0, 2.0], [2.0, 1.0]]))   # indefinite
    assert rc == 2
    _, rc = oracle.chol(np.array([[np.nan, 0.0], [0.0, 1.0]]))
    assert rc == 1


# --------------------------------------------------------------------------
# Breakdown fallback (CGS2 on the failed block)
# --------------------------------------------------------------------------

def test_fallback_on_hilbert_block():
    """A 60 x 12 Hilbert block has cond ~ 1e13 > 1/sqrt(eps): its Gram matrix is
    not numerically positive definite, so the block falls back to CGS2 and the
    result is still a QR factorisation satisfying the loop invariants."""
    w = 12
    Y = inputs.uniform_matrix(60, 3 * w, seed=8)
    i, j = np.arange(60), np.arange(w)
    Y[:, w:2 * w] = 1.0 / (i[:, None] + j[None, :] + 1.0)
    out = oracle.cgs_qr(Y, w, check_invariants=True)
    assert out["info"] == 2
    assert list(out["block_flags"]) == [0, 1, 0]
    assert np.linalg.norm(Y - out["Q"] @ out["R"]) < 1e-14 * np.linalg.norm(Y)
    i1, i2, i3, i4 = out["inv"]
    assert i1 < 16 and i2 < 16 and i3 == 0 and i4 == 0


def test_zero_column_is_flagged():
    Y = inputs.uniform_matrix(30, 12, seed=9)
    Y[:, 5] = 0.0
    out = oracle.cgs_qr(Y, 4)
    assert out["info"] == 2
    assert out["block_flags"][1] == 3
    assert out["R"][5, 5] == 0.0 and not out["Q"][:, 5].any()
    np.testing.assert_allclose(out["Q"] @ out["R"], Y, atol=1e-13)


def test_invalid_arguments():
    import ctypes
    lib = oracle._load()
    assert lib.ora_cgs_qr(3, 4, 1, None, 3, None, 4, 0, None, None, None) == -2
    assert lib.ora_cgs_qr(4, 4, 0, None, 4, None, 4, 0, None, None, None) == -3
    assert lib.ora_cgs_qr(4, 4, 2, None, 3, None, 4, 0, None, None, None) == -5
    del ctypes


# --------------------------------------------------------------------------
# Solve and its adjoint
# --------------------------------------------------------------------------

def test_solve_grad_against_finite_differences():
    """dL/dA and dL/db of L = w . solve(A, b) by central differences (h = 1e-6)."""
    n = 12
    A = inputs.uniform_matrix(n, n, seed=21) + 4 * np.eye(n)
    rhs = inputs.uniform_vector(n, seed=22)
    w = inputs.uniform_vector(n, seed=23)
    Q, R = oracle.householder_qr(A)
    x, _ = oracle.qr_solve(Q, R, rhs)
    dA, db, rc = oracle.qr_solve_grad(Q, R, x, w)
    assert rc == 0

    def loss(A_, b_):
        Qh, Rh = oracle.householder_qr(A_)
        xh, _ = oracle.qr_solve(Qh, Rh, b_)
        return float(w @ xh)

    h = 1e-6
    for (i, j) in [(0, 0), (3, 7), (11, 2), (5, 5)]:
        Ap, Am = A.copy(), A.copy()
        Ap[i, j] += h
        Am[i, j] -= h
        fd = (loss(Ap, rhs) - loss(Am, rhs)) / (2 * h)
        assert abs(fd - dA[i, j]) < 1e-7 * max(1.0, abs(fd))
    for i in range(n):
        bp, bm = rhs.copy(), rhs.copy()
        bp[i] += h
        bm[i] -= h
        fd = (loss(A, bp) - loss(A, bm)) / (2 * h)
        assert abs(fd - db[i]) < 1e-7 * max(1.0, abs(fd))
    # closed form: db = A^{-T} w, dA = -db x^T
    np.testing.assert_allclose(db, np.linalg.solve(A.T, w), atol=1e-12)
    np.testing.assert_allclose(dA, -np.outer(db, x), atol=1e-12)
