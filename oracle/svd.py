"""CPU FP64 oracle for the truncated-SVD drivers of arXiv 2403.06218, Sec. 2:
RandSVD (Algorithm 1) and LancSVD (Algorithm 2).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the HIP library and its
binding never do, and the two share no code.

Each step follows the algorithm in the paper's order and notation.  The
orthogonalisations are the oracle's own CholeskyQR2 / CGS-CQR2 / CGS-QR
(``oracle.c``, with the Section 3 CGS2 fallback), the products with A are
plain numpy matrix products and the small r x r SVD is numpy's (LAPACK): a
library primitive used as one step.  Random start matrices are inputs.

Readings of the paper (where the text is garbled or silent):
  * Algorithm 2 S8 prints V_T = [Q_1 ... Q_k] Vbar^T; the factorisation
    B_k = Ubar S Vbar^T and A ~ Pbar_k B_k P_k^T give V_T = P_k Vbar.
  * B_k is assembled from the triangular factors the orthogonalisations
    return: L_i = (the R factor of S3)^T on the diagonal blocks, R_i (S5) on
    the blocks below them; the coefficient blocks H_i, Hbar_i are not part
    of it (in exact arithmetic they vanish except where they repeat L_i and
    R_{i-1}^T).
  * The residual of a computed triplet is ||A v_j - sigma_j u_j||_2 / sigma_j
    (u_j left, in R^m; v_j right, in R^n).
  * r must be a multiple of b (the paper assumes it).
"""
from __future__ import annotations

import numpy as np

from . import cgs_qr, orth_against_fb


def _orth(Q, P=None):
    """Orthogonalise the block Q (against P): returns (Q, H, R, fallback_rc)."""
    return orth_against_fb(Q, P)


def randsvd(A, r: int, p: int, b: int, Q0):
    """Algorithm 1 (RandSVD).  A (m x n), start Q0 (n x r).  Returns
    (U_T (m x r), sigma (r,), V_T (n x r), info) where info lists the CGS-QR
    info of every factorisation."""
    A = np.asarray(A, dtype=np.float64)
    Q = np.asarray(Q0, dtype=np.float64)
    infos = []
    Qbar = R = None
    for _ in range(p):
        Ybar = A @ Q                          # S1  Ybar_j = A Q_{j-1}
        f = cgs_qr(Ybar, b)                   # S2  Ybar_j = Qbar_j Rbar_j (Alg. 3)
        Qbar = f["Q"]
        infos.append(f["info"])
        Y = A.T @ Qbar                        # S3  Y_j = A^T Qbar_j
        f = cgs_qr(Y, b)                      # S4  Y_j = Q_j R_j (Alg. 3)
        Q, R = f["Q"], f["R"]
        infos.append(f["info"])
    Ub, s, Vbt = np.linalg.svd(R)             # S5  R_p = Ubar S Vbar^T
    U = Qbar @ Vbt.T                          # S6  U_T = Qbar_p Vbar
    V = Q @ Ub                                # S7  V_T = Q_p Ubar
    return U, s, V, infos


def block_bidiagonal(Ls, Rs):
    """B_k of Section 2.2: L_1 .. L_k on the diagonal blocks, R_1 .. R_{k-1}
    on the blocks below them (b x b each)."""
    k = len(Ls)
    b = Ls[0].shape[0]
    B = np.zeros((k * b, k * b))
    for i in range(k):
        B[i * b:(i + 1) * b, i * b:(i + 1) * b] = Ls[i]
        if i + 1 < k:
            B[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = Rs[i]
    return B


def lancsvd(A, r: int, p: int, b: int, Qbar_start, keep_last: bool = False):
    """Algorithm 2 (LancSVD) with the basic restart.  A (m x n), start block
    Qbar_start (m x b, orthonormalised in S1).  Returns a dict with U (m x r),
    sigma (r,), V (n x r), B (the last B_k), and, with keep_last, the bases
    of the last restart (P, Pbar, Qnext = Qbar_{k+1}, Rk) and the fallback
    codes of every orthogonalisation."""
    A = np.asarray(A, dtype=np.float64)
    if r % b:
        raise ValueError("r must be a multiple of b")
    k = r // b
    Qbar, _, _, rc0 = _orth(Qbar_start)            # S1  random orthonormal Qbar_1 (Alg. 4)
    codes = [rc0]
    for j in range(p):
        Pbar = [Qbar]
        P = []
        Ls, Rs = [], []
        for i in range(k):
            Qi = A.T @ Pbar[i]                     # S2  Q_i = A^T Qbar_i
            if i == 0:
                Qi, _, LT, rc = _orth(Qi)          # S3a Q_1 = Q_1 L_1^T (Alg. 4)
            else:
                Qi, _, LT, rc = _orth(Qi, np.hstack(P))  # S3b against P_{i-1} (Alg. 5)
            codes.append(rc)
            P.append(Qi)
            Ls.append(LT.T)
            Qn = A @ Qi                            # S4  Qbar_{i+1} = A Q_i
            Qn, _, Ri, rc = _orth(Qn, np.hstack(Pbar))  # S5 against Pbar_i (Alg. 5)
            codes.append(rc)
            Pbar.append(Qn)
            Rs.append(Ri)
        B = block_bidiagonal(Ls, Rs)
        Ub, s, Vbt = np.linalg.svd(B)              # S6  B_k = Ubar S Vbar^T
        if j < p - 1:
            Qbar = np.hstack(Pbar[:k]) @ Ub[:, :b]  # S7  restart with Pbar_k Ubar_1
    V = np.hstack(P) @ Vbt.T                        # S8  V_T = P_k Vbar
    U = np.hstack(Pbar[:k]) @ Ub                    # S9  U_T = Pbar_k Ubar
    out = {"U": U, "sigma": s, "V": V, "B": B, "codes": codes}
    if keep_last:
        out.update({"P": np.hstack(P), "Pbar": np.hstack(Pbar[:k]), "Qnext": Pbar[k], "Rk": Rs[-1]})
    return out


def residuals(A, U, s, V, count: int | None = None):
    """R_j = ||A v_j - sigma_j u_j||_2 / sigma_j for the first `count` triplets."""
    c = len(s) if count is None else count
    A = np.asarray(A, dtype=np.float64)
    return np.linalg.norm(A @ V[:, :c] - U[:, :c] * s[:c], axis=0) / s[:c]
