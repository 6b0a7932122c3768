"""Seeded synthetic inputs shared by the HIP path's tests, the benchmark and the oracle's checks.

This module holds no arithmetic of the factorisation: it only draws numbers.
The element stream is counter based, so any single row or column of a large
matrix can be regenerated on the CPU without materialising the rest.

Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), in the form of Vigna's public-domain reference
``splitmix64.c``.  For seed ``s`` the stream state starts at
``key = mix(s + GAMMA)`` and the element with linear index ``t`` is
``z = mix(key + (t + 1) * GAMMA)`` (mod 2^64), i.e. output t of a SplitMix64
stream seeded with ``key``.  A uniform double in [0, 1) is ``(z >> 11) * 2^-53``
and a value in [lo, hi) is ``lo + (hi - lo) * u`` rounded as a product then a sum
(exact for [-1, 1) and [-0.5, 0.5)).  Element (i, j) of a rows x cols matrix has
linear index ``t = i + j * rows`` (column-major, independent of any padding).

The HIP fill kernel in ``csrc/synth.hip`` implements the same definition
independently, so a GPU-resident input of any size matches this module bit for bit.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int) -> np.uint64:
    with np.errstate(over="ignore"):
        return _mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + GAMMA)[()]


def uniform01(seed: int, idx) -> np.ndarray:
    """Uniform doubles in [0, 1) for linear indices ``idx`` (any integer array)."""
    key = stream_key(seed)
    t = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _mix(key + (t + np.uint64(1)) * GAMMA)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _affine(u: np.ndarray, lo: float, hi: float) -> np.ndarray:
    scale = np.float64(hi) - np.float64(lo)
    return np.float64(lo) + scale * u


def uniform_matrix(rows: int, cols: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """rows x cols column-major (Fortran-order) float64 matrix of i.i.d. U[lo, hi)."""
    out = np.empty((rows, cols), dtype=np.float64, order="F")
    step = max(1, (1 << 24) // max(rows, 1))
    for j0 in range(0, cols, step):
        j1 = min(cols, j0 + step)
        t = np.arange(j0 * rows, j1 * rows, dtype=np.uint64)
        out[:, j0:j1] = _affine(uniform01(seed, t), lo, hi).reshape((j1 - j0, rows)).T
    return out


def uniform_rows(rows: int, cols: int, seed: int, row_idx, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Selected rows (len(row_idx) x cols) of ``uniform_matrix(rows, cols, seed)``."""
    r = np.asarray(row_idx, dtype=np.uint64)[:, None]
    c = np.arange(cols, dtype=np.uint64)[None, :]
    return _affine(uniform01(seed, r + c * np.uint64(rows)), lo, hi)


def uniform_cols(rows: int, cols: int, seed: int, col_idx, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Selected columns (rows x len(col_idx)) of ``uniform_matrix(rows, cols, seed)``."""
    del cols
    r = np.arange(rows, dtype=np.uint64)[:, None]
    c = np.asarray(col_idx, dtype=np.uint64)[None, :]
    return np.asfortranarray(_affine(uniform01(seed, r + c * np.uint64(rows)), lo, hi))


def uniform_vector(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return _affine(uniform01(seed, np.arange(n, dtype=np.uint64)), lo, hi)


def normal_matrix(rows: int, cols: int, seed: int) -> np.ndarray:
    """Standard normal entries by Box-Muller on two counter streams (CPU only)."""
    t = np.arange(rows * cols, dtype=np.uint64)
    u1 = uniform01(seed, t)
    u2 = uniform01(seed ^ 0x5DEECE66D, t)
    z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
    return np.asfortranarray(z.reshape((cols, rows)).T)


def diag_dominant(n: int, seed: int) -> np.ndarray:
    """Off-diagonal U[-0.5, 0.5), diagonal = sum_{j != i} |a_ij| + 1 (row sums)."""
    A = uniform_matrix(n, n, seed, -0.5, 0.5)
    np.fill_diagonal(A, 0.0)
    d = np.abs(A).sum(axis=1) + 1.0
    A[np.arange(n), np.arange(n)] = d
    return A


def batch_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """``count`` integers drawn uniformly from [lo, hi] (inclusive)."""
    u = uniform01(seed, np.arange(count, dtype=np.uint64))
    return (lo + np.floor(u * (hi - lo + 1))).astype(np.int64)


def packed_offsets(sizes) -> np.ndarray:
    """Start of each n_i x n_i matrix in a packed column-major batch (ld = n_i)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    off = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes * sizes, out=off[1:])
    return off


def packed_matrix(sizes, i: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Matrix i of a packed batch filled as one stream: element (r, c) of matrix
    i is stream element off_i + r + c n_i (the layout of a flat device buffer
    filled by the GPU generator as a single column)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    n = int(sizes[i])
    o = int(packed_offsets(sizes)[i])
    t = np.arange(o, o + n * n, dtype=np.uint64)
    return np.asfortranarray(_affine(uniform01(seed, t), lo, hi).reshape((n, n)).T)


def packed_vector(sizes, i: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Vector i (length n_i) of a packed batch of vectors filled as one stream."""
    sizes = np.asarray(sizes, dtype=np.int64)
    o = int(sizes[:i].sum())
    t = np.arange(o, o + int(sizes[i]), dtype=np.uint64)
    return _affine(uniform01(seed, t), lo, hi)


def svd_test_sigma(n: int) -> np.ndarray:
    """Singular values of the dense truncated-SVD benchmark (Sec. 4, dense
    problems): sigma_i = 10^(15 i / (n/2) - 14) for 1 <= i <= n/2 and 1e-14
    for the rest, returned in decreasing order (largest 10, at i = n/2)."""
    h = n // 2
    i = np.arange(1, h + 1, dtype=np.float64)
    top = 10.0 ** (15.0 * i / h - 14.0)
    return np.concatenate([top[::-1], np.full(n - h, 1e-14)])


def _unit_normals(count: int, n: int, seed: int) -> list:
    """``count`` unit vectors of length n with N(0, 1) directions (counter stream)."""
    out = []
    for c in range(count):
        t = np.arange(n, dtype=np.uint64) + np.uint64(c * n)
        u1 = uniform01(seed, t)
        u2 = uniform01(seed ^ 0x5DEECE66D, t)
        v = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
        out.append(v / np.linalg.norm(v))
    return out


def svd_test_parts(m: int, n: int, seed: int) -> dict:
    """The random ingredients of ``svd_test_matrix``: unit vectors of four
    Householder reflectors for each of the orthogonal factors Z and Y, and per
    row block l of X a sign vector and a column permutation."""
    if m % n:
        raise ValueError("m must be a multiple of n")
    c = m // n
    zs = _unit_normals(4, n, seed + 1)
    ys = _unit_normals(4, n, seed + 2)
    signs, perms = [], []
    for l in range(c):
        t = np.arange(n, dtype=np.uint64)
        signs.append(np.where(uniform01(seed + 3 + 2 * l, t) < 0.5, -1.0, 1.0))
        perms.append(np.argsort(uniform01(seed + 4 + 2 * l, t), kind="stable"))
    return {"c": c, "zs": zs, "ys": ys, "signs": signs, "perms": perms, "sigma": svd_test_sigma(n)}


def svd_test_matrix(m: int, n: int, seed: int):
    """A = X Sigma Y^T (m x n, column-major) with the singular values of
    ``svd_test_sigma``.  Y = H(y1) H(y2) H(y3) H(y4) is a product of four random
    Householder reflectors H(v) = I - 2 v v^T (dense and orthogonal); X (m x n,
    m a multiple c of n) stacks c row blocks D_l Z P_l / sqrt(c) with Z another
    such product, D_l random signs and P_l random column permutations, so that
    X^T X = I in exact arithmetic and large m stays cheap (block l of A is
    D_l (Z P_l Sigma) Y^T / sqrt(c); the reflectors are applied, never
    factorised).  Returns (A, sigma)."""
    parts = svd_test_parts(m, n, seed)
    c, sig = parts["c"], parts["sigma"]
    Z = np.eye(n)
    for z in parts["zs"]:
        Z -= 2.0 * np.outer(Z @ z, z)
    A = np.empty((m, n), order="F")
    for l in range(c):
        M = Z[:, parts["perms"][l]] * sig
        for y in reversed(parts["ys"]):
            M -= 2.0 * np.outer(M @ y, y)
        A[l * n:(l + 1) * n, :] = parts["signs"][l][:, None] * M / np.sqrt(c)
    return A, sig


def svd_test_matrix_device(m: int, n: int, seed: int, device="cuda"):
    """``svd_test_matrix`` built on the GPU with torch from the same random
    ingredients (the same matrix up to rounding), column-major (m, n) with
    leading dimension m; for sizes the host cannot hold (m = 1e6, n = 1e4 is
    80 GB)."""
    import torch
    parts = svd_test_parts(m, n, seed)
    c = parts["c"]
    sig = torch.from_numpy(parts["sigma"]).to(device)
    Z = torch.eye(n, dtype=torch.float64, device=device)
    for z in parts["zs"]:
        zt = torch.from_numpy(z).to(device)
        Z.sub_(2.0 * torch.outer(Z @ zt, zt))
    ys = [torch.from_numpy(y).to(device) for y in reversed(parts["ys"])]
    A = torch.empty((n, m), dtype=torch.float64, device=device).t()
    for l in range(c):
        M = Z.index_select(1, torch.from_numpy(parts["perms"][l]).to(device)) * sig
        for yt in ys:
            M.sub_(2.0 * torch.outer(M @ yt, yt))
        d = torch.from_numpy(parts["signs"][l]).to(device)
        A[l * n:(l + 1) * n, :] = d[:, None] * M / float(np.sqrt(c))
        del M
    return A, parts["sigma"]


def sparse_matrix(m: int, n: int, nnz: int, seed: int):
    """Synthetic sparse m x n matrix in CSR form (int32 row pointers and
    sorted column indices, float64 values U[-1, 1)) with about ``nnz``
    nonzeros: heavy-tailed row lengths (length_i proportional to
    (1 - u_i)^(-1/2), at least 1, at most n, rescaled to the requested total)
    and uniformly drawn columns, duplicates within a row dropped.  Returns
    (rowptr, col, val)."""
    u = uniform01(seed, np.arange(m, dtype=np.uint64))
    w = (1.0 - u) ** -0.5
    lens = np.maximum(1, np.minimum(n, np.round(w * (nnz / w.sum())))).astype(np.int64)
    total = int(lens.sum())
    rows = np.repeat(np.arange(m, dtype=np.int64), lens)
    cols = np.floor(uniform01(seed + 1, np.arange(total, dtype=np.uint64)) * n).astype(np.int64)
    key = np.unique(rows * n + cols)
    rows, cols = key // n, key % n
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    vals = _affine(uniform01(seed + 2, np.arange(key.size, dtype=np.uint64)), -1.0, 1.0)
    return rowptr.astype(np.int32), cols.astype(np.int32), vals
