"""Flop counts of the factorisation from the paper's cost model (Table 1).

CA4(b, q)     = S1+S4 (2 b^2 q) + S3+S6 (2 b^2 q) + S2+S5 (2 b^3/3) + S7 (b^3)
CA5(b, q, s)  = S1+S6 (4 b q s) + S2+S7 (4 b q s) + S3+S8 (4 b^2 q)
                + S5+S10 (2 b^2 q) + S4+S9 (2 b^3/3) + S11 (b^3) + S12 (b s)
CA3(b, q, r)  = CA4(b, q) + sum_{j=2}^{k} CA5(b, q, (j-1) b),  k = r / b

For r not a multiple of b the last block has width w = r - (k-1) b and its
term is CA5(w, q, (k-1) b) (the widths enter Table 1 through b only).
The solve x = R^{-1} Q^T rhs adds 2 n^2 (product) + n^2 (substitution).
"""
from __future__ import annotations


def ca4(b: int, q: int) -> float:
    b, q = float(b), float(q)
    return 4.0 * b * b * q + 5.0 / 3.0 * b ** 3


def ca5(b: int, q: int, s: int) -> float:
    b, q, s = float(b), float(q), float(s)
    return 8.0 * b * q * s + 6.0 * b * b * q + 5.0 / 3.0 * b ** 3 + b * s


def ca3(b: int, q: int, r: int) -> float:
    if r <= 0:
        return 0.0
    k = -(-r // b)
    total = ca4(min(b, r), q)
    for j in range(2, k + 1):
        s = (j - 1) * b
        total += ca5(min(b, r - s), q, s)
    return total


def solve_flops(n: int) -> float:
    return 3.0 * float(n) * float(n)


def householder_flops(q: int, r: int) -> float:
    """Householder-equivalent count 2 q r^2 - 2 r^3 / 3 (for comparison only)."""
    return 2.0 * q * r * r - 2.0 * r ** 3 / 3.0
