"""Writes lancsvd_dense_m100000_n10000.json: the CPU oracle's truncated SVDs of
the paper's dense test matrix (Sec. 4, dense problems) at m = 1e5, n = 1e4,
seed 0 (A = X Sigma Y^T from paper_2403_06218_amd.inputs, start blocks N(0, 1)
from the same module): LancSVD with b = 16, r = 64 and p in {1, 4}, RandSVD
with b = 16, r = 16 and p in {1, 4}.  For each run it stores sigma_1..10 and
the residuals ||A v_j - sigma_j u_j|| / sigma_j, j = 1..10.

Calls only the oracle and the input generators (about three minutes and
10 GB of host memory).  Run from the repository root:
    python tests/golden/make_lancsvd_dense.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import svd as osvd  # noqa: E402
from paper_2403_06218_amd import inputs  # noqa: E402

M, N, SEED = 100000, 10000, 0


def main():
    A, sig = inputs.svd_test_matrix(M, N, SEED)
    out = {"m": M, "n": N, "seed": SEED, "sigma_exact_1_10": sig[:10].tolist(), "runs": {}}
    Q1 = inputs.normal_matrix(M, 16, SEED + 1)
    for p in (1, 4):
        ref = osvd.lancsvd(A, 64, p, 16, Q1)
        res = osvd.residuals(A, ref["U"], ref["sigma"], ref["V"], 10)
        out["runs"]["lancsvd_p%d" % p] = {"b": 16, "r": 64, "p": p, "sigma_1_10": ref["sigma"][:10].tolist(),
                                           "residual_1_10": res.tolist()}
    Q0 = inputs.normal_matrix(N, 16, SEED + 1)
    for p in (1, 4):
        U, s, V, _ = osvd.randsvd(A, 16, p, 16, Q0)
        res = osvd.residuals(A, U, s, V, 10)
        out["runs"]["randsvd_p%d" % p] = {"b": 16, "r": 16, "p": p, "sigma_1_10": s[:10].tolist(),
                                           "residual_1_10": res.tolist()}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lancsvd_dense_m100000_n10000.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
