"""Benchmark: FP64 CGS-QR factorisation (Algorithms 3-5) + solve on one MI355X.

One step = cqr_factor of a fresh, already-resident n x n matrix with i.i.d.
U[-1, 1] entries, then cqr_solve for one right-hand side.  GFLOP/s uses the
paper's cost model (Table 1): CA3(b, n, n) + 3 n^2 per step.

Prints one JSON line.  Also reports, for the kernel role that takes the most
time, its algorithmic rate from HIP events recorded around every launch on the
launch stream (roofline), and the CPU oracle timed on a bounded sample of the
same workload (cpu_baseline).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GFLOP/s at n=32768: BF16-MFMA LU+FP64 IR vs FP64 LUPP, HPL resid<16"
PEAK_FP64_MFMA_TFLOPS = 78.6  # MI355X dense FP64 matrix peak
PEAK_HBM_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=32768)
    p.add_argument("--b", type=int, default=128)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-target-s", type=float, default=15.0, help="target oracle time for the CPU sample")
    p.add_argument("--no-mixed", action="store_true", help="skip the BF16 + FP64-refinement form")
    p.add_argument("--calib-copy-mib", type=int, default=0,
                   help="before the run, copy this many MiB device-to-device once (reference kernel for HBM counters)")
    return p.parse_args()


def cpu_baseline(n: int, b: int, seed: int, target_s: float) -> dict:
    """The oracle's CGS-QR (plain C, OpenMP loops) on the first r0 columns of the
    same n x n input (q = n rows), r0 grown until the run takes ~target_s."""
    import oracle
    from paper_2403_06218_amd import costmodel, inputs

    def run(r0):
        Y = inputs.uniform_cols(n, n, seed, np.arange(r0))
        t0 = time.perf_counter()
        oracle.cgs_qr(Y, b)
        return time.perf_counter() - t0

    r0 = min(n, 2 * b)
    dt = run(r0)
    rate = costmodel.ca3(b, n, r0) / dt
    while r0 + b <= n and costmodel.ca3(b, n, r0 + b) / rate < target_s:
        r0 += b
    if r0 > 2 * b:
        dt = run(r0)
    fl = costmodel.ca3(b, n, r0)
    return {"value": round(fl / dt / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "oracle CGS-QR (Algs. 3-5, FP64) of the first %d columns of the same %dx%d input, b=%d: "
                      "%.3e flops (Table 1) in %.2f s" % (r0, n, n, b, fl, dt)}


def bench_mixed(cqr, torch, n: int, b: int, K: int, W: int, seed: int, fp64_ms: float) -> dict:
    """BF16-MFMA CGS-QR + FP64 iterative refinement on the diagonally dominant
    workload (off-diagonal U[-0.5, 0.5], diagonal = row sum of |.| + 1).
    Value = the same nominal flop count as the FP64 form / (factor + refine)."""
    from paper_2403_06218_amd import costmodel
    dev = torch.device("cuda:0")
    Y = cqr.colmajor(n, n, device=dev)
    cqr.synth_uniform(Y, seed + 17, -0.5, 0.5)
    Y.diagonal().zero_()
    Y.diagonal().copy_(Y.abs().sum(dim=1) + 1.0)
    rhs = torch.empty(n, dtype=torch.float64, device=dev)
    cqr.synth_uniform(rhs.view(n, 1), seed + 18)
    Q = cqr.colmajor(n, n, device=dev, dtype=torch.float32)
    R = cqr.colmajor(n, n, device=dev, dtype=torch.float32)
    import ctypes
    nb = ctypes.c_size_t(0)
    cqr._native.lib().cqr_workspace_size_mixed(n, n, b, cqr.PREC_BF16, ctypes.byref(nb))
    work = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)

    def step():
        _, _, info = cqr.qr_mixed(Y, b, Q=Q, R=R, work=work)
        x, iters, res = cqr.solve_ir(Y, Q, R, rhs, maxiter=50, tol=16.0)
        return info, iters, res

    for _ in range(W):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = [step() for _ in range(K)]
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / K
    t1 = time.perf_counter()
    cqr.qr_mixed(Y, b, Q=Q, R=R, work=work)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t1
    flops = costmodel.ca3(b, n, n) + costmodel.solve_flops(n)
    return {"value": round(flops / el / 1e9, 2), "unit": "GFLOP/s", "ms_per_step": round(el * 1e3, 2),
            "factor_ms": round(tf * 1e3, 2), "speedup_vs_fp64": round(fp64_ms / (el * 1e3), 3),
            "ir_iterations": [o[1] for o in out], "hpl_scaled_residual": [o[2] for o in out],
            "info": [o[0] for o in out], "dtype": "bf16 mfma (fp32 acc) + f64 panel + f64 refinement",
            "workload": "n=%d, b=%d, off-diagonal U[-0.5,0.5], diagonal = row sum + 1, 1 RHS U[-1,1]" % (n, b)}


def measured_traffic(role: str):
    """HBM bytes per launch of `role` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None if the GEMM source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    src = os.path.join(ROOT, "paper_2403_06218_amd", "csrc", "gemm_f64.hip")
    try:
        meta = json.load(open(path))
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if meta.get("gemm_source_sha256") != digest or role not in meta.get("roles", {}):
        return None
    return meta["roles"][role]["hbm_bytes_per_launch"]


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2403_06218_amd as cqr
    from paper_2403_06218_amd import costmodel, inputs

    n, b, K, W = args.n, args.b, args.steps, args.warmup
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    # Inputs: one resident copy of Y per step (the factorisation overwrites it).
    ncopies = K + W
    Ys = []
    for _ in range(ncopies):
        Y = cqr.colmajor(n, n, device=dev)
        cqr.synth_uniform(Y, args.seed)
        Ys.append(Y)
    rhs = torch.empty(n, dtype=torch.float64, device=dev)
    cqr.synth_uniform(rhs.view(n, 1), args.seed + 1)
    R = cqr.colmajor(n, n, device=dev)
    work = torch.empty(cqr.workspace_size(n, n, b), dtype=torch.uint8, device=dev)
    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    swork = torch.empty(max(256, 8 * n), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step(i):
        Q, Rr, info, flags = cqr.qr(Ys[i], b, R=R, work=work)
        x = cqr.solve(Q, Rr, rhs, work=swork)
        return info, x

    for i in range(W):
        step(i)
    torch.cuda.synchronize()

    cqr.prof_reset()
    cqr.prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    x = None
    for i in range(W, W + K):
        info, x = step(i)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cqr.prof_enable(False)

    flops_step = costmodel.ca3(b, n, n) + costmodel.solve_flops(n)
    ms_step = 1e3 * elapsed / K
    value = flops_step / (elapsed / K) / 1e9

    roles = {}
    for name in cqr.prof_names():
        r = cqr.prof_query(name)
        if r["launches"]:
            roles[name] = r
    dom = max(roles, key=lambda k: roles[k]["ms"])
    d = roles[dom]
    achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12
    traffic = measured_traffic(dom)
    roofline = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 3), "peak": PEAK_FP64_MFMA_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_MFMA_TFLOPS, 4),
                "traffic": round(traffic) if traffic else None, "traffic_unit": "HBM bytes per launch",
                "algorithmic_bytes_per_launch": round(d["bytes"] / d["launches"]),
                "launches_per_step": d["launches"] // K, "avg_launch_ms": round(d["ms"] / d["launches"], 4)}
    breakdown = {k: {"ms_per_step": round(v["ms"] / K, 3), "launches_per_step": v["launches"] // K,
                     "tflops": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 3) if v["flops"] else None}
                 for k, v in sorted(roles.items(), key=lambda kv: -kv[1]["ms"])}

    # Sampled checks on the last step's result: HPL-style residual on sampled rows
    # of Y (regenerated on the CPU), and orthogonality of sampled column pairs.
    Q = Ys[W + K - 1]
    rng = np.random.default_rng(123)
    rows = np.sort(rng.choice(n, size=min(n, 64), replace=False))
    Yrows = inputs.uniform_rows(n, n, args.seed, rows)
    xh = x.cpu().numpy()
    bh = inputs.uniform_vector(n, args.seed + 1)
    res = np.abs(Yrows @ xh - bh[rows]).max()
    hpl_rows = res / (np.abs(Yrows).sum(axis=1).max() * np.abs(xh).max() * n * 2.0 ** -52)
    cols = np.sort(rng.choice(n, size=min(n, 16), replace=False))
    Qc = Q[:, torch.from_numpy(cols).to(dev)].cpu().numpy()
    orth = np.abs(Qc.T @ Qc - np.eye(len(cols))).max()

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(ms_step, 2), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "FP64 CGS-QR (Algs. 3-5) + solve, n=%d, b=%d, U[-1,1] entries, 1 RHS" % (n, b),
                   "n": n, "b": b, "rhs": 1, "seed": args.seed, "form": "fp64",
                   "flops_per_step": flops_step, "flop_model": "Table 1 CA3(b,n,n) + 3n^2"},
        "roofline": roofline,
        "breakdown": breakdown,
        "checks": {"info": infos, "hpl_scaled_residual_sampled_rows": float(hpl_rows),
                   "max_offdiag_QtQ_sampled_cols": float(orth)},
    }
    if not args.no_mixed:
        del Ys
        torch.cuda.empty_cache()
        out["mixed"] = bench_mixed(cqr, torch, n, b, K, W, args.seed, ms_step)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, b, args.seed, args.cpu_target_s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
