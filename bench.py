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
PEAK_FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix peak
PEAK_BF16_MFMA_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak
PEAK_FP8_MFMA_TFLOPS = 5000.0  # MI355X dense FP8 matrix peak


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=32768)
    p.add_argument("--b", type=int, default=0, help="block width of the FP64 form; 0 = autotune over --b-candidates")
    p.add_argument("--b-candidates", default="64,128,256")
    p.add_argument("--c3-n", type=int, default=0, help="order of the diagonally dominant comparison (0 = --n)")
    p.add_argument("--c3-fp64-steps", type=int, default=3,
                   help="timed FP64 steps on the diagonally dominant matrix (the speed-up's denominator)")
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-target-s", type=float, default=15.0, help="target oracle time for the CPU sample")
    p.add_argument("--no-mixed", action="store_true", help="skip the BF16 + FP64-refinement form")
    p.add_argument("--mixed-b", type=int, default=256, help="block width of the BF16 form")
    p.add_argument("--no-tiled", action="store_true", help="low-precision forms: column-major finished columns")
    p.add_argument("--no-batched", action="store_true", help="skip the batched form (10,000 uneven sizes)")
    p.add_argument("--no-adjoint", action="store_true", help="skip the adjoint form (256 x n=512)")
    p.add_argument("--no-tune", action="store_true", help="batched form: keep the library's default plan")
    p.add_argument("--no-tall", action="store_true", help="skip the paper's tall-skinny shape (q up to 1e6, r=64, b=16)")
    p.add_argument("--no-svd", action="store_true", help="skip the truncated-SVD benchmark (Sec. 4 dense)")
    p.add_argument("--svd-m", default="100000,1000000", help="row counts m of the truncated-SVD benchmark")
    p.add_argument("--svd-p", default="1,4", help="restart cycles p of the truncated-SVD benchmark")
    p.add_argument("--no-fp64", action="store_true", help="profiling aid: skip the FP64 n x n measurement")
    p.add_argument("--counters-only", action="store_true",
                   help="profiler driver: one untimed FP64 step (--b) and, unless --no-mixed, one BF16 and one FP8 "
                        "factorisation of the diagonally dominant matrix, and unless --no-batched one FP64 and one "
                        "FP32 call of the batched form; no checks, no JSON line")
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


def _graph_ms(torch, run, reset, K, W):
    """Captures run() in a hipGraph and times K replays (after W) with HIP events
    on the current stream; reset() (untimed) restores the inputs before each."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        reset()
        run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    times = []
    for i in range(W + K):
        reset()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        if i >= W:
            times.append(e0.elapsed_time(e1))
    return float(np.median(times)), times


def bench_batched(torch, K: int, W: int, seed: int, tune: bool) -> dict:
    """10,000 square systems, n uniform in [8, 256], U[-1, 1) entries, one RHS
    each, FP64 and FP32: the whole batch (factor + solve) in one hipGraph replay."""
    from paper_2403_06218_amd import batched, costmodel, inputs
    sizes = inputs.batch_sizes(10000, 8, 256, seed=seed)
    out = {"workload": "10000 matrices, n ~ U[8, 256] (integer), U[-1,1) entries, 1 RHS each",
           "flop_model": "sum over matrices of Table 1 CA3(b_i, n_i, n_i) + 3 n_i^2"}
    for dt, name, peak in ((torch.float64, "f64", PEAK_FP64_MFMA_TFLOPS), (torch.float32, "f32",
                                                                           PEAK_FP32_MFMA_TFLOPS)):
        t0 = time.perf_counter()
        tuned = batched.tune(dt, buckets=((0, 64), (64, 128), (128, 256), (256, 512)), count=1024) if tune else None
        tune_s = time.perf_counter() - t0
        insts = batched.instances()
        plan = batched.get_plan(dt)
        batch = batched.PackedBatch(sizes, dtype=dt)
        batched._fill(batch, seed + 100)
        a0, b0 = batch.A.clone(), batch.B.clone()
        work = torch.empty(max(batched.workspace_size(batch.count), 1), dtype=torch.uint8, device="cuda")

        def reset():
            batch.A.copy_(a0)
            batch.B.copy_(b0)

        ms, times = _graph_ms(torch, lambda: batched.factor_solve(batch, work), reset, K, W)
        flops = 0.0
        uniq, cnt = np.unique(sizes, return_counts=True)
        for nn, c in zip(uniq, cnt):
            flops += c * (costmodel.ca3(batched.block_width(int(nn), dt), int(nn), int(nn))
                          + costmodel.solve_flops(int(nn)))
        info = batch.info.cpu().numpy()
        eps = 2.0 ** -52 if dt == torch.float64 else 2.0 ** -23
        rng = np.random.default_rng(7)
        worst = 0.0
        for i in rng.choice(batch.count, 64, replace=False):
            n = int(sizes[i])
            o, vo = int(batch.offsets[i]), int(batch.voffsets[i])
            Y = a0[o:o + n * n].view(n, n).t().double()
            x = batch.B[vo:vo + n].double()
            r = (Y @ x - b0[vo:vo + n].double()).abs().max() / (Y.abs().sum(dim=1).max() * x.abs().max() * n * eps)
            worst = max(worst, float(r))
        tflops = flops / (ms * 1e-3) / 1e12
        out[name] = {"ms_per_batch": round(ms, 3), "matrices_per_s": round(batch.count / (ms * 1e-3), 1),
                     "value": round(tflops * 1e3, 2), "unit": "GFLOP/s", "flops_per_batch": flops,
                     "roofline": {"bound": "mfma", "achieved": round(tflops, 3), "peak": peak, "unit": "TFLOP/s",
                                  "frac": round(tflops / peak, 4)},
                     "plan": {"hi": plan["hi"], "instances": [insts[i] for i in plan["inst"]]},
                     "tune_s": round(tune_s, 2) if tuned else None,
                     "tune_ms": tuned["timings_ms"] if tuned else None,
                     "fallback_matrices": int((info > 0).sum()), "invalid": int((info < 0).sum()),
                     "hpl_scaled_residual_max_of_64_sampled": worst,
                     "replay_ms_min_max": [round(min(times), 3), round(max(times), 3)]}
        del batch, a0, b0
        torch.cuda.empty_cache()
    return out


def bench_adjoint(torch, K: int, W: int, seed: int) -> dict:
    """256 systems n = 512 (U[-1, 1) + 4 I, RHS U[-1, 1)), loss = sum(w x):
    forward (batched factor + solve) and the adjoint kernel, FP64 and FP32."""
    from paper_2403_06218_amd import batched, costmodel
    from paper_2403_06218_amd import synth_uniform
    count, n = 256, 512
    out = {"workload": "256 matrices n=512, U[-1,1) + 4I, RHS and w U[-1,1), loss = sum(w*x)"}
    for dt, name in ((torch.float64, "f64"), (torch.float32, "f32")):
        batch = batched.PackedBatch([n] * count, dtype=dt)
        tmp = torch.empty(batch.A.numel(), dtype=torch.float64, device="cuda")
        synth_uniform(tmp.view(-1, 1), seed + 300)
        A3 = tmp.view(count, n, n)
        A3.diagonal(dim1=1, dim2=2).add_(4.0)
        batch.A.copy_(tmp)
        tb = torch.empty(batch.B.numel(), dtype=torch.float64, device="cuda")
        synth_uniform(tb.view(-1, 1), seed + 301)
        batch.B.copy_(tb)
        synth_uniform(tb.view(-1, 1), seed + 302)
        g = tb.to(dt)
        a0, b0 = batch.A.clone(), batch.B.clone()
        del tmp
        work = torch.empty(max(batched.workspace_size(count), 1), dtype=torch.uint8, device="cuda")

        def reset():
            batch.A.copy_(a0)
            batch.B.copy_(b0)

        fwd_ms, _ = _graph_ms(torch, lambda: batched.factor_solve(batch, work), reset, K, W)
        reset()
        batched.factor_solve(batch, work)
        dA = torch.empty_like(batch.A)
        db = torch.empty_like(batch.B)
        # The backward kernel takes about a quarter millisecond, so one launch
        # per graph replay would charge it the replay's launch latency: the
        # graph holds REP back-to-back calls (each reads Q, R, x and g and
        # writes dA and db, the same work every time) and a call is 1/REP of a
        # replay; the one-call replay is reported beside it.
        REP = 8

        def bwd_rep():
            for _ in range(REP):
                batched.solve_backward(batch, g, dA, db)

        bwd_rep_ms, _ = _graph_ms(torch, bwd_rep, lambda: None, K, W)
        bwd_ms = bwd_rep_ms / REP
        bwd_one_ms, _ = _graph_ms(torch, lambda: batched.solve_backward(batch, g, dA, db), lambda: None, K, W)
        es = batch.A.element_size()
        # Algorithmic bytes per matrix: read Q (n^2) and the upper triangle of R
        # (n(n+1)/2), write dA (n^2); vectors x, g, db (3n).
        bytes_ = count * es * (2.0 * n * n + n * (n + 1) / 2.0 + 3.0 * n)
        gbs = bytes_ / (bwd_ms * 1e-3) / 1e9
        fwd_flops = count * (costmodel.ca3(batched.block_width(n, dt), n, n) + costmodel.solve_flops(n))
        out[name] = {"forward_ms": round(fwd_ms, 3), "backward_ms": round(bwd_ms, 4),
                     "backward_calls_per_replay": REP, "backward_ms_one_call_replay": round(bwd_one_ms, 3),
                     "forward_gflops": round(fwd_flops / (fwd_ms * 1e-3) / 1e9, 1),
                     "backward_roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                                           "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                                           "algorithmic_bytes": bytes_},
                     "info_nonzero": int((batch.info.cpu() != 0).sum())}
        del batch, a0, b0, dA, db
        torch.cuda.empty_cache()
    return out


def bench_tall(cqr, torch, K: int, W: int, seed: int) -> dict:
    """The paper's orthogonalisation shape inside LancSVD (Sec. 4, dense
    experiments: b = 16, r = 64): CGS-QR of Y in R^{q x 64}, N(0, 1) entries,
    q in {1e5, 2.5e5, 7.5e5, 1e6}.  HBM-bound; algorithmic bytes
    8 q (5 b + sum_{j=2..4} (4 s_j + 9 b)) with s_j = 16 (j - 1)."""
    from paper_2403_06218_amd import costmodel, inputs
    r, b = 64, 16
    out = {"workload": "CGS-QR of q x 64, b=16, N(0,1) entries (Box-Muller on the counter stream)"}
    for q in (100000, 250000, 750000, 1000000):
        Y0 = torch.from_numpy(np.ascontiguousarray(inputs.normal_matrix(q, r, seed + q).T)).cuda().t()
        Ys = [Y0.t().contiguous().t() for _ in range(K + W)]
        R = cqr.colmajor(r, r)
        work = torch.empty(cqr.workspace_size(q, r, b), dtype=torch.uint8, device="cuda")
        for i in range(W):
            cqr.qr(Ys[i], b, R=R, work=work)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = [cqr.qr_async(Ys[W + i], b, R=R, work=work)[2] for i in range(K)]
        torch.cuda.synchronize()
        infos = [int(v[0]) for v in infos]
        ms = (time.perf_counter() - t0) / K * 1e3
        Yp = Ys[0]
        Yp.copy_(Y0)
        cqr.prof_reset()
        cqr.prof_enable(True)
        cqr.qr(Yp, b, R=R, work=work)
        torch.cuda.synchronize()
        cqr.prof_enable(False)
        roles = {}
        for name in cqr.prof_names():
            rr = cqr.prof_query(name)
            if rr["launches"]:
                roles[name] = {"ms": round(rr["ms"], 4), "launches": rr["launches"]}
        alg_bytes = 8.0 * q * (5 * b + sum(4 * 16 * (j - 1) + 9 * b for j in range(2, 5)))
        gbs = alg_bytes / (ms * 1e-3) / 1e9
        Q = Ys[-1]
        cols = torch.tensor([0, 17, 40, 63], device="cuda")
        qc = Q[:, cols]
        gram = (qc.unsqueeze(2) * qc.unsqueeze(1)).sum(dim=0)
        orth = float((gram - torch.eye(4, device="cuda", dtype=torch.float64)).abs().max())
        out["q=%d" % q] = {"ms": round(ms, 3), "GB_per_s": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM_GBS, 4),
                           "gflops": round(costmodel.ca3(b, q, r) / (ms * 1e-3) / 1e9, 1), "info": infos,
                           "max_offdiag_QtQ_4_cols": orth, "breakdown": roles}
        del Ys, Y0, Q
        torch.cuda.empty_cache()
    return out


def bench_lancsvd(torch, seed: int, ms_list, ps, n: int = 10000) -> dict:
    """The paper's dense truncated-SVD benchmark (Sec. 4): A = X Sigma Y^T,
    m x n with n = 1e4, m in ms_list, sigma_i = 10^(15 i/(n/2) - 14) for the
    top half and 1e-14 for the rest; LancSVD with b = 16, r = 64 and p restart
    cycles, RandSVD with r = 16 for comparison at the same p.  Reports time,
    the residuals R_1 and R_10 (||A v_j - sigma_j u_j|| / sigma_j) and the
    error of sigma_1..10 against the constructed values; HBM rate of the
    products with A (the dominant, HBM-bound role)."""
    import paper_2403_06218_amd as cqr
    from paper_2403_06218_amd import inputs, svd
    out = {"workload": "A = X Sigma Y^T (Sec. 4 dense), n=%d, LancSVD b=16 r=64, RandSVD r=16 b=16; "
                       "start blocks N(0,1)" % n}
    for m in ms_list:
        A, sig = inputs.svd_test_matrix_device(m, n, seed)
        torch.cuda.synchronize()
        entry = {}
        for method, r, b in (("lancsvd", 64, 16), ("randsvd", 16, 16)):
            rows = m if method == "lancsvd" else n
            Q1 = torch.from_numpy(np.ascontiguousarray(inputs.normal_matrix(rows, b if method == "lancsvd" else r,
                                                                            seed + 1).T)).cuda().t()
            work = torch.empty(svd.workspace_size(svd.LANCZOS if method == "lancsvd" else svd.RANDOMIZED, m, n, r, b),
                               dtype=torch.uint8, device="cuda")
            fn = svd.lancsvd if method == "lancsvd" else svd.randsvd
            for p in ps:
                fn(A, r, b, p, Q1, work=work)  # warm-up
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                U, s, V, info = fn(A, r, b, p, Q1, work=work, sync=False)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                cqr.prof_reset()
                cqr.prof_enable(True)
                fn(A, r, b, p, Q1, work=work, sync=False)
                torch.cuda.synchronize()
                cqr.prof_enable(False)
                ap = cqr.prof_query("aprod")
                res = svd.residuals(A, U, s, V, 10).cpu().numpy()
                sg = s.cpu().numpy()
                entry["%s_p%d" % (method, p)] = {
                    "ms": round(ms, 2), "info": int(info[0]), "R_1": float(res[0]), "R_10": float(res[9]),
                    "sigma_err_max_1_10": float(np.abs(sg[:10] - sig[:10]).max() / sig[0]),
                    "aprod_ms": round(ap["ms"], 2), "aprod_launches": ap["launches"],
                    "aprod_GB_per_s": round(ap["bytes"] / (ap["ms"] * 1e-3) / 1e9, 1) if ap["ms"] else None}
                del U, s, V
            del work, Q1
        out["m=%d" % m] = entry
        # compact view for the summary: LancSVD at the largest p
        best = entry["lancsvd_p%d" % max(ps)]
        entry["ms"], entry["R_1"], entry["R_10"] = best["ms"], best["R_1"], best["R_10"]
        del A
        torch.cuda.empty_cache()
    return out


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


def _fill_c3(cqr, torch, Y, seed):
    """The diagonally dominant workload in place: off-diagonal U[-0.5, 0.5),
    diagonal = off-diagonal |row| sum + 1."""
    cqr.synth_uniform(Y, seed, -0.5, 0.5)
    Y.diagonal().zero_()
    n = Y.shape[1]
    rs = torch.zeros(Y.shape[0], dtype=torch.float64, device=Y.device)
    for j in range(0, n, 4096):
        rs += Y[:, j:j + 4096].abs().sum(dim=1)
    Y.diagonal().copy_(rs + 1.0)


def hpl_residual(torch, Y, x, rhs) -> float:
    """||Y x - rhs||_inf / (||Y||_inf ||x||_inf n eps) over the whole matrix
    (a check, outside every timed region; Y is the unfactored input)."""
    n = Y.shape[0]
    r = torch.mv(Y, x) - rhs
    rs = torch.zeros(n, dtype=torch.float64, device=Y.device)
    for j in range(0, Y.shape[1], 4096):
        rs += Y[:, j:j + 4096].abs().sum(dim=1)
    return float(r.abs().max() / (rs.max() * x.abs().max() * n * 2.0 ** -52))


def _event_ms(torch, fn):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    out = fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), out


def tune_block_width(cqr, torch, Y, rhs, seed, cands) -> tuple:
    """Pick the FP64 block width: one untimed factorisation + solve per
    candidate, then one timed (HIP events) per candidate on a fresh copy of the
    same input.  Returns (best b, {b: ms})."""
    dev = Y.device
    n = Y.shape[0]
    R = cqr.colmajor(n, n, device=dev)
    swork = torch.empty(cqr.solve_workspace_size(n), dtype=torch.uint8, device=dev)
    works = {b: torch.empty(cqr.workspace_size(n, n, b), dtype=torch.uint8, device=dev) for b in cands}

    def run(b):
        Q, Rr, info, _ = cqr.qr_async(Y, b, R=R, work=works[b])
        return cqr.solve(Q, Rr, rhs, work=swork)

    times = {}
    for rep in range(2):
        for b in cands:
            cqr.synth_uniform(Y, seed)
            torch.cuda.synchronize()
            ms, _ = _event_ms(torch, lambda: run(b))
            if rep == 1:
                times[b] = round(ms, 2)
    del works, R, swork
    torch.cuda.empty_cache()
    best = min(times, key=lambda b: times[b])
    return best, times


def bench_fp64(args, torch, cqr, costmodel, inputs):
    """The FP64 factorisation + solve at n (the metric's workload)."""
    n, K, W = args.n, args.steps, args.warmup
    dev = torch.device("cuda:0")
    rhs = torch.empty(n, dtype=torch.float64, device=dev)
    cqr.synth_uniform(rhs.view(n, 1), args.seed + 1)

    # Inputs: one resident copy of Y per step (the factorisation overwrites it).
    Ys = []
    for _ in range(K + W):
        Y = cqr.colmajor(n, n, device=dev)
        cqr.synth_uniform(Y, args.seed)
        Ys.append(Y)
    if args.b > 0:
        b, tune = args.b, None
    else:
        cands = [int(v) for v in args.b_candidates.split(",")]
        b, tune = tune_block_width(cqr, torch, Ys[0], rhs, args.seed, cands)
        cqr.synth_uniform(Ys[0], args.seed)
    R = cqr.colmajor(n, n, device=dev)
    work = torch.empty(cqr.workspace_size(n, n, b), dtype=torch.uint8, device=dev)
    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    swork = torch.empty(cqr.solve_workspace_size(n), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step(i):
        Q, Rr, info, flags = cqr.qr_async(Ys[i], b, R=R, work=work)
        x = cqr.solve(Q, Rr, rhs, work=swork)
        return info, x

    for i in range(W):
        step(i)
    torch.cuda.synchronize()

    # Timed region: K steps, no per-launch profiling.
    t0 = time.perf_counter()
    infos = []
    x = None
    for i in range(W, W + K):
        info, x = step(i)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    infos = [int(v[0]) for v in infos]
    Qlast = Ys[W + K - 1]

    flops_step = costmodel.ca3(b, n, n) + costmodel.solve_flops(n)
    ms_step = 1e3 * elapsed / K
    value = flops_step / (elapsed / K) / 1e9

    # Separate profiled pass (HIP events around every launch, on the launch
    # stream) for the per-role breakdown and the dominant kernel's roofline.
    Yp = Ys[0]
    cqr.synth_uniform(Yp, args.seed)
    cqr.prof_reset()
    cqr.prof_enable(True)
    _, xp = step(0)
    torch.cuda.synchronize()
    cqr.prof_enable(False)
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
                "launches_per_step": d["launches"], "avg_launch_ms": round(d["ms"] / d["launches"], 4)}
    breakdown = {k: {"ms_per_step": round(v["ms"], 3), "launches_per_step": v["launches"],
                     "tflops": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 3) if v["flops"] else None}
                 for k, v in sorted(roles.items(), key=lambda kv: -kv[1]["ms"])}

    # Checks on the result: the profiled pass repeats the last timed step on
    # the same input, so its x must be the same bits; the HPL residual over
    # the whole (regenerated) matrix; orthogonality of sampled columns of Q.
    same_bits = bool(torch.equal(x, xp))
    Yc = Ys[1] if K + W > 1 else cqr.colmajor(n, n, device=dev)
    cqr.synth_uniform(Yc, args.seed)
    hpl = hpl_residual(torch, Yc, x, rhs)
    rng = np.random.default_rng(123)
    cols = torch.from_numpy(np.sort(rng.choice(n, size=min(n, 64), replace=False))).to(dev)
    Qc = Qlast[:, cols]
    orth = float((Qc.t() @ Qc - torch.eye(len(cols), dtype=torch.float64, device=dev)).abs().max())
    valid = all(v == 0 for v in infos) and hpl < 16.0 and same_bits
    del Ys, Yc, Qc, R, work, swork
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(ms_step, 2), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "FP64 CGS-QR (Algs. 3-5) + solve, n=%d, b=%d, U[-1,1] entries, 1 RHS" % (n, b),
                   "n": n, "b": b, "b_tuning_ms": tune, "rhs": 1, "seed": args.seed, "form": "fp64",
                   "flops_per_step": flops_step, "flop_model": "Table 1 CA3(b,n,n) + 3n^2"},
        "roofline": roofline,
        "breakdown": breakdown,
        "checks": {"valid": valid, "info": infos, "hpl_scaled_residual": hpl, "x_bits_repeatable": same_bits,
                   "max_offdiag_QtQ_64_sampled_cols": orth},
    }
    return out, b


def bench_c3(cqr, torch, n: int, b64: int, bmix: int, K: int, W: int, K64: int, seed: int) -> dict:
    """The diagonally dominant workload (off-diagonal U[-0.5, 0.5], diagonal =
    row sum of |.| + 1, RHS U[-1, 1]) through three forms on the same matrix:
    FP64 CGS-QR + solve, and BF16 / FP8 MFMA CGS-QR + FP64 iterative
    refinement.  Speed-ups are against the FP64 form on this matrix, and each
    low-precision x is compared with the FP64 form's x."""
    from paper_2403_06218_amd import costmodel
    dev = torch.device("cuda:0")
    Y = cqr.colmajor(n, n, device=dev)
    _fill_c3(cqr, torch, Y, seed + 17)
    rhs = torch.empty(n, dtype=torch.float64, device=dev)
    cqr.synth_uniform(rhs.view(n, 1), seed + 18)
    out = {"workload": "n=%d, off-diagonal U[-0.5,0.5], diagonal = row sum + 1, 1 RHS U[-1,1]" % n}

    # FP64 form on this matrix (the copy into the working buffer is not timed).
    Yw = cqr.colmajor(n, n, device=dev)
    R = cqr.colmajor(n, n, device=dev)
    work = torch.empty(cqr.workspace_size(n, n, b64), dtype=torch.uint8, device=dev)
    swork = torch.empty(cqr.solve_workspace_size(n), dtype=torch.uint8, device=dev)

    def fp64_step():
        Q, Rr, info, _ = cqr.qr_async(Yw, b64, R=R, work=work)
        return info, cqr.solve(Q, Rr, rhs, work=swork)

    times, infos = [], []
    x64 = None
    for i in range(1 + K64 if K64 > 0 else 0):
        Yw.copy_(Y)
        torch.cuda.synchronize()
        ms, (info, x64) = _event_ms(torch, fp64_step)
        if i:
            times.append(ms)
            infos.append(int(info[0]))
    fp64_ms = float(np.median(times)) if times else None
    flops = costmodel.ca3(b64, n, n) + costmodel.solve_flops(n)
    if fp64_ms:
        out["fp64"] = {"b": b64, "ms_per_step": round(fp64_ms, 2), "value": round(flops / (fp64_ms * 1e-3) / 1e9, 2),
                       "unit": "GFLOP/s", "info": infos, "hpl_scaled_residual": hpl_residual(torch, Y, x64, rhs)}
    del Yw, R, work, swork
    torch.cuda.empty_cache()

    Q = cqr.colmajor(n, n, device=dev, dtype=torch.float32)
    R = cqr.colmajor(n, n, device=dev, dtype=torch.float32)
    import ctypes
    for prec, name in ((cqr.PREC_BF16, "bf16"), (cqr.PREC_FP8, "fp8")):
        nb = ctypes.c_size_t(0)
        cqr._native.lib().cqr_workspace_size_mixed(n, n, bmix, prec, ctypes.byref(nb))
        work = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)

        def step():
            _, _, info, _ = cqr.qr_mixed_async(Y, bmix, prec=prec, Q=Q, R=R, work=work)
            x, iters, res = cqr.solve_ir(Y, Q, R, rhs, maxiter=50, tol=16.0)
            return info, iters, res, x

        for _ in range(W):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res_list = [step() for _ in range(K)]
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / K
        xm = res_list[-1][3]
        # Per-role launch times of one more factorisation (library HIP events).
        cqr.prof_reset()
        cqr.prof_enable(True)
        cqr.qr_mixed_async(Y, bmix, prec=prec, Q=Q, R=R, work=work)
        torch.cuda.synchronize()
        cqr.prof_enable(False)
        roles = {}
        for rn in cqr.prof_names():
            r = cqr.prof_query(rn)
            if r["launches"]:
                roles[rn] = {"ms": round(r["ms"], 3), "launches": r["launches"],
                             "tflops": round(r["flops"] / (r["ms"] * 1e-3) / 1e12, 2) if r["flops"] else None}
        fms = sum(v["ms"] for v in roles.values())
        lp = {k: v for k, v in roles.items() if k in ("proj", "update") and v["tflops"]}
        dom = max(lp, key=lambda k: lp[k]["ms"]) if lp else None
        peak = PEAK_BF16_MFMA_TFLOPS if prec == cqr.PREC_BF16 else PEAK_FP8_MFMA_TFLOPS
        roofline = ({"bound": "mfma", "kernel": dom, "achieved": lp[dom]["tflops"], "peak": peak, "unit": "TFLOP/s",
                     "frac": round(lp[dom]["tflops"] / peak, 4), "avg_launch_ms": round(lp[dom]["ms"] /
                                                                                       lp[dom]["launches"], 4)}
                    if dom else None)
        rel = float((xm - x64).abs().max() / x64.abs().max()) if x64 is not None else None
        out[name] = {"b": bmix, "value": round(flops / el / 1e9, 2), "unit": "GFLOP/s", "ms_per_step": round(el * 1e3, 2),
                     "speedup_vs_fp64_same_matrix": round(fp64_ms / (el * 1e3), 3) if fp64_ms else None,
                     "ir_iterations": [o[1] for o in res_list], "hpl_scaled_residual": [o[2] for o in res_list],
                     "info": [int(o[0][0]) for o in res_list], "max_rel_diff_x_vs_fp64_form": rel,
                     "roofline": roofline, "factor_ms_profiled": round(fms, 2),
                     "non_gemm_ms": round(sum(v["ms"] for k, v in roles.items() if k not in ("proj", "update")), 2),
                     "factor_breakdown": roles,
                     "dtype": ("bf16" if prec == cqr.PREC_BF16 else "fp8 e4m3 (per-column pow2 scales)")
                     + " mfma (fp32 acc) + f64 panel + f64 refinement"}
        del work
        torch.cuda.empty_cache()
    del Y, Q, R
    torch.cuda.empty_cache()
    return out


def summary(out: dict) -> dict:
    """The figures a reader needs first, gathered at the end of the line."""
    s = {}
    if out.get("value") is not None:
        s["fp64"] = {"gflops": out["value"], "b": out["config"].get("b"), "mfma_frac_dominant": out["roofline"]["frac"],
                     "frac_of_fp64_peak_end_to_end": round(out["value"] / 1e3 / PEAK_FP64_MFMA_TFLOPS, 4),
                     "hpl": out["checks"]["hpl_scaled_residual"], "valid": out["checks"]["valid"]}
    c3 = out.get("c3")
    if c3:
        s["c3_fp64_ms"] = c3["fp64"]["ms_per_step"] if "fp64" in c3 else None
        for k in ("bf16", "fp8"):
            if k in c3:
                v = c3[k]
                s["c3_" + k] = {"ms": v["ms_per_step"], "speedup_vs_fp64": v["speedup_vs_fp64_same_matrix"],
                                "hpl_max": max(v["hpl_scaled_residual"]), "iters": max(v["ir_iterations"]),
                                "rel_dx": v["max_rel_diff_x_vs_fp64_form"],
                                "mfma_frac": v["roofline"]["frac"] if v["roofline"] else None}
    bt = out.get("batched")
    if bt:
        for k in ("f64", "f32"):
            if k in bt:
                s["batched_" + k] = {"ms": bt[k]["ms_per_batch"], "mfma_frac": bt[k]["roofline"]["frac"]}
    ad = out.get("adjoint")
    if ad:
        for k in ("f64", "f32"):
            if k in ad:
                s["adjoint_" + k] = {"fwd_ms": ad[k]["forward_ms"], "bwd_ms": ad[k]["backward_ms"],
                                     "bwd_hbm_frac": ad[k]["backward_roofline"]["frac"]}
    ts = out.get("tall_skinny")
    if ts and "q=1000000" in ts:
        s["tall_q1e6_hbm_frac"] = ts["q=1000000"]["frac_hbm"]
    sv = out.get("lancsvd")
    if sv:
        s["lancsvd"] = {k: {"ms": v["ms"], "R1": v["R_1"], "R10": v["R_10"]} for k, v in sv.items() if k.startswith("m=")}
    return s


def counters_only(args, torch, cqr):
    """One step of each form with nothing else around it, for hardware
    counter passes (rocprofv3 --pmc), which need few launches per run."""
    n, b = args.n, (args.b if args.b > 0 else 128)
    dev = torch.device("cuda:0")
    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    Y = cqr.colmajor(n, n, device=dev)
    rhs = torch.empty(n, dtype=torch.float64, device=dev)
    cqr.synth_uniform(rhs.view(n, 1), args.seed + 1)
    if not args.no_fp64:
        cqr.synth_uniform(Y, args.seed)
        Q, R, info, _ = cqr.qr_async(Y, b)
        cqr.solve(Q, R, rhs)
        torch.cuda.synchronize()
        del R
        print("counters-only: fp64 n=%d b=%d info=%d" % (n, b, int(info[0])), flush=True)
    if not args.no_mixed:
        _fill_c3(cqr, torch, Y, args.seed + 17)
        for prec in (cqr.PREC_BF16, cqr.PREC_FP8):
            _, _, info, _ = cqr.qr_mixed_async(Y, args.mixed_b, prec=prec)
            torch.cuda.synchronize()
            print("counters-only: prec=%d n=%d b=%d info=%d" % (prec, n, args.mixed_b, int(info[0])), flush=True)
    if not args.no_batched:
        # The batched form's workload, one eager call per element type with
        # the library's default plan.
        del Y, rhs
        torch.cuda.empty_cache()
        from paper_2403_06218_amd import batched, inputs
        sizes = inputs.batch_sizes(10000, 8, 256, seed=args.seed)
        for dt in (torch.float64, torch.float32):
            batch = batched.PackedBatch(sizes, dtype=dt)
            batched._fill(batch, args.seed + 100)
            work = torch.empty(max(batched.workspace_size(batch.count), 1), dtype=torch.uint8, device=dev)
            batched.factor_solve(batch, work)
            torch.cuda.synchronize()
            print("counters-only: batched %s, %d matrices, %d fallbacks" % (
                dt, batch.count, int((batch.info > 0).sum())), flush=True)
            del batch, work


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2403_06218_amd as cqr
    from paper_2403_06218_amd import costmodel, inputs

    n, K, W = args.n, args.steps, args.warmup
    torch.cuda.set_device(torch.device("cuda:0"))
    if args.counters_only:
        counters_only(args, torch, cqr)
        return
    if args.no_tiled:
        cqr.set_mixed_layout(False)
    if args.no_fp64:
        b = args.b if args.b > 0 else 128
        out = {"metric": METRIC, "value": None, "unit": "GFLOP/s", "n_gpus": 1, "steps": K, "warmup": W,
               "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64", "data": "synthetic", "config": {"workload": "sub-benchmarks only (--no-fp64)"}}
    else:
        out, b = bench_fp64(args, torch, cqr, costmodel, inputs)
    if not args.no_mixed:
        torch.cuda.empty_cache()
        out["c3"] = bench_c3(cqr, torch, args.c3_n or n, b, args.mixed_b, K, W, args.c3_fp64_steps, args.seed)
    if not args.no_batched:
        out["batched"] = bench_batched(torch, K, W, args.seed, not args.no_tune)
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(torch, K, W, args.seed)
    if not args.no_tall:
        out["tall_skinny"] = bench_tall(cqr, torch, K, W, args.seed)
    if not args.no_svd:
        out["lancsvd"] = bench_lancsvd(torch, args.seed, [int(v) for v in args.svd_m.split(",")],
                                       [int(v) for v in args.svd_p.split(",")])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, b, args.seed, args.cpu_target_s)
    out["summary"] = summary(out)
    print(json.dumps(out), flush=True)
    if out.get("value") is not None and not out["checks"]["valid"]:
        print("bench.py: the FP64 result failed its checks (info, HPL residual < 16, repeatable bits)",
              file=sys.stderr)
        sys.exit(3)


if __name__ == "__main__":
    main()
