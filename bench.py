"""Benchmark: RPCA background modelling by ADMM with CPA singular value
shrinkage on one MI355X.

Workload: a 1024 x 1024 synthetic frame matrix (rank-40 background from U(0,1)
factors min-max normalised to [0,1], plus 5% additive U(-1,1) outliers), soft
shrinkage tau = 1/rho = 10, eta/rho = 10/32, K = 30 Chebyshev terms, power
iteration bound warm-started across iterations.  One step = one ADMM
iteration = one full shrink (Gram, bound, coefficients, 29 recurrence GEMMs)
plus the elementwise ADMM updates.  Inputs are resident in HBM before timing.

Prints one JSON line (see the repository's benchmark contract)."""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

M = N = 1024
K = 30
INV_RHO = 10.0
ETA_OVER_RHO = 10.0 / 32.0
MFMA_FP32_PEAK_TFLOPS = 157.3
METRIC = "shrunk matrices/sec & TFLOP/s at rel. Frobenius err ≤1e-3 vs FP64 SVT"


def cpu_baseline(I, budget_s: float = 15.0):
    """The FP64 oracle's ADMM iterations on the host, for about budget_s seconds."""
    import numpy as np
    from oracle import drivers
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    X = I.astype(np.float64)
    t0 = time.perf_counter()
    done = 0
    # run growing batches of iterations from the same start until the budget is used
    while True:
        drivers.rpca_admm(X, INV_RHO, ETA_OVER_RHO, 1, K)
        done += 1
        el = time.perf_counter() - t0
        if el >= budget_s or done >= 50:
            break
    return {"value": done / el, "unit": "matrices/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{done} FP64 oracle ADMM iterations (one shrink each: Algorithm 1 H-form, "
                      f"K={K}, 1024x1024) in {el:.1f} s"}


def bench_batched(cpa, torch, np, synth, timed_runs: int = 5):
    """Batched weighted soft shrinkage of 8192 patch-group matrices (64 x U{40..120},
    rank 4 + N(0, 0.2^2)), K = 16, per-matrix power bound, one persistent launch."""
    import math
    flat, ms, ns, offs, _, _ = synth.patch_groups(batch=8192)
    dev = torch.device("cuda:0")
    sig = 0.2
    recs = []
    for nj in ns:
        wc = 2 * math.sqrt(2) * sig * sig * math.sqrt(float(nj))
        wsg = (8.0 + math.sqrt(float(nj))) ** 2 * sig * sig
        recs.append(cpa.weighted_fn(wc, wsg, 1e-6))
    rec_t = torch.frombuffer(bytearray(cpa.shrinkage_records(recs)), dtype=torch.uint8).to(dev)
    X = torch.from_numpy(flat).to(dev)
    m = torch.from_numpy(ms).to(dev)
    n = torch.from_numpy(ns).to(dev)
    off = torch.from_numpy(offs).to(dev)
    lam = torch.zeros(len(ms), dtype=torch.float64, device=dev)
    opts = cpa.Opts(K=16)
    Y = torch.empty_like(X)
    for _ in range(2):
        cpa.shrink_batched(X, m, n, off, cpa.soft(0.0), opts, shrink_per_matrix=rec_t, out=Y, lambda_out=lam)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(timed_runs):
        cpa.shrink_batched(X, m, n, off, cpa.soft(0.0), opts, shrink_per_matrix=rec_t, out=Y, lambda_out=lam)
    e1.record()
    torch.cuda.synchronize()
    ms_batch = e0.elapsed_time(e1) / timed_runs
    d = np.minimum(ms, ns).astype(np.float64)
    e = np.maximum(ms, ns).astype(np.float64)
    flop = float(np.sum(16 * 2.0 * d * d * e))
    # baseline: the same matrices through per-matrix dense calls (first 128, FP32, power bound)
    nb = 128
    Xs = [X[int(offs[i]):int(offs[i]) + int(ms[i] * ns[i])].view(int(ms[i]), int(ns[i])) for i in range(nb)]
    outs = [torch.empty_like(x) for x in Xs]
    for i in range(8):
        cpa.shrink_dense(Xs[i], recs[i], opts, out=outs[i])
    torch.cuda.synchronize()
    e0.record()
    for i in range(nb):
        cpa.shrink_dense(Xs[i], recs[i], opts, out=outs[i])
    e1.record()
    torch.cuda.synchronize()
    ms_single = e0.elapsed_time(e1) / nb
    # accuracy on a sample: vs the FP64 CPA at the device bound, and vs exact SVT
    from oracle import cpa as ocpa
    from oracle import exact, metrics
    from oracle.shrinkage import Shrinkage
    Yh = Y.cpu().numpy()
    lamh = lam.cpu().numpy()
    e_cpa, e_svt = [], []
    for i in range(0, 8192, 256):
        Xi = flat[offs[i]:offs[i] + ms[i] * ns[i]].reshape(ms[i], ns[i]).astype(np.float64)
        Yi = Yh[offs[i]:offs[i] + ms[i] * ns[i]].reshape(ms[i], ns[i]).astype(np.float64)
        r = recs[i]
        sh = Shrinkage(3, 0.0, r.w_c, r.w_sigma, r.w_eps)
        e_cpa.append(metrics.rel_fro(Yi, ocpa.cpa_shrink(Xi, sh, float(lamh[i]), 16), Xi))
        e_svt.append(metrics.rel_fro(Yi, exact.svt_svd(Xi, sh), Xi))
    return {
        "workload": "8192 patch groups 64 x U{40..120}, rank 4 + N(0,0.2^2), weighted soft, K=16, power bound",
        "value": round(8192 / (ms_batch / 1e3), 1), "unit": "matrices/s", "ms_per_batch": round(ms_batch, 4),
        "tflops": round(flop / (ms_batch * 1e-3) / 1e12, 3),
        "baseline_per_matrix_dense_fp32": {"value": round(1e3 / ms_single, 1), "unit": "matrices/s",
                                           "sample": f"{nb} matrices, one cpa_shrink_dense call each"},
        "err_vs_fp64_cpa_max": float("%.3e" % max(e_cpa)),
        "err_vs_fp64_svt_median": float("%.3e" % float(np.median(e_svt))),
        "err_vs_fp64_svt_max": float("%.3e" % max(e_svt)),
    }


def bench_sparse(cpa, torch, np, synth):
    """Sparse completion-shaped shrink: S 20000 x 4000 with 2% observed entries (CSR,
    1.6M nonzeros) of a rank-10 N(0,1) product, K = 25, soft tau = 0.5 sqrt(Lambda),
    operator form (W = S^T Y_k, then S W with the fused recurrence update)."""
    m, n, K = 20000, 4000, 25
    _, _, rowptr, cols, vals = synth.completion()
    dev = torch.device("cuda:0")
    r = torch.from_numpy(rowptr).to(dev)
    c = torch.from_numpy(cols).to(dev)
    v = torch.from_numpy(vals).to(dev)
    out = torch.empty((m, n), device=dev, dtype=torch.float32)
    _, info = cpa.shrink_csr(m, n, r, c, v, cpa.soft(1.0), cpa.Opts(K=2), out=out, info=True)
    tau = 0.5 * (info["Lambda"] / 1.01) ** 0.5
    opts = cpa.Opts(K=K, warm_start=True)
    cpa.shrink_csr(m, n, r, c, v, cpa.soft(tau), opts, out=out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record()
    for _ in range(reps):
        cpa.shrink_csr(m, n, r, c, v, cpa.soft(tau), opts, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms_shrink = e0.elapsed_time(e1) / reps
    cpa.timing_enable(True)
    cpa.shrink_csr(m, n, r, c, v, cpa.soft(tau), opts, out=out)
    torch.cuda.synchronize()
    step_ms, steps = cpa.timing_read("recurrence")
    cpa.timing_enable(False)
    nnz = int(vals.size)
    dense = 4.0 * m * n
    # algorithmic bytes of a middle step: S^T Y_k reads Y_k and the transposed pattern
    # (row, source position, value), writes W; S W reads the CSR pattern and W, reads
    # Y_k, Y_{k-1} and the accumulator, writes the accumulator and Y_{k+1}
    step_bytes = (dense + 12.0 * nnz + 4.0 * n * n) + (8.0 * nnz + 4.0 * n * n + 5 * dense)
    avg_step_us = 1e3 * step_ms / max(steps, 1)
    return {
        "workload": "CSR 20000 x 4000, 1.6M nonzeros (2%), rank-10 N(0,1) values, soft, K=25, operator form",
        "ms_per_shrink": round(ms_shrink, 3), "shrinks_per_s": round(1e3 / ms_shrink, 2),
        "spmm_pair_avg_us": round(avg_step_us, 1),
        "roofline": {"bound": "hbm", "achieved": round(step_bytes / (avg_step_us * 1e-6) / 1e9, 1),
                     "peak": 8000.0, "unit": "GB/s",
                     "frac": round(step_bytes / (avg_step_us * 1e-6) / 1e9 / 8000.0, 4),
                     "bytes_per_step": step_bytes, "traffic": None},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-sparse", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1705_07112_amd as cpa
    import synth

    dev = torch.device("cuda:0")
    I, _, _ = synth.rpca_frames(M, N)
    Id = torch.from_numpy(I).to(dev)
    opts = cpa.Opts(K=K, warm_start=True, power_iters=100)
    run = cpa.RpcaAdmm(Id, INV_RHO, ETA_OVER_RHO, opts)
    Et = torch.zeros(args.warmup + args.steps, dtype=torch.float64, device=dev)
    if args.warmup:
        run.iterate(args.warmup, Et[:args.warmup])
    torch.cuda.synchronize()

    # timed region: `steps` ADMM iterations, replayed from the library's captured graph
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    run.iterate(args.steps, Et[args.warmup:])
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)

    # roofline pass: the same iterations again with every GEMM launch bracketed by
    # HIP events on the launch stream (event timing needs direct launches)
    cpa.timing_enable(True)
    run.iterate(args.steps)
    torch.cuda.synchronize()
    rec_ms, rec_n = cpa.timing_read("recurrence")
    gram_ms, gram_n = cpa.timing_read("gram")
    cpa.timing_enable(False)

    flop_gemm = 2.0 * M * N * min(M, N)
    flop_shrink = K * flop_gemm            # Gram + (K-1) recurrence products
    ms_per_step = ms / args.steps
    value = args.steps / (ms / 1e3)
    rec_avg_us = 1e3 * rec_ms / max(rec_n, 1)
    achieved = flop_gemm / (rec_avg_us * 1e-6) / 1e12

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "matrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rpca_admm_1024x1024_rank40_outliers5pct_soft_K30",
                   "m": M, "n": N, "K": K, "inv_rho": INV_RHO, "eta_over_rho": ETA_OVER_RHO,
                   "bound": "power, warm-started", "parallelism": "single GPU"},
        "tflops": round(flop_shrink * value / 1e12, 3),
        "wall_s_timed": round(wall, 4),
        "roofline": {"bound": "mfma", "kernel": "recurrence GEMM (FP32 MFMA, fused Chebyshev epilogue)",
                     "achieved": round(achieved, 3), "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / MFMA_FP32_PEAK_TFLOPS, 4), "traffic": None,
                     "avg_launch_us": round(rec_avg_us, 3), "launches": rec_n,
                     "flop_per_launch": flop_gemm,
                     "timing": "HIP events around each launch, same workload, pass right after the timed region",
                     "gram_avg_us": round(1e3 * gram_ms / max(gram_n, 1), 3)},
    }

    # the same workload with the split-precision recurrence (bf16 hi + lo)
    run2 = cpa.RpcaAdmm(Id, INV_RHO, ETA_OVER_RHO, cpa.Opts(K=K, warm_start=True, power_iters=100, precision="bf16x3"))
    run2.iterate(args.warmup)
    torch.cuda.synchronize()
    t0.record()
    run2.iterate(args.steps)
    t1.record()
    torch.cuda.synchronize()
    ms2 = t0.elapsed_time(t1)
    cpa.timing_enable(True)
    run2.iterate(args.steps)
    torch.cuda.synchronize()
    rec2_ms, rec2_n = cpa.timing_read("recurrence")
    cpa.timing_enable(False)
    out["bf16x3"] = {"value": round(args.steps / (ms2 / 1e3), 3), "ms_per_step": round(ms2 / args.steps, 4),
                     "recurrence_avg_us": round(1e3 * rec2_ms / max(rec2_n, 1), 3),
                     "note": "same ADMM workload; recurrence products as bf16 hi/lo x3 on the BF16 matrix cores"}

    if not args.no_accuracy:
        # errors of one shrink of the current ADMM iterate (L + U1) on the device
        from oracle import cpa as ocpa
        from oracle import exact, metrics
        from oracle.shrinkage import Shrinkage
        Xd = (run.block(0) + run.block(4)).contiguous()
        Yd, info = cpa.shrink_dense(Xd, cpa.soft(INV_RHO), cpa.Opts(K=K), info=True)
        X64 = Xd.cpu().numpy().astype(np.float64)
        Y = Yd.cpu().numpy().astype(np.float64)
        sh = Shrinkage(0, INV_RHO)
        out["err_vs_fp64_cpa"] = float("%.3e" % metrics.rel_fro(Y, ocpa.cpa_shrink(X64, sh, info["Lambda"], K), X64))
        out["err_vs_fp64_svt"] = float("%.3e" % metrics.rel_fro(Y, exact.svt_svd(X64, sh), X64))
        Y2 = cpa.shrink_dense(Xd, cpa.soft(INV_RHO), cpa.Opts(K=K, Lambda=info["Lambda"], precision="bf16x3"))
        out["bf16x3"]["err_vs_fp64_cpa"] = float("%.3e" % metrics.rel_fro(
            Y2.cpu().numpy().astype(np.float64), ocpa.cpa_shrink(X64, sh, info["Lambda"], K), X64))
        out["E_t_last"] = float("%.3e" % Et[-1].item())

    if not args.no_batched:
        out["batched"] = bench_batched(cpa, torch, np, synth)

    if not args.no_sparse:
        out["sparse"] = bench_sparse(cpa, torch, np, synth)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(I)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
