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
SAMPLES = {}   # GPU results of the other legs kept for the oracle leg's FP64 CPA comparison
# Lanczos steps of the batched leg's bound: on 400 patch groups drawn like the leg's, 8 steps
# reach the largest eigenvalue to 2e-15 relative (the bound then adds its 1% margin)
LANCZOS_STEPS_BATCHED = 8


def cpu_baseline(I, budget_s: float = 15.0, check=None, samples=None):
    """The FP64 oracle's ADMM iterations on the host, for about budget_s seconds.

    check: optional (X, {name: Y_gpu}, Lambda) -- one shrink input, GPU results
    and the bound they used; the oracle's CPA of X at that bound (untimed) gives
    each result's relative Frobenius error against FP64 Algorithm 1.
    samples: optional {leg: [(X, Y_gpu, (kind, tau, w_c, w_sigma, w_eps), Lambda, K), ...]};
    the largest such error over each leg's sample is reported as well."""
    import numpy as np
    from oracle import drivers
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    X = I.astype(np.float64)

    def timed(budget, cap):
        # one ADMM iteration from the start state per call, until the budget is used
        t0 = time.perf_counter()
        done = 0
        while True:
            drivers.rpca_admm(X, INV_RHO, ETA_OVER_RHO, 1, K)
            done += 1
            el = time.perf_counter() - t0
            if el >= budget or done >= cap:
                return done, el

    done, el = timed(budget_s, 50)
    with threadpool_limits(limits=1):
        done1, el1 = timed(0.8 * budget_s, 8)
    cpu_model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    res = {"value": done / el, "unit": "matrices/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{done} FP64 oracle ADMM iterations (one shrink each: Algorithm 1 H-form, "
                     f"K={K}, 1024x1024) in {el:.1f} s on {threads} BLAS threads",
           "single_thread": {"value": done1 / el1, "unit": "matrices/s", "cores": 1,
                             "sample": f"{done1} of the same iterations in {el1:.1f} s, BLAS limited to one thread"},
           "cpu_model": cpu_model, "host_cpus": os.cpu_count()}
    if check is not None:
        from oracle import cpa as ocpa
        from oracle import metrics
        from oracle.shrinkage import Shrinkage
        Xc, outs, lam = check
        ref = ocpa.cpa_shrink(Xc, Shrinkage(0, INV_RHO), lam, K)
        res["err_vs_fp64_cpa"] = {k: float("%.3e" % metrics.rel_fro(v, ref, Xc)) for k, v in outs.items()}
    if samples:
        from oracle import cpa as ocpa
        from oracle import metrics
        from oracle.shrinkage import Shrinkage
        worst = {}
        for leg, items in samples.items():
            e = 0.0
            for Xs, Ys, sh, lam_s, K_s in items:
                ref = ocpa.cpa_shrink(Xs, Shrinkage(*sh), lam_s, K_s)
                e = max(e, metrics.rel_fro(Ys, ref, Xs))
            worst[leg] = {"max": float("%.3e" % e), "matrices": len(items)}
        res["err_vs_fp64_cpa_samples"] = worst
    return res


def measured_traffic(path: str = os.path.join(ROOT, "profiles", "piece_gemm_f32_1024_K30_pmc_traffic.md")):
    """HBM bytes per launch of the symmetric piece product from its committed counter summary,
    or None when the summary is missing or the kernel source changed since."""
    import hashlib
    try:
        fields = {}
        for line in open(path):
            if ":" in line and line.startswith("    ") and not line.strip().startswith("rocprofv3"):
                k, v = line.strip().split(":", 1)
                fields[k.strip()] = v.strip()
        # one or more source files (comma-separated), hashed in order as one byte string
        h = hashlib.sha256()
        for src in fields["kernel_source"].split(","):
            h.update(open(os.path.join(ROOT, src.strip()), "rb").read())
        if h.hexdigest() != fields["kernel_source_sha256"]:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def exact_shrink(X, g):
    """U g(Sigma) V^T by LAPACK's SVD in FP64 (the definition of singular value shrinkage)."""
    import numpy as np
    U, sv, Vt = np.linalg.svd(X, full_matrices=False)
    return (U * g(sv)) @ Vt


def rel_fro(A, B, scale):
    """||A - B||_F / ||scale||_F (the accuracy legs pass the reference itself as scale)."""
    import numpy as np
    d = float(np.linalg.norm(scale))
    return float(np.linalg.norm(A - B)) / (d if d > 0 else 1.0)


K_METRIC = 512


def bench_metric_order(cpa, torch, np, Id, args):
    """RPCA ADMM of the headline workload at K = K_METRIC, with the error of its shrink
    against the exact soft shrinkage at the start and the end of the timed window."""
    def shrink_error(run):
        Xd = (run.block(0) + run.block(4)).contiguous()
        Y = cpa.shrink_dense(Xd, cpa.soft(INV_RHO), cpa.Opts(K=K_METRIC)).cpu().numpy().astype(np.float64)
        X64 = Xd.cpu().numpy().astype(np.float64)
        ex = exact_shrink(X64, lambda sv: np.maximum(sv - INV_RHO, 0.0))
        return rel_fro(Y, ex, ex)

    run = cpa.RpcaAdmm(Id, INV_RHO, ETA_OVER_RHO, cpa.Opts(K=K_METRIC, warm_start=True, power_iters=100))
    Et = torch.zeros(max(args.warmup, args.steps, 1), dtype=torch.float64, device=Id.device)
    run.iterate(max(args.warmup, 1), Et)
    torch.cuda.synchronize()
    e0 = shrink_error(run)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    run.iterate(args.steps, Et)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    e1 = shrink_error(run)
    s_ps = math.isqrt(K_METRIC - 1) + 1
    j_ps = -(-K_METRIC // s_ps)
    return {"K": K_METRIC, "value": round(args.steps / (ms / 1e3), 3), "unit": "matrices/s",
            "ms_per_step": round(ms / args.steps, 4),
            "err_vs_fp64_svt": [float("%.3e" % e0), float("%.3e" % e1)],
            "meets_metric": bool(max(e0, e1) <= 1e-3),
            "products_per_shrink": 1 + (s_ps - 1) + (j_ps - 1) + 1,
            "note": "same ADMM workload at the order whose CPA is within 1e-3 of the exact shrinkage (errors on "
                    "the iterates opening and closing the timed window); matrix-polynomial route, "
                    f"s={s_ps}, J={j_ps}"}


def bench_designs(cpa, torch, np, Xd, X64, ex, Lam, orders=(10, 20, 30, 50)):
    """Other polynomial designs against CPA on the ADMM iterate (Sec. IV-B: least squares
    and minimax, eq. l_p_norm_for_approximation): host FP64 coefficients
    (cpa_design_coeffs) run through the same device evaluation (opts.coeffs) at the
    same bound; error against the exact soft shrinkage, host design time, device time."""
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    out = {}
    for K in orders:
        row = {}
        for kind in ("chebyshev", "lsq", "minimax"):
            w0 = time.perf_counter()
            c, resp_err = cpa.design_coeffs(cpa.soft(INV_RHO), Lam, K, kind)
            design_ms = 1e3 * (time.perf_counter() - w0)
            cd = torch.from_numpy(c).to(Xd.device)
            o = cpa.Opts(K=K, bound="given", Lambda=Lam, coeffs=cd)
            Y = cpa.shrink_dense(Xd, cpa.soft(INV_RHO), o)
            torch.cuda.synchronize()
            t0.record()
            for _ in range(5):
                cpa.shrink_dense(Xd, cpa.soft(INV_RHO), o)
            t1.record()
            torch.cuda.synchronize()
            err = rel_fro(Y.cpu().numpy().astype(np.float64), ex, ex)
            row[kind] = {"err_vs_fp64_svt": float("%.3e" % err), "response_err": float("%.3e" % resp_err),
                         "design_ms": round(design_ms, 3), "shrink_ms": round(t0.elapsed_time(t1) / 5, 4)}
        out[f"K{K}"] = row
    out["note"] = ("soft shrinkage of the 1024 x 1024 ADMM iterate at its device bound; 'chebyshev' is CPA; "
                   "lsq over 2000 uniform samples of [0, Lambda], minimax on an 8000-point Chebyshev-spaced grid "
                   "(Remez); response_err: largest |h - p| on the design's own points (0 at CPA's nodes); "
                   "same kernels for all three (given coefficients)")
    return out


def bench_batched(cpa, torch, np, synth, timed_runs: int = 10, main_only: bool = False):
    """Batched weighted soft shrinkage of 8192 patch-group matrices (64 x U{40..120},
    rank 4 + N(0, 0.2^2)), K = 16, per-matrix bound: one persistent launch,
    captured in a graph after the autotuner picked its configuration.  Main figure:
    split-precision products (bf16 hi/lo x3, FP32 accumulation) with the 8-step
    Lanczos bound; beside it the power-iteration bound (tol 1e-7) and FP32
    products with either bound, and the largest relative difference between the
    two bounds over the batch."""
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
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def run_plan(precision, bound="lanczos"):
        lam = torch.zeros(len(ms), dtype=torch.float64, device=dev)
        # a fixed number of Lanczos steps (power_tol = 0: no per-step Ritz test)
        kw = {"bound": "lanczos", "lanczos_steps": LANCZOS_STEPS_BATCHED, "power_tol": 0.0} if bound == "lanczos" else {}
        plan = cpa.BatchedPlan(X, m, n, off, cpa.soft(0.0), cpa.Opts(K=16, precision=precision, **kw),
                               shrink_per_matrix=rec_t, lambda_out=lam)
        plan.run()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(timed_runs):
            plan.run()
        e1.record()
        torch.cuda.synchronize()
        ms_b = e0.elapsed_time(e1) / timed_runs
        tun = plan.tuning
        Yh = plan.out.cpu().numpy()
        plan.close()
        return ms_b, tun, Yh, lam

    ms_split, tun_split, Ysh, lam_sp = run_plan("bf16x3")
    if main_only:   # the main plan alone (for counter runs)
        return {"workload": "8192 patch groups, K=16, split precision, 8-step Lanczos bound (main plan only)",
                "value": round(8192 / (ms_split / 1e3), 1), "unit": "matrices/s", "ms_per_batch": round(ms_split, 4)}
    ms_32, tun_32, Yh, lam = run_plan("fp32")
    ms_split_p, tun_split_p, Ysh_p, lam_sp_p = run_plan("bf16x3", "power")
    ms_32_p, tun_32_p, _, _ = run_plan("fp32", "power")
    rel = torch.abs(lam_sp - lam_sp_p) / lam_sp_p
    lam_diff = float(torch.max(rel).item())
    # the matrix where the two bounds differ most, against its largest eigenvalue (LAPACK)
    iw = int(torch.argmax(rel).item())
    Xw = flat[offs[iw]:offs[iw] + ms[iw] * ns[iw]].reshape(ms[iw], ns[iw]).astype(np.float64)
    lmax_w = float(np.linalg.eigvalsh(Xw.T @ Xw if ms[iw] >= ns[iw] else Xw @ Xw.T)[-1])
    lam_worst = {"matrix": iw, "lanczos_over_lambda_max": round(float(lam_sp[iw].item()) / lmax_w, 6),
                 "power_over_lambda_max": round(float(lam_sp_p[iw].item()) / lmax_w, 6)}
    d = np.minimum(ms, ns).astype(np.float64)
    e = np.maximum(ms, ns).astype(np.float64)
    flop = float(np.sum(16 * 2.0 * d * d * e))
    # baseline: the same matrices through per-matrix dense calls (first 128, FP32, power bound)
    opts = cpa.Opts(K=16)
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
    # accuracy on a sample against the exact weighted shrinkage (LAPACK SVD):
    # g(s) = s - w(s^2) when s > w(s^2), w(x) = w_c / (sqrt(max(x - w_sigma, 0)) + w_eps)
    e_svt, e_svt_split, e_svt_split_p = [], [], []
    for i in range(0, 8192, 256):
        Xi = flat[offs[i]:offs[i] + ms[i] * ns[i]].reshape(ms[i], ns[i]).astype(np.float64)
        Yi = Yh[offs[i]:offs[i] + ms[i] * ns[i]].reshape(ms[i], ns[i]).astype(np.float64)
        Ys = Ysh[offs[i]:offs[i] + ms[i] * ns[i]].reshape(ms[i], ns[i]).astype(np.float64)
        Ysp = Ysh_p[offs[i]:offs[i] + ms[i] * ns[i]].reshape(ms[i], ns[i]).astype(np.float64)
        r = recs[i]

        def g(sv, r=r):
            w = r.w_c / (np.sqrt(np.maximum(sv * sv - r.w_sigma, 0.0)) + r.w_eps)
            return np.where(sv > w, sv - w, 0.0)
        ex = exact_shrink(Xi, g)
        e_svt.append(rel_fro(Yi, ex, ex))
        e_svt_split.append(rel_fro(Ys, ex, ex))
        e_svt_split_p.append(rel_fro(Ysp, ex, ex))
        rec = (3, 0.0, r.w_c, r.w_sigma, r.w_eps)
        SAMPLES.setdefault("batched_fp32", []).append((Xi, Yi, rec, float(lam[i].item()), 16))
        SAMPLES.setdefault("batched_bf16x3", []).append((Xi, Ys, rec, float(lam_sp[i].item()), 16))

    def tun_rec(t):
        return {"grid": t["grid"], "pair": t["pair"], "order": t["order"], "candidates": t["candidates"],
                "tuned_us": round(t["best_us"], 1), "untuned_us": round(t["default_us"], 1)}
    return {
        "workload": "8192 patch groups 64 x U{40..120}, rank 4 + N(0,0.2^2), weighted soft, K=16, "
                    f"{LANCZOS_STEPS_BATCHED}-step Lanczos bound (all steps, no early stop)",
        "precision": "bf16x3 (split products, FP32 accumulation)",
        "value": round(8192 / (ms_split / 1e3), 1), "unit": "matrices/s", "ms_per_batch": round(ms_split, 4),
        "tflops": round(flop / (ms_split * 1e-3) / 1e12, 3),
        "launch": "one persistent launch per batch, replayed from a captured graph",
        "autotuner": tun_rec(tun_split),
        "err_vs_fp64_svt_median": float("%.3e" % float(np.median(e_svt_split))),
        "err_vs_fp64_svt_max": float("%.3e" % max(e_svt_split)),
        "bound_rel_diff_lanczos_vs_power_max": float("%.3e" % lam_diff),
        "bound_worst_matrix": lam_worst,
        "power_bound": {"value": round(8192 / (ms_split_p / 1e3), 1), "unit": "matrices/s",
                        "ms_per_batch": round(ms_split_p, 4), "autotuner": tun_rec(tun_split_p),
                        "note": "the same split plan with the power-iteration bound (power_tol 1e-7, at most 100 "
                                "products)",
                        "err_vs_fp64_svt_median": float("%.3e" % float(np.median(e_svt_split_p))),
                        "fp32_value": round(8192 / (ms_32_p / 1e3), 1)},
        "fp32": {"value": round(8192 / (ms_32 / 1e3), 1), "unit": "matrices/s", "ms_per_batch": round(ms_32, 4),
                 "tflops": round(flop / (ms_32 * 1e-3) / 1e12, 3), "autotuner": tun_rec(tun_32),
                 "err_vs_fp64_svt_median": float("%.3e" % float(np.median(e_svt))),
                 "err_vs_fp64_svt_max": float("%.3e" % max(e_svt))},
        "baseline_per_matrix_dense_fp32": {"value": round(1e3 / ms_single, 1), "unit": "matrices/s",
                                           "sample": f"{nb} matrices, one cpa_shrink_dense call each"},
    }


def bench_sparse(cpa, torch, np, synth):
    """Sparse completion-shaped shrink: S 20000 x 4000 with 2% observed entries (CSR,
    1.6M nonzeros) of a rank-10 N(0,1) product, K = 25, soft tau = 0.5 sqrt(Lambda).
    Main figure: the default route (matrix polynomial: Gram S^T S by one sparse
    product, the polynomial on the 4000 x 4000 side, one product S p).  Beside it:
    the operator-form recurrence (W = S^T Y_k, then S W with the fused update)."""
    m, n, K = 20000, 4000, 25
    u_f, v_f, rowptr, cols, vals = synth.completion()
    dev = torch.device("cuda:0")
    r = torch.from_numpy(rowptr).to(dev)
    c = torch.from_numpy(cols).to(dev)
    v = torch.from_numpy(vals).to(dev)
    out = torch.empty((m, n), device=dev, dtype=torch.float32)
    _, info = cpa.shrink_csr(m, n, r, c, v, cpa.soft(1.0), cpa.Opts(K=2), out=out, info=True)
    tau = 0.5 * (info["Lambda"] / 1.01) ** 0.5
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    res = {}
    for ev in ("auto", "recurrence"):
        opts = cpa.Opts(K=K, warm_start=True, eval=ev)
        cpa.shrink_csr(m, n, r, c, v, cpa.soft(tau), opts, out=out)
        torch.cuda.synchronize()
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
        tot_ms, launches = cpa.timing_read("recurrence")
        cpa.timing_enable(False)
        res[ev] = (ms_shrink, 1e3 * tot_ms / max(launches, 1), launches)
    nnz = int(vals.size)
    dense = 4.0 * m * n
    # operator form, algorithmic bytes of a middle step: S^T Y_k reads Y_k and the
    # transposed pattern (row, value), writes W; S W reads the CSR pattern and W, reads
    # Y_k, Y_{k-1} and the accumulator, writes the accumulator and Y_{k+1}
    step_bytes = (dense + 8.0 * nnz + 4.0 * n * n) + (8.0 * nnz + 4.0 * n * n + 5 * dense)
    ms_p, us_p, l_p = res["auto"]
    ms_r, us_r, l_r = res["recurrence"]
    # the cold bound alone on the operator form (K = 2: the bound, then one product):
    # the power iteration against the Lanczos rule, both from the seeded vector
    bound_cold = {}
    for rule in ("power", "lanczos"):
        ob = cpa.Opts(K=2, bound=rule)
        _, ib = cpa.shrink_csr(m, n, r, c, v, cpa.soft(tau), ob, out=out, info=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(3):
            cpa.shrink_csr(m, n, r, c, v, cpa.soft(tau), ob, out=out)
        e1.record()
        torch.cuda.synchronize()
        bound_cold[rule] = {"ms_per_call": round(e0.elapsed_time(e1) / 3, 3), "Lambda": ib["Lambda"],
                            "products_or_steps": ib["power_iters_done"]}
    flop_gemm = 2.0 * n * n * n
    nt_s = (n + 63) // 64
    flop_issued = (nt_s * (nt_s + 1) // 2) * 64.0 * 64.0 * 2.0 * n
    # the whole completion: 100 SVT iterations (Cai, Candes, Shen: tau = 5 sqrt(m n),
    # delta = 1.2 m n / |Omega|), each a K = 25 shrink on the default route
    iters = 100
    tau_svt = 5.0 * math.sqrt(m * n)
    delta = 1.2 * m * n / nnz
    resid = torch.zeros(iters, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t_svt = time.perf_counter()
    e0.record()
    X, k0 = cpa.svt_complete(m, n, r, c, v, tau_svt, delta, iters, cpa.Opts(K=K, warm_start=True), out=out,
                             resid=resid)
    e1.record()
    torch.cuda.synchronize()
    wall_svt = time.perf_counter() - t_svt
    ms_svt = e0.elapsed_time(e1)
    Mt = torch.from_numpy(u_f).to(dev) @ torch.from_numpy(v_f).to(dev).T
    rel_m = float(torch.linalg.norm(X - Mt) / torch.linalg.norm(Mt))
    del Mt
    svt = {"iterations": iters, "K": K, "tau": round(tau_svt, 1), "delta": round(delta, 2), "k0": k0,
           "ms_total": round(ms_svt, 1), "wall_s": round(wall_svt, 3), "iterations_per_s": round(iters / (ms_svt / 1e3), 2),
           "final_observed_residual": float("%.3e" % float(resid[-1])), "rel_err_vs_ground_truth": float("%.3e" % rel_m)}
    return {
        "workload": "CSR 20000 x 4000, 1.6M nonzeros (2%), rank-10 N(0,1) values, soft, K=25",
        "route": "matrix polynomial: Gram S^T S (sparse), polynomial on 4000 x 4000 (FP32 MFMA), Y = S p (sparse)",
        "ms_per_shrink": round(ms_p, 3), "shrinks_per_s": round(1e3 / ms_p, 2),
        "roofline": {"bound": "mfma", "kernel": "4000^3 polynomial GEMM (symmetric: upper-triangle 64 x 64 tiles)",
                     "achieved": round(flop_gemm / (us_p * 1e-6) / 1e12, 2),
                     "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(flop_gemm / (us_p * 1e-6) / 1e12 / MFMA_FP32_PEAK_TFLOPS, 4),
                     "flop_convention": "2 n^3 per product (the product it computes); the kernel issues the "
                                        f"{nt_s * (nt_s + 1) // 2} tiles on and above the diagonal of {nt_s * nt_s}",
                     "issued_tflops": round(flop_issued / (us_p * 1e-6) / 1e12, 2),
                     "issued_frac": round(flop_issued / (us_p * 1e-6) / 1e12 / MFMA_FP32_PEAK_TFLOPS, 4),
                     "avg_launch_us": round(us_p, 1), "launches": l_p, "traffic": None},
        "svt_completion": svt,
        "cold_bound_K2": dict(bound_cold, note="one cold K = 2 call per rule (bound on S^T S through two "
                                               "sparse products per product or step, then one product)"),
        "operator_form": {"ms_per_shrink": round(ms_r, 3), "shrinks_per_s": round(1e3 / ms_r, 2),
                          "spmm_pair_avg_us": round(us_r, 1),
                          "roofline": {"bound": "hbm", "achieved": round(step_bytes / (us_r * 1e-6) / 1e9, 1),
                                       "peak": 8000.0, "unit": "GB/s",
                                       "frac": round(step_bytes / (us_r * 1e-6) / 1e9 / 8000.0, 4),
                                       "bytes_per_step": step_bytes, "traffic": None},
                          # what actually bounds it: every nonzero gathers a whole row of the
                          # dense operand (Y_k in S^T Y_k, W in S W), served from L2 / MALL
                          "gathers": {"bytes_per_step": 2.0 * nnz * n * 4,
                                      "achieved_TBps": round(2.0 * nnz * n * 4 / (us_r * 1e-6) / 1e12, 2),
                                      "note": "2 nnz n 4 bytes of row gathers per step, "
                                              "25x the algorithmic HBM bytes"}},
    }


def bench_sparsified(cpa, torch, np, synth, reps: int = 10):
    """Algorithm 1 with the 8 x 8 block DCT and truncation on a 1024 x 1024 input
    that is sparse in that transform (block-smooth, rank 4, N(0, 1e-3^2) noise;
    its transformed Gram is concentrated on the (1024/8)^2 block DC entries),
    K = 30, soft tau = 0.2 sigma_1, keeping 1.6% and 3% of the entries: hat H by
    the matrix polynomial on the nonempty block (the default) and by the sparse
    recurrence; beside them the dense matrix-polynomial route on the same input."""
    n, K = 1024, 30
    X64 = synth.block_smooth(n, n, rank=4, noise=1e-3, seed=synth.BASE_SEED + 6)
    X = torch.from_numpy(X64.astype(np.float32)).cuda()
    s1 = float(np.linalg.svd(X64, compute_uv=False)[0])
    tau = 0.2 * s1
    g = lambda sv: np.maximum(sv - tau, 0.0)
    ex = exact_shrink(X64, g)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    opts = cpa.Opts(K=K)
    warm = cpa.Opts(K=K, warm_start=True)
    Yd = torch.empty_like(X)
    ms_dense = timed(lambda: cpa.shrink_dense(X, cpa.soft(tau), opts, out=Yd))
    ms_dense_w = timed(lambda: cpa.shrink_dense(X, cpa.soft(tau), warm, out=Yd))
    ms_dense_l = timed(lambda: cpa.shrink_dense(X, cpa.soft(tau), cpa.Opts(K=K, bound="lanczos"), out=Yd))
    ms_dense_lw = timed(lambda: cpa.shrink_dense(X, cpa.soft(tau), cpa.Opts(K=K, bound="lanczos", warm_start=True),
                                                 out=Yd))
    dense_err = rel_fro(Yd.cpu().numpy().astype(np.float64), ex, ex)
    out = {"workload": "1024 x 1024 block-smooth (rank 4, 8-blocks) + N(0,1e-3^2), block DCT 8x8, K=30, soft "
                       "tau = 0.2 sigma_1, power bound",
           "dense_polynomial_route": {"ms_per_shrink": round(ms_dense, 4), "ms_per_shrink_warm": round(ms_dense_w, 4),
                                      "lanczos_ms_per_shrink": round(ms_dense_l, 4),
                                      "lanczos_ms_per_shrink_warm": round(ms_dense_lw, 4),
                                      "err_vs_fp64_svt": float("%.3e" % dense_err)},
           "keep": [],
           "note": "cold: every call starts its power iteration from the seeded vector; warm: from the previous "
                   "call's vector (as inside an ADMM run), on both routes.  lanczos_bound: both routes with the "
                   "Lanczos bound (at most 12 steps, early stop at power_tol), speedups against the dense route "
                   "with the same bound (and, beside it, with the power bound)"}
    Ys = torch.empty_like(X)
    opts_rec = cpa.Opts(K=K, eval="recurrence")
    opts_lz = cpa.Opts(K=K, bound="lanczos")
    warm_lz = cpa.Opts(K=K, bound="lanczos", warm_start=True)
    for frac in (0.016, 0.03):
        keep = int(frac * n * n)
        ms_s = timed(lambda: cpa.shrink_dense_sparsified(X, cpa.soft(tau), opts, keep=keep, out=Ys))
        ms_sw = timed(lambda: cpa.shrink_dense_sparsified(X, cpa.soft(tau), warm, keep=keep, out=Ys))
        ms_r = timed(lambda: cpa.shrink_dense_sparsified(X, cpa.soft(tau), opts_rec, keep=keep, out=Ys))
        # the Lanczos bound on the compact block (blocks up to 256 wide)
        lz = None
        try:
            ms_l = timed(lambda: cpa.shrink_dense_sparsified(X, cpa.soft(tau), opts_lz, keep=keep, out=Ys))
            ms_lw = timed(lambda: cpa.shrink_dense_sparsified(X, cpa.soft(tau), warm_lz, keep=keep, out=Ys))
            _, il = cpa.shrink_dense_sparsified(X, cpa.soft(tau), opts_lz, keep=keep, out=Ys, info=True)
            lz = {"ms_per_shrink": round(ms_l, 4), "speedup_vs_dense": round(ms_dense_l / ms_l, 3),
                  "ms_per_shrink_warm": round(ms_lw, 4), "speedup_vs_dense_warm": round(ms_dense_lw / ms_lw, 3),
                  "speedup_vs_dense_power_bound": round(ms_dense / ms_l, 3),
                  "Lambda": il["Lambda"], "steps": il["power_iters_done"]}
        except cpa.CpaError as e:
            lz = {"unsupported": str(e)}
        _, info = cpa.shrink_dense_sparsified(X, cpa.soft(tau), opts, keep=keep, out=Ys, info=True)
        Yh = Ys.cpu().numpy().astype(np.float64)
        out["keep"].append({"fraction": frac, "keep": keep, "nnz": info["nnz"], "eps": float("%.5e" % info["eps"]),
                            "ms_per_shrink": round(ms_s, 4), "speedup_vs_dense": round(ms_dense / ms_s, 3),
                            "ms_per_shrink_warm": round(ms_sw, 4), "speedup_vs_dense_warm": round(ms_dense_w / ms_sw, 3),
                            "sparse_recurrence_ms_per_shrink": round(ms_r, 4),
                            "lanczos_bound": lz, "Lambda": info["Lambda"],
                            "power_products": info["power_iters_done"],
                            "err_vs_fp64_svt": float("%.3e" % rel_fro(Yh, ex, ex)),
                            "err_vs_dense_route": float("%.3e" % rel_fro(Yh, Yd.cpu().numpy().astype(np.float64),
                                                                         Yd.cpu().numpy().astype(np.float64)))})
    # the paper's image shape (2560 x 1920, one colour component; Gram side 1920),
    # the same kind of input, 1.6% kept
    m2, n2 = 2560, 1920
    X2h = synth.block_smooth(m2, n2, rank=4, noise=1e-3, seed=synth.BASE_SEED + 8)
    X2 = torch.from_numpy(X2h.astype(np.float32)).cuda()
    lam2, _ = cpa.spectral_bound(X2, cpa.Opts(K=K))
    tau2 = 0.2 * math.sqrt(lam2)
    Y2d = torch.empty_like(X2)
    Y2s = torch.empty_like(X2)
    keep2 = int(0.016 * n2 * n2)
    ms2_d = timed(lambda: cpa.shrink_dense(X2, cpa.soft(tau2), opts, out=Y2d))
    ms2_dw = timed(lambda: cpa.shrink_dense(X2, cpa.soft(tau2), warm, out=Y2d))
    ms2_s = timed(lambda: cpa.shrink_dense_sparsified(X2, cpa.soft(tau2), opts, keep=keep2, out=Y2s))
    ms2_sw = timed(lambda: cpa.shrink_dense_sparsified(X2, cpa.soft(tau2), warm, keep=keep2, out=Y2s))
    olz, wlz = cpa.Opts(K=K, bound="lanczos"), cpa.Opts(K=K, bound="lanczos", warm_start=True)
    ms2_dl = timed(lambda: cpa.shrink_dense(X2, cpa.soft(tau2), olz, out=Y2d))
    ms2_sl = timed(lambda: cpa.shrink_dense_sparsified(X2, cpa.soft(tau2), olz, keep=keep2, out=Y2s))
    ms2_dlw = timed(lambda: cpa.shrink_dense(X2, cpa.soft(tau2), wlz, out=Y2d))
    ms2_slw = timed(lambda: cpa.shrink_dense_sparsified(X2, cpa.soft(tau2), wlz, keep=keep2, out=Y2s))
    Yd2 = Y2d.cpu().numpy().astype(np.float64)
    out["paper_shape"] = {
        "workload": "2560 x 1920 block-smooth (rank 4, 8-blocks) + N(0,1e-3^2), block DCT 8x8, K=30, soft "
                    "tau = 0.2 sqrt(Lambda), keep 1.6% of 1920^2",
        "dense_ms_per_shrink": round(ms2_d, 4), "dense_ms_per_shrink_warm": round(ms2_dw, 4),
        "sparsified_ms_per_shrink": round(ms2_s, 4), "sparsified_ms_per_shrink_warm": round(ms2_sw, 4),
        "speedup_vs_dense": round(ms2_d / ms2_s, 3), "speedup_vs_dense_warm": round(ms2_dw / ms2_sw, 3),
        "lanczos_bound": {"dense_ms_per_shrink": round(ms2_dl, 4), "sparsified_ms_per_shrink": round(ms2_sl, 4),
                          "speedup_vs_dense": round(ms2_dl / ms2_sl, 3),
                          "dense_ms_per_shrink_warm": round(ms2_dlw, 4),
                          "sparsified_ms_per_shrink_warm": round(ms2_slw, 4),
                          "speedup_vs_dense_warm": round(ms2_dlw / ms2_slw, 3)},
        "err_vs_dense_route": float("%.3e" % rel_fro(Y2s.cpu().numpy().astype(np.float64), Yd2, Yd2))}
    return out


def bench_inpaint(cpa, torch, np, synth, warmup: int = 2, iters: int = 10):
    """Texture inpainting (Appendix A) at the paper's image size: one 2560 x 1920
    colour component (portrait, as in Sec. V-C) of a synthetic periodic texture
    (the paper's images are not available), a 300 x 300 missing block with an
    8-pixel surrounding frame, K = 20, (1/rho, eta/rho) = (6, 0.1) as for
    Bricks.  Times ADMM iterations (two 2-D DCTs of four FP32 products, the
    elementwise steps and one CPA shrink with a warm-started power bound)."""
    m, n = 2560, 1920
    hole = (m // 2 - 150, m // 2 + 150, n // 2 - 150, n // 2 + 150)
    I, om, bd, L0 = synth.texture(m, n, terms=4, hole=hole, border=8, seed=synth.BASE_SEED + 7)
    dev = torch.device("cuda:0")
    run = cpa.Inpaint(torch.from_numpy(I.astype(np.float32)).to(dev), torch.from_numpy(om), 6.0, 0.1,
                      cpa.Opts(K=20, warm_start=True, power_iters=100),
                      border=torch.from_numpy(bd.astype(np.float32)))
    Et = torch.zeros(max(warmup, iters), dtype=torch.float64, device=dev)
    run.iterate(warmup, Et)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    run.iterate(iters, Et)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    reg = om == 0.0
    l = run.L.cpu().numpy().astype(np.float64)
    out = {"workload": "texture inpainting 2560 x 1920 (one colour component), 300 x 300 hole, 8-px frame, K=20, "
                       "1/rho=6, eta/rho=0.1, power bound warm-started",
           "ms_per_iteration": round(ms, 4), "iterations_per_s": round(1e3 / ms, 2),
           "iterations_done": warmup + iters, "E_t_last": float("%.3e" % Et[iters - 1].item()),
           "hole_rel_err_after": float("%.3e" % (np.linalg.norm((l - L0)[reg]) / np.linalg.norm(L0[reg])))}
    del run
    # the same problem with z1 by the sparsified shrink (full DCT) and the adaptive
    # keep of eq. (recommendation_epsilon); each iteration reads E_t back
    runs = cpa.Inpaint(torch.from_numpy(I.astype(np.float32)).to(dev), torch.from_numpy(om), 6.0, 0.1,
                       cpa.Opts(K=20, warm_start=True, power_iters=100),
                       border=torch.from_numpy(bd.astype(np.float32)))
    chunk = 40
    Es = torch.zeros(chunk, dtype=torch.float64, device=dev)
    keeps = runs.iterate_scheduled(warmup, Es, transform="dct")
    torch.cuda.synchronize()
    e_prev = Es[warmup - 1].item() if warmup else float("inf")
    # run on until the schedule has reached its third case (E_t below E_m) for a while,
    # at most sched_max iterations, timing every iteration after the warm-up
    sched_max, done = 400, 0
    k3 = cpa.keep_schedule(0.0, n)
    t = time.perf_counter()
    while done < sched_max:
        keeps += runs.iterate_scheduled(chunk, Es, transform="dct", E_prev=e_prev)
        torch.cuda.synchronize()
        e_prev = Es[chunk - 1].item()
        done += chunk
        if keeps[-chunk:].count(k3) == chunk:
            break
    ms_s = (time.perf_counter() - t) * 1e3 / done
    ls = runs.L.cpu().numpy().astype(np.float64)
    hist = {}
    for k_ in keeps:
        hist[str(k_)] = hist.get(str(k_), 0) + 1
    out["scheduled_dct"] = {
        "ms_per_iteration": round(ms_s, 4), "iterations": warmup + done, "keep_counts": hist,
        "first_iteration_at_keep": {str(k_): keeps.index(k_) for k_ in sorted(set(keeps))},
        "E_t_last": float("%.3e" % e_prev),
        "hole_rel_err_after": float("%.3e" % (np.linalg.norm((ls - L0)[reg]) / np.linalg.norm(L0[reg]))),
        "note": "z1 by the sparsified shrink (T = full DCT-II, polynomial on the kept block) with k from "
                "eq. (recommendation_epsilon), warm-started bound; host-timed, one E_t read-back per iteration; "
                "run until the schedule's third case held for a whole chunk of iterations (at most 400)"}
    return out


def bench_predictor(cpa, torch, np, synth, n_train: int = 32768, n_eval: int = 8192, epochs: int = 40,
                    gate: float = 1e-2, lr: float = 2e-3, quantiles=(0.99, 0.9)):
    """Learned bound / order predictor on patch groups 64 x U{40..120} with rank
    U{1..16} and noise sigma U[0.05, 0.5] (soft tau_j = sigma_j (sqrt(64) + sqrt(n_j))).
    Labels come from the method on the GPU (converged power bound; smallest K of
    {4, 6, .., 64} whose result is within `gate` of the exact shrinkage), training
    from the library's kernels.  Gain: matrices/s of the predicted path (no power
    iteration, per-matrix K, growth check on) over plain CPA (power bound, one K for
    all: the smallest whose pass rate of the gate reaches the predicted path's), on
    a held-out batch."""
    from paper_1705_07112_amd import predictor as P
    dev = torch.device("cuda:0")

    def make(batch, seed):
        flat, ms, ns, offs, _, noises = synth.patch_groups(batch=batch, rank_range=(1, 16),
                                                           noise_range=(0.05, 0.5), seed=seed)
        taus = noises * (np.sqrt(ms) + np.sqrt(ns))
        t = time.perf_counter()
        ex = P.exact_soft_batch(flat, ms, ns, offs, taus)
        return {"ms": ms, "ns": ns, "offs": offs, "taus": taus, "X": torch.from_numpy(flat).to(dev), "m": torch.from_numpy(ms).to(dev),
                "n": torch.from_numpy(ns).to(dev), "off": torch.from_numpy(offs).to(dev),
                "recs": P.soft_records(torch, taus, dev), "Yex": torch.from_numpy(ex).to(dev),
                "t_exact": time.perf_counter() - t}

    tr = make(n_train, synth.BASE_SEED + 4)
    ev = make(n_eval, synth.BASE_SEED + 5)
    torch.cuda.synchronize()
    t = time.perf_counter()
    feat, targ, kstar, miss = P.make_labels(torch, tr["X"], tr["m"], tr["n"], tr["off"], tr["recs"], tr["ms"],
                                            tr["ns"], tr["offs"], tr["Yex"], gate=gate)
    torch.cuda.synchronize()
    t_label = time.perf_counter() - t
    ok = torch.isfinite(targ).all(dim=1)
    gen = torch.Generator().manual_seed(0)
    idx = torch.nonzero(ok).flatten().cpu()
    idx = idx[torch.randperm(idx.numel(), generator=gen)].to(dev)
    feat, targ = feat[idx].contiguous(), targ[idx].contiguous()
    mean = feat.double().mean(0).cpu().numpy()
    std = feat.double().std(0).cpu().numpy()
    model = torch.from_numpy(P.init_model(0, mean, std)).to(dev)
    adam = torch.zeros(2 * cpa.PRED_PARAMS, dtype=torch.float32, device=dev)
    losses = torch.zeros(epochs, dtype=torch.float64, device=dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    cpa.predictor_train(feat, targ, model, adam, 0, quantiles, batch_size=1024, epochs=epochs, lr=lr,
                        epoch_loss=losses)
    e1.record()
    torch.cuda.synchronize()
    ms_train = e0.elapsed_time(e1)
    lh = losses.cpu().numpy()

    nb = int(ev["m"].numel())
    bounds = P.segment_bounds(torch, ev["ms"], ev["ns"], ev["offs"], dev)
    Y = torch.empty_like(ev["X"])
    lam = torch.zeros(nb, dtype=torch.float64, device=dev)
    kout = torch.zeros(nb, dtype=torch.int32, device=dev)
    st = torch.zeros(nb, dtype=torch.int32, device=dev)
    popts = cpa.Opts(K=64, check=True)

    def predicted():
        cpa.shrink_batched_predicted(ev["X"], ev["m"], ev["n"], ev["off"], cpa.soft(0.0), popts, model, K_min=4,
                                     shrink_per_matrix=ev["recs"], out=Y, lambda_out=lam, K_out=kout, status=st)

    def plain(Kc):
        cpa.shrink_batched(ev["X"], ev["m"], ev["n"], ev["off"], cpa.soft(0.0), cpa.Opts(K=Kc),
                           shrink_per_matrix=ev["recs"], out=Y)

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_pred = timed(predicted)
    Yh, lamh, kh = Y.cpu().numpy(), lam.cpu().numpy(), kout.cpu().numpy()
    Xh = ev["X"].cpu().numpy()
    for i in range(0, nb, 256):
        o, sz = int(ev["offs"][i]), int(ev["ms"][i]) * int(ev["ns"][i])
        shp = (int(ev["ms"][i]), int(ev["ns"][i]))
        SAMPLES.setdefault("predicted", []).append((Xh[o:o + sz].reshape(shp).astype(np.float64),
                                                    Yh[o:o + sz].reshape(shp).astype(np.float64),
                                                    (0, float(ev["taus"][i]), 0.0, 0.0, 0.0), float(lamh[i]),
                                                    int(kh[i])))
    err, ref2 = P.rel_errors(torch, Y, ev["Yex"], bounds)
    pass_pred = float((err <= gate).double().mean())
    k_mean = float(kout.double().mean())
    fb = float((st == 1).double().mean())
    plain_rows = []
    chosen = None
    for Kc in P.K_GRID:
        plain(Kc)
        e, _ = P.rel_errors(torch, Y, ev["Yex"], bounds, ref2)
        pr = float((e <= gate).double().mean())
        plain_rows.append((Kc, pr))
        if pr >= pass_pred:
            chosen = (Kc, pr)
            break
    if chosen is None:
        chosen = plain_rows[-1]
    ms_plain = timed(lambda: plain(chosen[0]))
    return {
        "workload": f"train {n_train} / held-out {n_eval} patch groups 64 x U{{40..120}}, rank U{{1..16}}, "
                    f"sigma U[0.05,0.5], soft tau = sigma (sqrt m + sqrt n); gate: rel. err <= {gate:g} vs exact",
        "labels": {"seconds_gpu_method_runs": round(t_label, 2),
                   "seconds_exact_svd_host": round(tr["t_exact"] + ev["t_exact"], 2),
                   "K_star_mean": round(float(kstar.double().mean()), 2),
                   "miss_frac": round(float(miss.double().mean()), 4)},
        "train": {"epochs": epochs, "batch": 1024, "lr": lr, "quantiles": list(quantiles),
                  "ms_per_epoch": round(ms_train / epochs, 3), "loss_first": round(float(lh[0]), 5),
                  "loss_last": round(float(lh[-1]), 5)},
        "predicted": {"pass_rate": round(pass_pred, 4), "matrices_per_s": round(nb / (ms_pred / 1e3), 1),
                      "ms_per_batch": round(ms_pred, 4), "K_mean": round(k_mean, 2), "fallback_frac": round(fb, 4)},
        "plain_cpa": {"K": chosen[0], "pass_rate": round(chosen[1], 4),
                      "matrices_per_s": round(nb / (ms_plain / 1e3), 1), "ms_per_batch": round(ms_plain, 4)},
        "gain": round(ms_plain / ms_pred, 3),
        "as_stated": "not measured as stated (200k training matrices, K* for a 1e-3 gate on orders up to 128): "
                     "the batched kernel takes K <= 64, and soft thresholding on this family meets 1e-3 against "
                     "the exact shrinkage for almost no matrix at K <= 64 (its kink at tau limits the polynomial), "
                     f"so the gate is {gate:g} and the run trains on {n_train} matrices to stay within the bench's "
                     "time; the gain test in the GPU suite asserts gain > 1 at equal pass rate",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-main-only", action="store_true",
                    help="run only the batched leg's main plan (split precision, Lanczos bound)")
    ap.add_argument("--no-sparse", action="store_true")
    ap.add_argument("--no-predictor", action="store_true")
    ap.add_argument("--no-sparsified", action="store_true")
    ap.add_argument("--no-inpaint", action="store_true")
    ap.add_argument("--no-metric-order", action="store_true", help="skip the K = 512 leg at the metric's error bar")
    ap.add_argument("--no-designs", action="store_true", help="skip the least-squares / minimax comparison")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(a row-sharded X would need one all-reduce of the d x d Gram partials per shrink; "
              "that path is not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "launches": 3}), flush=True)
        return

    import paper_1705_07112_amd as cpa
    import synth

    def progress(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    I, _, _ = synth.rpca_frames(M, N)
    Id = torch.from_numpy(I).to(dev)
    opts = cpa.Opts(K=K, warm_start=True, power_iters=100)
    run = cpa.RpcaAdmm(Id, INV_RHO, ETA_OVER_RHO, opts)
    # one E_t buffer for the warm-up and the timed call: the captured iteration
    # bakes in its pointer, so the warm-up also captures the graph the timed call
    # replays (each call writes E_t from index 0)
    Et = torch.zeros(max(args.warmup, args.steps), dtype=torch.float64, device=dev)
    if args.warmup:
        run.iterate(args.warmup, Et)
    torch.cuda.synchronize()

    # timed region: `steps` ADMM iterations, replayed from the library's captured graph
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    run.iterate(args.steps, Et)
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)

    # spread of the step time (untimed for `value`): single replays, each
    # bracketed by its own pair of events on the same stream
    n_spread = max(args.steps, 20)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_spread)]
    for a_, b_ in ev:
        a_.record()
        run.iterate(1, Et)
        b_.record()
    torch.cuda.synchronize()
    per_step = np.array([a_.elapsed_time(b_) for a_, b_ in ev])

    # roofline pass: the same iterations again with every GEMM launch bracketed by
    # HIP events on the launch stream (event timing needs direct launches)
    cpa.timing_enable(True)
    run.iterate(args.steps)
    torch.cuda.synchronize()
    rec_ms, rec_n = cpa.timing_read("recurrence")
    gram_ms, gram_n = cpa.timing_read("gram")
    pc_ms, pc_n = cpa.timing_read("pieces")
    cpa.timing_enable(False)

    flop_gemm = 2.0 * M * N * min(M, N)
    # products per shrink: the Gram, then the matrix polynomial on the d x d side
    # (baby steps s - 1, giant steps J - 1, one product with X); the recurrence
    # over X would take K - 1 (reported as the equivalent rate)
    s_ps = math.isqrt(K - 1) + 1 if K > 1 else 1
    j_ps = -(-K // s_ps)
    products = 1 + (s_ps - 1) + (j_ps - 1) + 1
    flop_shrink = products * flop_gemm
    ms_per_step = ms / args.steps
    value = args.steps / (ms / 1e3)
    rec_avg_us = 1e3 * rec_ms / max(rec_n, 1)
    # the symmetric products (baby and giant steps) run in pieces: each tile above
    # the diagonal as two 64 x 32 halves, each diagonal tile's upper triangle;
    # issued MFMA blocks of 16 x 16: 16 per tile above the diagonal, 10 per diagonal tile
    nt = N // 64
    piece_blocks = 16 * nt * (nt - 1) // 2 + 10 * nt
    flop_piece_issued = piece_blocks * 16 * 16 * 2.0 * N
    pc_avg_us = 1e3 * pc_ms / max(pc_n, 1)
    n_sym = (s_ps - 1) + (j_ps - 1)
    flop_shrink_issued = flop_gemm * (1 + (products - 1 - n_sym)) + flop_piece_issued * n_sym
    achieved = flop_gemm / (pc_avg_us * 1e-6) / 1e12
    achieved_full = flop_gemm / (rec_avg_us * 1e-6) / 1e12

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
        "tflops_issued": round(flop_shrink_issued * value / 1e12, 3),
        "tflops_note": f"{products} products of 1024^3 per shrink (Gram + matrix polynomial, s={s_ps}, J={j_ps}) "
                       f"counted as full products; {n_sym} of them are symmetric and issue only their upper "
                       f"triangle (tflops_issued); the recurrence over X would take {K}",
        "wall_s_timed": round(wall, 4),
        "roofline": {"bound": "mfma",
                     "kernel": "symmetric matrix-polynomial product 1024^3 in pieces (gemm_f32_piece_kernel: FP32 "
                               "MFMA, direct global-to-LDS copies, mirrored stores)",
                     "achieved": round(achieved, 3), "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / MFMA_FP32_PEAK_TFLOPS, 4), "traffic": measured_traffic(),
                     "traffic_unit": "bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, copy-calibrated)",
                     "avg_launch_us": round(pc_avg_us, 3), "launches": pc_n,
                     "flop_per_launch": flop_gemm,
                     "flop_convention": "2 d^3 per product (the product it computes); the kernel issues "
                                        f"{flop_piece_issued / flop_gemm:.3f} of them (blocks on and above the diagonal)",
                     "issued_flop_per_launch": flop_piece_issued,
                     "issued_tflops": round(flop_piece_issued / (pc_avg_us * 1e-6) / 1e12, 3),
                     "issued_frac": round(flop_piece_issued / (pc_avg_us * 1e-6) / 1e12 / MFMA_FP32_PEAK_TFLOPS, 4),
                     "timing": "HIP events around each launch, same workload, pass right after the timed region",
                     "full_product": {"kernel": "gemm_f32_lds_kernel (Y = X p, the one non-symmetric product)",
                                      "avg_launch_us": round(rec_avg_us, 3), "launches": rec_n,
                                      "achieved": round(achieved_full, 3),
                                      "frac": round(achieved_full / MFMA_FP32_PEAK_TFLOPS, 4)},
                     "gram_avg_us": round(1e3 * gram_ms / max(gram_n, 1), 3)},
    }

    # achievable rates on this device, measured beside the spec peaks: pure-register
    # MFMA streams (cpa_peak_mfma) and a plain 256 MiB device copy
    peak32, clock32 = cpa.peak_mfma("fp32", clock=True)
    peak16 = cpa.peak_mfma("bf16")
    csrc = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    cdst = torch.empty_like(csrc)
    cdst.copy_(csrc)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(10):
        cdst.copy_(csrc)
    t1.record()
    torch.cuda.synchronize()
    copy_tbps = 10 * 2 * csrc.numel() * 4 / (t0.elapsed_time(t1) * 1e-3) / 1e12
    del csrc, cdst
    out["roofline"]["achievable_peak"] = round(peak32, 1)
    out["roofline"]["frac_of_achievable"] = round(achieved / peak32, 4)
    out["roofline"]["issued_frac_of_achievable"] = round(out["roofline"]["issued_tflops"] / peak32, 4)
    out["step_ms_spread"] = {"median": round(float(np.median(per_step)), 4),
                             "p10": round(float(np.percentile(per_step, 10)), 4),
                             "p90": round(float(np.percentile(per_step, 90)), 4), "steps": n_spread,
                             "method": "single graph replays after the timed region, each between two events"}
    out["achievable_peaks"] = {"mfma_fp32_tflops": round(peak32, 1), "mfma_bf16_tflops": round(peak16, 1),
                               "clock_ghz_under_fp32_mfma": round(clock32, 3),
                               "hbm_copy_tbps": round(copy_tbps, 2),
                               "method": "cpa_peak_mfma (register-only MFMA streams, 4 waves/SIMD); "
                                         "device copy of 256 MiB (read + write bytes)"}

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
    # the same workload with the three-term recurrence over X (the paper's evaluation order)
    run3 = cpa.RpcaAdmm(Id, INV_RHO, ETA_OVER_RHO, cpa.Opts(K=K, warm_start=True, power_iters=100, eval="recurrence"))
    run3.iterate(args.warmup)
    torch.cuda.synchronize()
    t0.record()
    run3.iterate(args.steps)
    t1.record()
    torch.cuda.synchronize()
    ms3 = t0.elapsed_time(t1)
    cpa.timing_enable(True)
    run3.iterate(args.steps)
    torch.cuda.synchronize()
    rec3_ms, rec3_n = cpa.timing_read("recurrence")
    cpa.timing_enable(False)
    rec3_us = 1e3 * rec3_ms / max(rec3_n, 1)
    out["recurrence_route"] = {
        "value": round(args.steps / (ms3 / 1e3), 3), "ms_per_step": round(ms3 / args.steps, 4),
        "note": "same ADMM workload, eval='recurrence': K-1 = 29 products Y_{k+1} = 2 Y_k Ghat - Y_{k-1} over X",
        "roofline": {"bound": "mfma", "kernel": "recurrence GEMM 1024^3 (FP32 MFMA, fused Chebyshev epilogue)",
                     "achieved": round(flop_gemm / (rec3_us * 1e-6) / 1e12, 3), "peak": MFMA_FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(flop_gemm / (rec3_us * 1e-6) / 1e12 / MFMA_FP32_PEAK_TFLOPS, 4),
                     "avg_launch_us": round(rec3_us, 3), "launches": rec3_n}}
    out["bf16x3"] = {"value": round(args.steps / (ms2 / 1e3), 3), "ms_per_step": round(ms2 / args.steps, 4),
                     "recurrence_avg_us": round(1e3 * rec2_ms / max(rec2_n, 1), 3),
                     "note": "same ADMM workload; recurrence products as bf16 hi/lo x3 on the BF16 matrix cores"}

    # FP64 path: one shrink of the 1024 x 1024 frames in double precision (recurrence,
    # K = 30, power bound), timed over a few calls
    X64d = Id.to(torch.float64)
    o64 = cpa.Opts(K=K, precision="fp64")
    cpa.shrink_dense(X64d, cpa.soft(INV_RHO), o64)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(3):
        cpa.shrink_dense(X64d, cpa.soft(INV_RHO), o64)
    t1.record()
    torch.cuda.synchronize()
    ms64 = t0.elapsed_time(t1) / 3
    flop64 = K * flop_gemm   # Gram + K - 1 recurrence products
    out["fp64"] = {"ms_per_shrink": round(ms64, 3), "shrinks_per_s": round(1e3 / ms64, 2),
                   "tflops": round(flop64 / (ms64 * 1e-3) / 1e12, 2), "peak_fp64_tflops": 78.6,
                   "note": "cpa_shrink_dense_f64 on the 1024 x 1024 frames: FP64 Gram, power bound and K - 1 = 29 "
                           "FP64 products (FP64 matrix cores, 64 x 64 tiles, 8 waves, K-steps of 32 split in two, two LDS stages, register prefetch)"}
    del X64d

    check = None
    if not args.no_accuracy:
        # one shrink of the current ADMM iterate (L + U1) on the device, against the
        # exact soft shrinkage (LAPACK SVD); the FP64 CPA comparison is made in the
        # oracle leg below
        Xd = (run.block(0) + run.block(4)).contiguous()
        Yd, info = cpa.shrink_dense(Xd, cpa.soft(INV_RHO), cpa.Opts(K=K), info=True)
        X64 = Xd.cpu().numpy().astype(np.float64)
        Y = Yd.cpu().numpy().astype(np.float64)
        ex = exact_shrink(X64, lambda sv: np.maximum(sv - INV_RHO, 0.0))
        out["err_vs_fp64_svt"] = float("%.3e" % rel_fro(Y, ex, ex))
        Y2 = cpa.shrink_dense(Xd, cpa.soft(INV_RHO), cpa.Opts(K=K, Lambda=info["Lambda"], precision="bf16x3"))
        Y2 = Y2.cpu().numpy().astype(np.float64)
        out["bf16x3"]["err_vs_fp64_svt"] = float("%.3e" % rel_fro(Y2, ex, ex))
        out["E_t_last"] = float("%.3e" % Et[args.steps - 1].item())
        check = (X64, {"fp32": Y, "bf16x3": Y2}, info["Lambda"])
        if not args.no_designs:
            out["designs"] = bench_designs(cpa, torch, np, Xd, X64, ex, info["Lambda"])

    # the same ADMM at the order where this workload's CPA meets the metric's error bar
    # (<= 1e-3 relative Frobenius against the exact shrinkage): K = 512 on the matrix-
    # polynomial route; the error is measured on the iterates that open and close the
    # timed window (LAPACK SVD of l + u1 on the host)
    if not args.no_metric_order:
        out["at_metric_error"] = bench_metric_order(cpa, torch, np, Id, args)
    progress("dense RPCA legs done")
    if not args.no_batched:
        out["batched"] = bench_batched(cpa, torch, np, synth, main_only=args.batched_main_only)
        progress("batched leg done")

    if not args.no_sparse:
        out["sparse"] = bench_sparse(cpa, torch, np, synth)
        progress("sparse leg done")

    if not args.no_sparsified:
        out["sparsified"] = bench_sparsified(cpa, torch, np, synth)
        progress("sparsified leg done")
    if not args.no_inpaint:
        out["inpaint"] = bench_inpaint(cpa, torch, np, synth)
        progress("inpaint leg done")
    if not args.no_predictor:
        out["predictor"] = bench_predictor(cpa, torch, np, synth)
        progress("predictor leg done")

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(I, check=check, samples=SAMPLES)
        progress("oracle leg done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
