"""The allocation-free dense shrink (cpa_shrink_dense_noalloc, workspace in the
library's static scratch) against the allocating entry point cpa_shrink_dense
on the same inputs, through the C ABI: calls in a row whose second input is
smaller than the first (the scratch keeps the first call's contents), both
evaluation routes and both Gram sides, the FP32 bar of 1e-5 relative Frobenius
plus a max-element bound, the oracle beside them, and the host-side rejection
of requests beyond the scratch."""
import numpy as np
import pytest

import synth
from oracle import cpa as ocpa
from oracle import metrics
from oracle.shrinkage import Shrinkage

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def _compare(X, sh, opts, label):
    import torch
    import paper_1705_07112_amd as cpa
    ref, iref = cpa.shrink_dense(X, sh, opts, info=True)
    out = torch.full_like(X, float("nan"))
    got, igot = cpa.shrink_dense_noalloc(X, sh, opts, out, info=True)
    torch.cuda.synchronize()
    r = ref.cpu().numpy().astype(np.float64)
    g = got.cpu().numpy().astype(np.float64)
    err = metrics.rel_fro(g, r, X.cpu().numpy().astype(np.float64))
    emax = float(np.max(np.abs(g - r))) / max(float(np.max(np.abs(r))), 1e-30)
    print(f"  {label}: noalloc vs shrink_dense rel_fro={err:.3e} max={emax:.3e} "
          f"bit-equal={bool(torch.equal(ref, got))} Lambda {igot['Lambda']:.9g} / {iref['Lambda']:.9g}", flush=True)
    assert np.all(np.isfinite(g))
    assert err <= TOL32 and emax <= 10 * TOL32
    assert igot["Lambda"] == pytest.approx(iref["Lambda"], rel=1e-6)
    return g, igot


def test_noalloc_matches_shrink_dense_in_a_row():
    import math
    import torch
    import paper_1705_07112_amd as cpa
    print("noalloc: 1024 x 1024 frames, K = 30, power bound (matrix-polynomial route)", flush=True)
    I, _, _ = synth.rpca_frames()
    X1 = torch.from_numpy(I).cuda()
    _compare(X1, cpa.soft(10.0), cpa.Opts(K=30), "1024x1024 K=30")
    print("noalloc: 200 x 150, K = 20, recurrence route (smaller than the call before)", flush=True)
    X2h = synth.as_f32_exact(synth.dense_lowrank(200, 150, rank=6, noise=0.1, seed=71))
    X2 = torch.from_numpy(X2h.astype(np.float32)).cuda()
    lam = float(np.linalg.eigvalsh(X2h.T @ X2h)[-1])
    Lam, tau = 1.01 * lam, 0.4 * math.sqrt(lam)
    g, _ = _compare(X2, cpa.soft(tau), cpa.Opts(K=20, Lambda=Lam, eval="recurrence"), "200x150 K=20 recurrence")
    ref = ocpa.cpa_shrink(X2h, Shrinkage(0, tau), Lam, 20)
    e = metrics.rel_fro(g, ref)
    print(f"  200x150 vs FP64 oracle rel_fro={e:.3e}", flush=True)
    assert e <= TOL32
    print("noalloc: 96 x 160 (left side), K = 13, hard threshold, growth check", flush=True)
    X3h = synth.as_f32_exact(synth.dense_lowrank(96, 160, rank=4, noise=0.2, seed=72))
    X3 = torch.from_numpy(X3h.astype(np.float32)).cuda()
    lam3 = float(np.linalg.eigvalsh(X3h @ X3h.T)[-1])
    _compare(X3, cpa.hard(0.3 * math.sqrt(lam3)), cpa.Opts(K=13, check=True), "96x160 K=13 check")


def test_noalloc_warm_start_and_limits():
    import torch
    import paper_1705_07112_amd as cpa
    print("noalloc: warm start across calls, then rejected sizes", flush=True)
    X = torch.from_numpy(synth.as_f32_exact(synth.dense_lowrank(300, 256, rank=5, noise=0.1, seed=73))
                         .astype(np.float32)).cuda()
    out = torch.empty_like(X)
    opts = cpa.Opts(K=16, warm_start=True, power_tol=1e-7)
    _, i1 = cpa.shrink_dense_noalloc(X, cpa.soft(1.0), opts, out, info=True)
    y1 = out.clone()
    _, i2 = cpa.shrink_dense_noalloc(X, cpa.soft(1.0), opts, out, info=True)
    torch.cuda.synchronize()
    print(f"  power products: cold {i1['power_iters_done']}, warm {i2['power_iters_done']}", flush=True)
    assert i2["power_iters_done"] < i1["power_iters_done"]
    assert abs(i2["Lambda"] - i1["Lambda"]) <= 1e-5 * i1["Lambda"]
    assert metrics.rel_fro(out.cpu().numpy(), y1.cpu().numpy()) <= 1e-4
    # beyond the scratch: 2048 x 2048 at K = 30 needs (1 + 14) * 16 MiB; Gram side above 4096
    big = torch.zeros((2048, 2048), device="cuda")
    with pytest.raises(cpa.CpaError) as e1:
        cpa.shrink_dense_noalloc(big, cpa.soft(1.0), cpa.Opts(K=30), torch.empty_like(big))
    wide = torch.zeros((8, 5000), device="cuda")
    with pytest.raises(cpa.CpaError) as e2:
        cpa.shrink_dense_noalloc(wide, cpa.soft(1.0), cpa.Opts(K=4, side="right"), torch.empty_like(wide))
    print(f"  rejected: {e1.value} | {e2.value}", flush=True)
    assert e1.value.status == cpa.ERR_SHAPE and e2.value.status == cpa.ERR_SHAPE
    # aliasing is an argument error, as for the allocating entry point
    with pytest.raises(cpa.CpaError) as e3:
        cpa.shrink_dense_noalloc(X, cpa.soft(1.0), cpa.Opts(K=4), X)
    assert e3.value.status == cpa.ERR_ARG
