"""FP64 shrinkage (cpa_shrink_dense_f64) against the FP64 oracle.

With FP64 arithmetic on both sides the results differ only by summation order,
so the bar is 1e-11 in relative Frobenius norm (the FP32 path's is 1e-5)."""
import math

import numpy as np
import pytest

import synth
from oracle import bound as obound
from oracle import cpa as ocpa
from oracle import metrics
from oracle.shrinkage import Shrinkage

pytestmark = pytest.mark.gpu

TOL64 = 1e-11


def _lib():
    import paper_1705_07112_amd as cpa
    return cpa


def _shrinks(cpa, lmax, kind):
    tau = 0.4 * math.sqrt(lmax)
    if kind == 0:
        return Shrinkage(0, tau), cpa.soft(tau)
    if kind == 1:
        return Shrinkage(1, tau), cpa.hard(tau)
    wc, ws = 0.3 * tau * tau, 0.05 * lmax
    return Shrinkage(3, 0.0, wc, ws, 1e-3), cpa.weighted_fn(wc, ws, 1e-3)


@pytest.mark.parametrize("shape,K,kind", [((64, 48), 20, 0), ((130, 70), 30, 1), ((70, 130), 30, 2),
                                          ((257, 129), 16, 0), ((33, 5), 2, 0), ((5, 33), 1, 1), ((1, 1), 3, 0)])
def test_f64_matches_oracle(shape, K, kind):
    import torch
    cpa = _lib()
    m, n = shape
    X = synth.dense_lowrank(m, n, rank=min(4, m, n), noise=0.2, seed=8800 + m + n)
    G = X.T @ X if m >= n else X @ X.T
    lmax = float(np.linalg.eigvalsh(G)[-1])
    Lam = 1.01 * lmax
    sh_o, sh_c = _shrinks(cpa, lmax, kind)
    ref = ocpa.cpa_shrink(X, sh_o, Lam, K)
    Y, info = cpa.shrink_dense(torch.from_numpy(X).cuda(), sh_c, cpa.Opts(K=K, Lambda=Lam, precision="fp64"),
                               info=True)
    torch.cuda.synchronize()
    err = metrics.rel_fro(Y.cpu().numpy(), ref, X)
    print(f"f64 {m}x{n} K={K} kind={kind}: rel_fro={err:.3e}", flush=True)
    assert Y.dtype == torch.float64
    assert err <= TOL64
    assert info["side"] == (0 if m >= n else 1)


def test_f64_padded_rows_and_both_sides():
    import torch
    cpa = _lib()
    m, n = 96, 80
    X = synth.dense_lowrank(m, n, rank=5, noise=0.3, seed=8900)
    buf = torch.zeros((m, n + 7), dtype=torch.float64)
    buf[:, :n] = torch.from_numpy(X)
    Xd = buf.cuda()[:, :n]
    for side in ("right", "left"):
        G = X.T @ X if side == "right" else X @ X.T
        lmax = float(np.linalg.eigvalsh(G)[-1])
        Lam, tau = 1.01 * lmax, 0.3 * math.sqrt(lmax)
        ref = ocpa.cpa_shrink(X, Shrinkage(0, tau), Lam, 24)
        Y = cpa.shrink_dense(Xd, cpa.soft(tau), cpa.Opts(K=24, Lambda=Lam, side=side))
        torch.cuda.synchronize()
        err = metrics.rel_fro(Y.cpu().numpy(), ref, X)
        print(f"f64 padded side={side}: rel_fro={err:.3e}", flush=True)
        assert err <= TOL64


def test_f64_power_bound_matches_oracle():
    """Power iteration on the FP64 Gram, converged (tol 1e-12): the bound agrees
    with the oracle's to 1e-10."""
    import torch
    cpa = _lib()
    for seed, (m, n) in enumerate([(200, 120), (64, 300), (1024, 256)]):
        X = synth.dense_lowrank(m, n, rank=5, noise=0.3, seed=9000 + seed)
        G = X.T @ X if m >= n else X @ X.T
        lam_o = obound.power_bound(G, seed=seed, max_iter=1000, tol=1e-12)[0]
        _, info = cpa.shrink_dense(torch.from_numpy(X).cuda(), cpa.soft(0.1),
                                   cpa.Opts(K=4, power_iters=1000, power_tol=1e-12, seed=seed), info=True)
        print(f"f64 bound {m}x{n}: gpu {info['Lambda']:.15g} oracle {lam_o:.15g} iters {info['power_iters_done']}",
              flush=True)
        assert abs(info["Lambda"] - lam_o) <= 1e-10 * lam_o


def test_f64_rejections():
    import torch
    cpa = _lib()
    X = torch.ones((16, 8), dtype=torch.float64, device="cuda")
    for o in (cpa.Opts(K=4, precision="bf16x3"), cpa.Opts(K=4, check=True), cpa.Opts(K=4, eval="polynomial")):
        with pytest.raises(cpa.CpaError):
            cpa.shrink_dense(X, cpa.soft(0.1), o)
    with pytest.raises(cpa.CpaError):
        cpa.shrink_dense(X, cpa.soft(0.1), cpa.Opts(K=4), out=X)


@pytest.mark.parametrize("shape,steps,tol", [((130, 70), 12, 1e-7), ((70, 130), 5, 0.0), ((300, 257), 32, 0.0),
                                             ((1100, 600), 12, 1e-7), ((40, 3), 12, 0.0)])
def test_f64_lanczos_bound(shape, steps, tol):
    """The Lanczos bound on the FP64 Gram (the grid kernel at every side, its
    vectors in the product buffer) against the oracle's lanczos_bound on the same
    Gram, and the shrink at that bound against the oracle's CPA.  FP64 on both
    sides: the bounds agree to rounding (1e-10 relative; the device brackets the
    Ritz value to 2^-30 of it, well inside)."""
    import torch
    cpa = _lib()
    m, n = shape
    print(f"case f64 lanczos {m}x{n} steps={steps} tol={tol}", flush=True)
    X = synth.dense_lowrank(m, n, rank=min(4, m, n), noise=0.2, seed=8900 + m + n)
    G = X.T @ X if m >= n else X @ X.T
    Lo, th_o, r_o, k_o, *_ = obound.lanczos_bound(G, seed=0, steps=steps, tol=tol)
    lmax = float(np.linalg.eigvalsh(G)[-1])
    sh_o, sh_c = _shrinks(cpa, lmax, 0)
    Y, info = cpa.shrink_dense(torch.from_numpy(X).cuda(), sh_c,
                               cpa.Opts(K=20, bound="lanczos", lanczos_steps=steps, power_tol=tol), info=True)
    torch.cuda.synchronize()
    print(f"  gpu {info['Lambda']:.15g} oracle {Lo:.15g} steps {info['power_iters_done']}/{k_o}", flush=True)
    if tol == 0.0:
        assert info["power_iters_done"] == k_o
    else:
        assert abs(info["power_iters_done"] - k_o) <= 1
    # a stop one step apart (a Ritz value moving by about tol) moves Lambda by about tol
    assert abs(info["Lambda"] - Lo) <= (1e-8 if info["power_iters_done"] == k_o else 2e-6) * Lo
    ref = ocpa.cpa_shrink(X, sh_o, info["Lambda"], 20)
    err = metrics.rel_fro(Y.cpu().numpy(), ref, X)
    print(f"  shrink rel_fro={err:.3e}", flush=True)
    assert err <= TOL64
