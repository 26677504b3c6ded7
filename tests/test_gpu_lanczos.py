"""GPU parity of the k-step Lanczos bound (CPA_BOUND_LANCZOS) with the oracle's
lanczos_bound: the dense entry points (one-workgroup kernel for Gram sides up to
256, the multi-workgroup kernel above), the sparsified shrink's compact block and
the batched path, plus the
shrink evaluated at the device's bound, the warm start from the Ritz vector and
the refusals (the FP64 entry point's parity is in test_gpu_f64.py).  The oracle runs in FP64 on the Gram of the FP32 input; the device
Gram is FP32 (MFMA), so bounds agree to about 1e-7 relative."""
import math

import numpy as np
import pytest

import synth
from tests import parity
from oracle import bound as obound
from oracle import cpa as ocpa
from oracle import metrics
from oracle import sparsify
from oracle.shrinkage import Shrinkage
from tests.test_gpu_sparsify import _gap_keep

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
LAM_TOL = 2e-6


def _gram(X):
    return X.T @ X if X.shape[0] >= X.shape[1] else X @ X.T


@pytest.mark.parametrize("shape", [(64, 48), (200, 120), (90, 300), (400, 256), (256, 4), (130, 70), (7, 1),
                                   (400, 300), (300, 700), (1100, 1024), (2100, 2050)])
@pytest.mark.parametrize("steps", [1, 5, 12, 32])
@pytest.mark.parametrize("tol", [0.0, 1e-7])
def test_dense_bound_matches_oracle(shape, steps, tol):
    """tol = 0: all the steps; tol = 1e-7 (the default): the early stop, whose step
    may differ by one where a Ritz value moves by about tol (the device forms the
    Ritz values to about 1e-9)."""
    import torch
    import paper_1705_07112_amd as cpa
    m, n = shape
    print(f"case lanczos bound {m}x{n} steps={steps} tol={tol}", flush=True)
    X = synth.as_f32_exact(synth.dense_lowrank(m, n, rank=min(5, m, n), noise=0.3, seed=7100 + m + n))
    G = _gram(X)
    Lo, th_o, r_o, k_o, *_ = obound.lanczos_bound(G, seed=0, steps=steps, tol=tol)
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    lam_g, info = cpa.spectral_bound(Xd, cpa.Opts(K=4, bound="lanczos", lanczos_steps=steps, power_tol=tol))
    print(f"  gpu {lam_g:.12g} oracle {Lo:.12g} theta {info['mu']:.12g}/{th_o:.12g} "
          f"resid {info['resid']:.4g}/{r_o:.4g} steps {info['power_iters_done']}/{k_o}", flush=True)
    if tol == 0.0:
        assert info["power_iters_done"] == k_o
    else:
        assert abs(info["power_iters_done"] - k_o) <= 1
    assert abs(lam_g - Lo) <= LAM_TOL * Lo
    assert abs(info["mu"] - th_o) <= LAM_TOL * th_o
    if r_o > 1e-3 * th_o and info["power_iters_done"] == k_o:
        assert abs(info["resid"] - r_o) <= 1e-4 * r_o
    if steps >= 12:
        assert lam_g >= float(np.linalg.eigvalsh(G)[-1]) * (1 - 1e-6)


@pytest.mark.parametrize("ev", ["recurrence", "polynomial"])
@pytest.mark.parametrize("shape,K", [((130, 70), 30), ((70, 130), 20), ((300, 256), 30), ((64, 64), 16),
                                     ((600, 300), 30), ((1100, 1024), 30)])
def test_dense_shrink_at_the_lanczos_bound(ev, shape, K):
    import torch
    import paper_1705_07112_amd as cpa
    m, n = shape
    print(f"case lanczos shrink {m}x{n} K={K} {ev}", flush=True)
    X = synth.as_f32_exact(synth.dense_lowrank(m, n, rank=4, noise=0.2, seed=7200 + m))
    G = _gram(X)
    Lo = obound.lanczos_bound(G, seed=0, steps=12, tol=1e-7)[0]
    tau = 0.3 * math.sqrt(Lo)
    Y, info = cpa.shrink_dense(torch.from_numpy(X.astype(np.float32)).cuda(), cpa.soft(tau),
                               cpa.Opts(K=K, bound="lanczos", eval=ev), info=True)
    torch.cuda.synchronize()
    assert abs(info["Lambda"] - Lo) <= LAM_TOL * Lo
    ref = ocpa.cpa_shrink(X, Shrinkage(0, tau), info["Lambda"], K)
    parity.check(Y.cpu().numpy(), ref, TOL32, X, f"lanczos shrink {m}x{n} {ev}")


def test_warm_start_from_the_ritz_vector():
    """The Ritz vector is the next call's start: one step from it gives its
    Rayleigh quotient, which matches the oracle's one step from the oracle's Ritz
    vector and is at least the converged theta up to rounding."""
    import torch
    import paper_1705_07112_amd as cpa
    X = synth.as_f32_exact(synth.dense_lowrank(150, 96, rank=4, noise=0.3, seed=7300))
    G = _gram(X)
    Lo, th, r, k, y = obound.lanczos_bound(G, seed=0, steps=12, tol=1e-7)[:5]
    L1 = obound.lanczos_bound(G, steps=1, v0=y)
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    cpa.spectral_bound(Xd, cpa.Opts(K=4, bound="lanczos", lanczos_steps=12))
    lam2, info2 = cpa.spectral_bound(Xd, cpa.Opts(K=4, bound="lanczos", lanczos_steps=1, warm_start=True))
    print(f"warm one step: gpu {info2['mu']:.12g} oracle {L1[1]:.12g} converged {th:.12g}", flush=True)
    assert abs(info2["mu"] - L1[1]) <= LAM_TOL * L1[1]
    assert info2["mu"] >= th * (1 - 1e-6)
    lam_cold, info_cold = cpa.spectral_bound(Xd, cpa.Opts(K=4, bound="lanczos", lanczos_steps=1))
    assert info2["mu"] > info_cold["mu"]


def test_sparsified_compact_block():
    """The compact block of the truncated transformed Gram (nonempty rows in
    ascending order, zero-padded to a multiple of 64), bound by Lanczos from the
    seeded start vector of the block's side; the shrink at that bound matches the
    oracle's sparsified shrink."""
    import torch
    import paper_1705_07112_amd as cpa
    X = synth.as_f32_exact(synth.block_smooth(512, 512, rank=4, noise=1e-3, seed=7400))
    T = sparsify.block_dct(512, 8)
    Phi, _ = sparsify.transformed_gram(X, T)
    keep = _gap_keep(Phi, 0.01)   # a keep count at a gap in |Phi|: FP32 and FP64 keep the same set
    eps = sparsify.kth_largest_abs(Phi, keep)
    Phil = sparsify.truncate(Phi, eps)
    rows = np.nonzero(np.any(Phil != 0.0, axis=1))[0]
    ns = rows.size
    nb = (ns + 63) // 64 * 64
    assert nb <= 256
    P = np.zeros((nb, nb))
    P[:ns, :ns] = Phil[np.ix_(rows, rows)]
    Lo = obound.lanczos_bound(P, seed=0, steps=12, tol=1e-7)[0]
    tau = 0.2 * math.sqrt(Lo)
    print(f"case sparsified lanczos: block {ns} -> {nb}", flush=True)
    Y, info = cpa.shrink_dense_sparsified(torch.from_numpy(X.astype(np.float32)).cuda(), cpa.soft(tau),
                                          cpa.Opts(K=20, bound="lanczos"), keep=keep, info=True)
    torch.cuda.synchronize()
    print(f"  gpu {info['Lambda']:.10g} oracle {Lo:.10g}", flush=True)
    assert abs(info["Lambda"] - Lo) <= 1e-5 * Lo
    # the Gram statistics stay intact beside the Lanczos slots
    fro = math.sqrt(float(np.sum((X.T @ X) ** 2)))
    assert abs(info["fro_gram"] - fro) <= 1e-5 * fro
    ref = sparsify.cpa_shrink_sparsified(X, Shrinkage(0, tau), info["Lambda"], 20, T, keep)[0]
    parity.check(Y.cpu().numpy(), ref, 1e-4, X, "sparsified lanczos")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_batched_lanczos_bound(precision):
    """Per-matrix k-step Lanczos inside the batched kernel against the oracle, and
    the shrink at each device bound."""
    import torch
    import paper_1705_07112_amd as cpa
    print(f"case batched lanczos {precision}", flush=True)
    shapes = [(64, 40), (64, 120), (64, 64), (40, 64), (17, 33), (64, 1), (3, 5), (64, 90)]
    mats = [synth.as_f32_exact(synth.dense_lowrank(a, b, rank=min(4, a, b), noise=0.2, seed=7500 + i))
            for i, (a, b) in enumerate(shapes)]
    ms = np.array([a.shape[0] for a in mats], dtype=np.int32)
    ns = np.array([a.shape[1] for a in mats], dtype=np.int32)
    offs = np.zeros(len(mats), dtype=np.int64)
    offs[1:] = np.cumsum([a.size for a in mats])[:-1]
    flat = np.concatenate([a.astype(np.float32).ravel() for a in mats])
    dev = "cuda"
    lam_out = torch.zeros(len(mats), dtype=torch.float64, device=dev)
    status = torch.full((len(mats),), -1, dtype=torch.int32, device=dev)
    taus = [0.3 * math.sqrt(float(np.linalg.eigvalsh(_gram(X))[-1])) for X in mats]
    recs = torch.frombuffer(bytearray(cpa.shrinkage_records([cpa.soft(t) for t in taus])), dtype=torch.uint8).to(dev)
    Y = cpa.shrink_batched(torch.from_numpy(flat).to(dev), torch.from_numpy(ms).to(dev), torch.from_numpy(ns).to(dev),
                           torch.from_numpy(offs).to(dev), cpa.soft(0.0),
                           cpa.Opts(K=16, bound="lanczos", precision=precision), shrink_per_matrix=recs,
                           lambda_out=lam_out, status=status)
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() == 0)
    Yh = Y.cpu().numpy()
    lam = lam_out.cpu().numpy()
    tol = TOL32 if precision == "fp32" else 1e-3
    for i, X in enumerate(mats):
        Lo = obound.lanczos_bound(_gram(X), seed=0, steps=12, tol=1e-7)[0]
        assert abs(lam[i] - Lo) <= LAM_TOL * Lo, (i, lam[i], Lo)
        ref = ocpa.cpa_shrink(X, Shrinkage(0, taus[i]), float(lam[i]), 16)
        Yi = Yh[offs[i]:offs[i] + X.size].reshape(X.shape).astype(np.float64)
        assert metrics.rel_fro(Yi, ref, X) <= tol, i


def test_sparsified_wide_compact_block():
    """A compact block wider than 256 (about 3% kept of a 1024 x 1024 transformed
    Gram) takes the multi-workgroup kernel.  Past the block-DC entries |Phi| has no
    2% gap, so the keep count sits at a 0.05% gap; entries that FP32 and FP64 might
    still order differently are some 1e-6 of lambda_max and leave the bound alone."""
    import torch
    import paper_1705_07112_amd as cpa
    X = synth.as_f32_exact(synth.block_smooth(1024, 1024, rank=4, noise=1e-3, seed=7450))
    T = sparsify.block_dct(1024, 8)
    Phi, _ = sparsify.transformed_gram(X, T)
    a = np.sort(np.abs(Phi).ravel())[::-1]
    cand = np.nonzero(a[:-1] / np.maximum(a[1:], 1e-300) > 1.0005)[0]
    keep = int(cand[np.argmin(np.abs(cand + 1 - int(0.03 * a.size)))] + 1)
    Phil = sparsify.truncate(Phi, sparsify.kth_largest_abs(Phi, keep))
    rows = np.nonzero(np.any(Phil != 0.0, axis=1))[0]
    ns = rows.size
    nb = (ns + 63) // 64 * 64
    print(f"case sparsified lanczos wide block: {ns} -> {nb}", flush=True)
    assert nb > 256
    P = np.zeros((nb, nb))
    P[:ns, :ns] = Phil[np.ix_(rows, rows)]
    Lo = obound.lanczos_bound(P, seed=0, steps=12, tol=1e-7)[0]
    _, info = cpa.shrink_dense_sparsified(torch.from_numpy(X.astype(np.float32)).cuda(), cpa.soft(1.0),
                                          cpa.Opts(K=20, bound="lanczos"), keep=keep, info=True)
    print(f"  gpu {info['Lambda']:.10g} oracle {Lo:.10g}", flush=True)
    assert abs(info["Lambda"] - Lo) <= 1e-5 * Lo
    fro = math.sqrt(float(np.sum((X.T @ X) ** 2)))
    assert abs(info["fro_gram"] - fro) <= 1e-5 * fro


def test_lanczos_refusals():
    import torch
    import paper_1705_07112_amd as cpa
    print("case lanczos refusals", flush=True)
    X = torch.randn(400, 300, device="cuda")
    with pytest.raises(cpa.CpaError) as e:          # Gram side above 4096
        cpa.spectral_bound(torch.randn(4200, 4100, device="cuda"), cpa.Opts(K=8, bound="lanczos"))
    assert e.value.status == cpa.ERR_UNSUPPORTED
    with pytest.raises(cpa.CpaError) as e:          # the FP64 path: 34 vectors of 32 exceed its 33 x 32 buffer
        cpa.shrink_dense(X[:33, :32].double().contiguous(), cpa.soft(1.0),
                         cpa.Opts(K=8, bound="lanczos", lanczos_steps=32))
    assert e.value.status == cpa.ERR_UNSUPPORTED
    with pytest.raises(cpa.CpaError) as e:          # at most 32 steps
        cpa.shrink_dense(X[:64, :32].contiguous(), cpa.soft(1.0), cpa.Opts(K=8, bound="lanczos", lanczos_steps=33))
    assert e.value.status == cpa.ERR_ARG
    rowptr = torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda")
    cols = torch.tensor([0, 4199], dtype=torch.int32, device="cuda")
    vals = torch.tensor([1.0, 2.0], device="cuda")
    with pytest.raises(cpa.CpaError) as e:          # the CSR path: n above 4096
        cpa.shrink_csr(2, 4200, rowptr, cols, vals, cpa.soft(0.1), cpa.Opts(K=4, bound="lanczos"))
    assert e.value.status == cpa.ERR_UNSUPPORTED


@pytest.mark.parametrize("shape", [(200, 120), (1100, 1024)])
def test_noalloc_entry_point_with_the_lanczos_bound(shape):
    """The allocation-free entry point runs the same Lanczos kernels (its Lanczos
    vectors in the static workspace's idle buffers) and returns the same bits."""
    import torch
    import paper_1705_07112_amd as cpa
    m, n = shape
    print(f"case noalloc lanczos {m}x{n}", flush=True)
    X = torch.from_numpy(synth.as_f32_exact(synth.dense_lowrank(m, n, rank=4, noise=0.2, seed=7600 + m))
                         .astype(np.float32)).cuda()
    opts = cpa.Opts(K=30, bound="lanczos")
    Y1, i1 = cpa.shrink_dense(X, cpa.soft(1.0), opts, info=True)
    Y2 = cpa.shrink_dense_noalloc(X, cpa.soft(1.0), opts, torch.empty_like(X))
    torch.cuda.synchronize()
    assert i1["power_iters_done"] >= 2
    assert torch.equal(Y1, Y2)
