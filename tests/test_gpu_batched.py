"""Batched persistent shrinkage (one workgroup per small matrix) against the
FP64 oracle, matrix by matrix.  Lambda is passed per matrix for parity; a
separate test compares the in-kernel power-iteration bound with the oracle's."""
import ctypes
import math

import numpy as np
import pytest

import synth
from tests import parity
from oracle import bound as obound
from oracle import cpa as ocpa
from oracle import metrics
from oracle.shrinkage import Shrinkage

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL_SPLIT = 1e-3   # split-precision products (bf16 hi/lo, FP32 accumulation)


def _pack(mats):
    ms = np.array([a.shape[0] for a in mats], dtype=np.int32)
    ns = np.array([a.shape[1] for a in mats], dtype=np.int32)
    offs = np.zeros(len(mats), dtype=np.int64)
    offs[1:] = np.cumsum([a.size for a in mats])[:-1]
    flat = np.concatenate([a.astype(np.float32).ravel() for a in mats]) if mats else np.zeros(0, np.float32)
    return flat, ms, ns, offs


def _gram(X):
    return X.T @ X if X.shape[0] >= X.shape[1] else X @ X.T


def _run(mats, shr, K, mode="given", lams=None, power_kw=None, precision="fp32"):
    import torch
    import paper_1705_07112_amd as cpa
    flat, ms, ns, offs = _pack(mats)
    dev = "cuda"
    X = torch.from_numpy(flat).to(dev)
    m = torch.from_numpy(ms).to(dev)
    n = torch.from_numpy(ns).to(dev)
    off = torch.from_numpy(offs).to(dev)
    recs = torch.frombuffer(bytearray(cpa.shrinkage_records(shr)), dtype=torch.uint8).to(dev)
    lam_in = torch.from_numpy(np.array(lams, dtype=np.float64)).to(dev) if lams is not None else None
    lam_out = torch.zeros(len(mats), dtype=torch.float64, device=dev)
    status = torch.full((len(mats),), -1, dtype=torch.int32, device=dev)
    opts = cpa.Opts(K=K, bound=mode, precision=precision, **(power_kw or {}))
    if mode == "given":
        opts.Lambda = 0.0
    Y = cpa.shrink_batched(X, m, n, off, cpa.soft(0.0), opts, shrink_per_matrix=recs, Lambda=lam_in,
                           lambda_out=lam_out, status=status)
    torch.cuda.synchronize()
    Yh = Y.cpu().numpy()
    outs = [Yh[offs[i]:offs[i] + mats[i].size].reshape(mats[i].shape).astype(np.float64) for i in range(len(mats))]
    return outs, lam_out.cpu().numpy(), status.cpu().numpy()


def _mats_and_params(shapes, seed):
    import paper_1705_07112_amd as cpa
    mats, shr_c, shr_o, lams = [], [], [], []
    for i, (mm, nn) in enumerate(shapes):
        X = synth.as_f32_exact(synth.dense_lowrank(mm, nn, rank=min(4, mm, nn), noise=0.2, seed=seed + i))
        lmax = float(np.linalg.eigvalsh(_gram(X))[-1]) if X.size else 0.0
        tau = 0.4 * math.sqrt(lmax)
        if i % 3 == 0:
            shr_c.append(cpa.soft(tau)); shr_o.append(Shrinkage(0, tau))
        elif i % 3 == 1:
            shr_c.append(cpa.hard(tau)); shr_o.append(Shrinkage(1, tau))
        else:
            wc, ws = 0.3 * tau * tau, 0.05 * lmax
            shr_c.append(cpa.weighted_fn(wc, ws, 1e-3)); shr_o.append(Shrinkage(3, 0.0, wc, ws, 1e-3))
        mats.append(X)
        lams.append(1.01 * lmax)
    return mats, shr_c, shr_o, lams


SHAPES = [(64, 40), (64, 120), (64, 64), (64, 63), (64, 65), (40, 64), (120, 64), (1, 1), (3, 5), (5, 3),
          (16, 17), (17, 16), (64, 128), (128, 64), (33, 100), (100, 33), (2, 128), (128, 2)]


@pytest.mark.parametrize("K", [1, 2, 16, 30])
def test_batched_matches_oracle_given_lambda(K):
    mats, shr_c, shr_o, lams = _mats_and_params(SHAPES, 11000 + K)
    outs, lam_out, status = _run(mats, shr_c, K, "given", lams)
    assert np.all(status == 0)
    worst = 0.0
    for X, Y, sh, lam in zip(mats, outs, shr_o, lams):
        ref = ocpa.cpa_shrink(X, sh, lam, K)
        err, mx = parity.errors(Y, ref, X)
        worst = max(worst, err, mx)
        assert err <= TOL32 and mx <= parity.ELEM_FACTOR * TOL32, (X.shape, K, err, mx)
    print(f"batched K={K}: worst rel_fro / max_elem {worst:.3e} over {len(mats)} matrices", flush=True)
    assert np.allclose(lam_out, lams)


@pytest.mark.parametrize("K", [1, 2, 16, 30])
def test_batched_split_precision_matches_oracle(K):
    """Split-precision recurrence (bf16 hi/lo products with FP32 accumulation) on
    the same shapes and shrinkages, within the split-precision bar."""
    mats, shr_c, shr_o, lams = _mats_and_params(SHAPES, 11500 + K)
    outs, lam_out, status = _run(mats, shr_c, K, "given", lams, precision="bf16x3")
    assert np.all(status == 0)
    worst = 0.0
    for X, Y, sh, lam in zip(mats, outs, shr_o, lams):
        ref = ocpa.cpa_shrink(X, sh, lam, K)
        err, mx = parity.errors(Y, ref, X)
        worst = max(worst, err, mx)
        assert err <= TOL_SPLIT and mx <= parity.ELEM_FACTOR * TOL_SPLIT, (X.shape, K, err, mx)
    print(f"batched split K={K}: worst rel_fro {worst:.3e} over {len(mats)} matrices", flush=True)
    assert np.allclose(lam_out, lams)


def test_batched_split_precision_power_bound_and_growth_check():
    """Split precision with the in-kernel power bound and the growth check on
    patch groups: the bound equals the FP32 path's (the Gram and the iteration
    do not depend on the product precision) and the shrink is within the bar."""
    flat, ms, ns, offs, ranks, noises = synth.patch_groups(batch=64, seed=12500)
    mats = [flat[offs[i]:offs[i] + ms[i] * ns[i]].reshape(ms[i], ns[i]).astype(np.float64) for i in range(64)]
    import paper_1705_07112_amd as cpa
    shr_c = [cpa.soft(0.3 * math.sqrt(float(np.linalg.eigvalsh(_gram(X))[-1]))) for X in mats]
    taus = [r.tau for r in shr_c]
    kw = {"power_iters": 200, "power_tol": 1e-9, "check": 1}
    o32, l32, s32 = _run(mats, shr_c, 16, "power", None, kw)
    osp, lsp, ssp = _run(mats, shr_c, 16, "power", None, kw, precision="bf16x3")
    assert np.all(ssp == 0) and np.all(s32 == 0)
    assert np.array_equal(l32, lsp)
    worst = 0.0
    for X, Y, tau, lam in zip(mats, osp, taus, lsp):
        ref = ocpa.cpa_shrink(X, Shrinkage(0, tau), lam, 16)
        worst = max(worst, metrics.rel_fro(Y, ref, X))
    print(f"patch groups split: shrink rel_fro {worst:.2e}", flush=True)
    assert worst <= TOL_SPLIT


def test_batched_patch_groups_and_power_bound():
    flat, ms, ns, offs, ranks, noises = synth.patch_groups(batch=96, seed=12000)
    mats = [flat[offs[i]:offs[i] + ms[i] * ns[i]].reshape(ms[i], ns[i]).astype(np.float64) for i in range(96)]
    import paper_1705_07112_amd as cpa
    sig = 0.2
    shr_c, shr_o = [], []
    for X in mats:
        nj = X.shape[1]
        wc, ws = 2 * math.sqrt(2) * sig * sig * math.sqrt(nj), (8 + math.sqrt(nj)) ** 2 * sig * sig
        shr_c.append(cpa.weighted_fn(wc, ws, 1e-6))
        shr_o.append(Shrinkage(3, 0.0, wc, ws, 1e-6))
    outs, lam_out, status = _run(mats, shr_c, 16, "power", None, {"power_iters": 200, "power_tol": 1e-9})
    assert np.all(status == 0)
    worst_l = worst_y = 0.0
    for X, Y, sh, lam_g in zip(mats, outs, shr_o, lam_out):
        lam_o = obound.power_bound(_gram(X), seed=0, max_iter=200, tol=1e-9)[0]
        worst_l = max(worst_l, abs(lam_g - lam_o) / lam_o)
        # parity of the shrink at the device's bound
        ref = ocpa.cpa_shrink(X, sh, lam_g, 16)
        worst_y = max(worst_y, metrics.rel_fro(Y, ref, X))
    print(f"patch groups: bound rel diff {worst_l:.2e}, shrink rel_fro {worst_y:.2e}", flush=True)
    assert worst_l <= 2e-6
    assert worst_y <= TOL32


def test_batched_rejects_out_of_range_shapes():
    mats, shr_c, _, lams = _mats_and_params([(65, 70), (64, 129), (64, 40)], 13000)
    outs, _, status = _run(mats, shr_c, 8, "given", lams)
    assert list(status) == [2, 2, 0]


def test_batched_binding_checks_its_tensors():
    """The binding rejects tensors of the wrong type, device or length, and
    matrices that extend past the end of X, before anything reaches the library."""
    import torch
    import paper_1705_07112_amd as cpa
    X = torch.zeros(64 * 40 + 64 * 50, device="cuda")
    m = torch.tensor([64, 64], dtype=torch.int32, device="cuda")
    n = torch.tensor([40, 50], dtype=torch.int32, device="cuda")
    off = torch.tensor([0, 64 * 40], dtype=torch.int64, device="cuda")
    opts = cpa.Opts(K=8)
    cpa.shrink_batched(X, m, n, off, cpa.soft(1.0), opts)
    with pytest.raises(TypeError):
        cpa.shrink_batched(X, m.long(), n, off, cpa.soft(1.0), opts)
    with pytest.raises(TypeError):
        cpa.shrink_batched(X, m, n, off.int(), cpa.soft(1.0), opts)
    with pytest.raises(TypeError):
        cpa.shrink_batched(X, m, n.cpu(), off, cpa.soft(1.0), opts)
    with pytest.raises(ValueError):
        cpa.shrink_batched(X, m, n[:1], off, cpa.soft(1.0), opts)
    with pytest.raises(ValueError):
        cpa.shrink_batched(X, m, n, off, cpa.soft(1.0), opts,
                           lambda_out=torch.zeros(1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        cpa.shrink_batched(X, m, n, off + 1, cpa.soft(1.0), opts)
    with pytest.raises(ValueError):
        cpa.BatchedPlan(X[:100], m, n, off, cpa.soft(1.0), opts)


def test_batched_rejects_damping():
    """Coefficient damping is not available on the batched path (checked before
    any launch)."""
    import paper_1705_07112_amd as cpa
    mats, shr_c, _, lams = _mats_and_params([(64, 40)], 13100)
    with pytest.raises(cpa.CpaError):
        _run(mats, shr_c, 8, "given", lams, power_kw={"damping": "jackson"})


def test_converged_power_bound_matches_oracle_on_hard_cases():
    """Converged power bounds (tol 1e-12) on matrices whose iteration stops on the
    tolerance late, including one whose top two eigenvalues nearly coincide; the
    wave that runs the iteration must leave the loop together (regression: a
    per-lane exit once returned about half of lambda_max here)."""
    import paper_1705_07112_amd as cpa
    flat, ms, ns, offs, _, _ = synth.patch_groups(batch=32768, rank_range=(1, 16), noise_range=(0.05, 0.5),
                                                  seed=synth.BASE_SEED + 4)
    g = np.random.Generator(np.random.PCG64(5))
    pick = [10625, 628, 1000, 1079, 2065] + sorted(g.choice(32768, size=120, replace=False).tolist())
    mats = [flat[offs[i]:offs[i] + ms[i] * ns[i]].reshape(ms[i], ns[i]).astype(np.float64) for i in pick]
    shr = [cpa.soft(0.0)] * len(mats)
    for batch in (mats, mats[:1]):
        _, lam_out, status = _run(batch, shr[:len(batch)], 2, "power", None,
                                  {"power_iters": 1000, "power_tol": 1e-12, "margin": 0.0})
        assert np.all(status == 0)
        for X, lg in zip(batch, lam_out):
            lo = obound.power_bound(_gram(X), seed=0, max_iter=1000, tol=1e-12, delta=0.0)[0]
            assert abs(lg - lo) <= 1e-4 * lo, (lg, lo)


def _patch_batch(batch, seed, extra_shapes=()):
    import torch
    import paper_1705_07112_amd as cpa
    flat, ms, ns, offs, _, _ = synth.patch_groups(batch=batch, seed=seed)
    mats = [flat[offs[i]:offs[i] + ms[i] * ns[i]].reshape(ms[i], ns[i]) for i in range(batch)]
    for k, (mm, nn) in enumerate(extra_shapes):
        mats.append(synth.as_f32_exact(synth.dense_lowrank(mm, nn, rank=2, noise=0.1, seed=seed + 100 + k)))
    flat, ms, ns, offs = _pack(mats)
    dev = "cuda"
    t = lambda a: torch.from_numpy(a).to(dev)
    sig = 0.2
    recs = [cpa.weighted_fn(2 * math.sqrt(2) * sig * sig * math.sqrt(float(nj)), (8 + math.sqrt(float(nj))) ** 2 * sig * sig,
                            1e-6) for nj in ns]
    rec_t = torch.frombuffer(bytearray(cpa.shrinkage_records(recs)), dtype=torch.uint8).to(dev)
    return t(flat), t(ms), t(ns), t(offs), rec_t


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_plan_replays_match_direct_calls_bitwise(precision):
    """A tuned plan (captured graph) gives the same bits as cpa_shrink_batched on
    the same inputs, on every replay, also after X changes between replays."""
    import torch
    import paper_1705_07112_amd as cpa
    X, m, n, off, rec_t = _patch_batch(700, 12600, extra_shapes=[(70, 70), (5, 3), (64, 130)])
    batch = int(m.numel())
    opts = cpa.Opts(K=16, precision=precision, check=True)
    lam_p = torch.zeros(batch, dtype=torch.float64, device="cuda")
    st_p = torch.full((batch,), -1, dtype=torch.int32, device="cuda")
    # skipped matrices (shapes outside the limits) are never written: start both outputs at zero
    plan = cpa.BatchedPlan(X, m, n, off, cpa.soft(0.0), opts, shrink_per_matrix=rec_t, out=torch.zeros_like(X),
                           lambda_out=lam_p, status=st_p)
    tun = plan.tuning
    print(f"plan {precision}: {tun}", flush=True)
    assert tun["candidates"] >= 4 and tun["best_us"] > 0 and tun["default_us"] > 0
    assert tun["best_us"] <= tun["default_us"] * 1.0000001
    for rep in range(3):
        if rep == 2:
            X.mul_(0.5).add_(0.01)   # new contents, same shapes
        Yp = plan.run().clone()
        lp, sp = lam_p.clone(), st_p.clone()
        torch.cuda.synchronize()
        lam_d = torch.zeros_like(lam_p)
        st_d = torch.full_like(st_p, -1)
        Yd = cpa.shrink_batched(X, m, n, off, cpa.soft(0.0), opts, shrink_per_matrix=rec_t, out=torch.zeros_like(X),
                                lambda_out=lam_d, status=st_d)
        torch.cuda.synchronize()
        assert torch.equal(Yp, Yd), rep
        assert torch.equal(lp, lam_d), rep
        assert torch.equal(sp, st_d), rep
        assert int((sp == 2).sum()) == 2 and int((sp == 0).sum()) + int((sp == 1).sum()) == batch - 2
    plan.close()


def test_untuned_plan_and_empty_batch():
    import torch
    import paper_1705_07112_amd as cpa
    X, m, n, off, rec_t = _patch_batch(50, 12700)
    plan = cpa.BatchedPlan(X, m, n, off, cpa.soft(0.0), cpa.Opts(K=8), shrink_per_matrix=rec_t, tune=False)
    tun = plan.tuning
    assert tun["candidates"] == 0 and tun["best_us"] == 0.0 and tun["pair"] == 2 and tun["order"] == "index"
    Yp = plan.run().clone()
    Yd = cpa.shrink_batched(X, m, n, off, cpa.soft(0.0), cpa.Opts(K=8), shrink_per_matrix=rec_t)
    torch.cuda.synchronize()
    assert torch.equal(Yp, Yd)
    plan.close()
    e32 = torch.zeros(0, dtype=torch.int32, device="cuda")
    e64 = torch.zeros(0, dtype=torch.int64, device="cuda")
    ef = torch.zeros(0, dtype=torch.float32, device="cuda")
    empty = cpa.BatchedPlan(ef, e32, e32, e64, cpa.soft(1.0), cpa.Opts(K=8))
    empty.run()
    torch.cuda.synchronize()
    assert empty.tuning["candidates"] == 0
    empty.close()
