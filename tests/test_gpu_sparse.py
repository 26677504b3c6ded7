"""Sparse (CSR) operator-form shrinkage and the SVT completion driver against
the FP64 oracle.  The oracle computes the same matrix from the densified S
(Algorithm 1); Lambda is passed explicitly for parity."""
import math

import numpy as np
import pytest

import synth
from tests import parity
from oracle import bound as obound
from oracle import cpa as ocpa
from oracle import drivers, metrics
from oracle.shrinkage import Shrinkage

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def _random_csr(m, n, frac, seed, empty_rows=(), empty_cols=()):
    g = synth.rng(seed)
    cnt = max(0, int(round(frac * m * n)))
    flat = np.sort(g.choice(m * n, size=cnt, replace=False)) if cnt else np.zeros(0, dtype=np.int64)
    rows, cols = flat // n, flat % n
    keep = ~np.isin(rows, list(empty_rows)) & ~np.isin(cols, list(empty_cols))
    rows, cols = rows[keep], cols[keep]
    vals = g.standard_normal(len(rows)).astype(np.float32)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    S = np.zeros((m, n))
    S[rows, cols] = vals
    return rowptr, cols.astype(np.int32), vals, S


def _gpu_csr(m, n, rowptr, cols, vals, sh_c, opts, info=False):
    import torch
    import paper_1705_07112_amd as cpa
    r = torch.from_numpy(rowptr).cuda()
    c = torch.from_numpy(cols).cuda()
    v = torch.from_numpy(vals).cuda()
    res = cpa.shrink_csr(m, n, r, c, v, sh_c, opts, info=info)
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("m,n,frac,K", [(64, 48, 0.1, 20), (300, 120, 0.05, 16), (2000, 400, 0.02, 25),
                                        (129, 129, 0.03, 7), (1100, 1025, 0.01, 3), (50, 1, 0.5, 5)])
def test_csr_matches_oracle(m, n, frac, K):
    import paper_1705_07112_amd as cpa
    rowptr, cols, vals, S = _random_csr(m, n, frac, 20000 + m + n, empty_rows=(0, 3), empty_cols=(1,))
    G = S.T @ S
    lmax = float(np.linalg.eigvalsh(G)[-1])
    Lam, tau = 1.01 * lmax, 0.3 * math.sqrt(lmax)
    Y = _gpu_csr(m, n, rowptr, cols, vals, cpa.soft(tau), cpa.Opts(K=K, Lambda=Lam)).cpu().numpy()
    ref = ocpa.cpa_shrink(S, Shrinkage(0, tau), Lam, K)
    parity.check(Y, ref, TOL32, S, f"csr {m}x{n} nnz={len(vals)} K={K}")


def test_csr_edge_cases():
    import torch
    import paper_1705_07112_amd as cpa
    # no nonzeros: Lambda = 0 and Y = 0
    rowptr = np.zeros(11, dtype=np.int32)
    Y, info = _gpu_csr(10, 4, rowptr, np.zeros(0, np.int32), np.zeros(0, np.float32), cpa.soft(1.0),
                       cpa.Opts(K=5), info=True)
    assert info["Lambda"] == 0.0 and torch.count_nonzero(Y).item() == 0
    # one nonzero: singular value |s|, soft shrink to (|s| - tau)_+ up to the CPA error
    rowptr = np.array([0, 0, 1, 1], dtype=np.int32)
    Y, info = _gpu_csr(3, 2, rowptr, np.array([1], np.int32), np.array([3.0], np.float32), cpa.soft(1.0),
                       cpa.Opts(K=30), info=True)
    ref = ocpa.cpa_shrink(np.array([[0, 0], [0, 3.0], [0, 0]]), Shrinkage(0, 1.0), info["Lambda"], 30)
    assert metrics.rel_fro(Y.cpu().numpy(), ref) <= TOL32
    with pytest.raises(cpa.CpaError):
        _gpu_csr(2, 3, np.array([0, 0, 0], np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32),
                 cpa.soft(1.0), cpa.Opts(K=3))


def test_csr_operator_bound_matches_oracle():
    import paper_1705_07112_amd as cpa
    rowptr, cols, vals, S = _random_csr(2000, 400, 0.02, 20500)
    G = S.T @ S
    lam_o = obound.power_bound(G, seed=0, max_iter=200, tol=1e-9, cap=float(np.trace(G)))[0]
    _, info = _gpu_csr(2000, 400, rowptr, cols, vals, cpa.soft(1.0),
                       cpa.Opts(K=2, power_iters=200, power_tol=1e-9), info=True)
    print(f"operator bound gpu={info['Lambda']:.10g} oracle={lam_o:.10g}", flush=True)
    assert abs(info["Lambda"] - lam_o) <= 2e-6 * lam_o


@pytest.mark.parametrize("ev", ["auto", "recurrence"])
def test_csr_full_size_sampled_rows(ev):
    """20000 x 4000, 2% observed (1.6M entries), K = 25, on both routes (the
    operator form is eval = recurrence): rows from the first, middle and last
    row panels of the result against the oracle's Y-form on the same rows, with
    the Gram from a sparse product."""
    import scipy.sparse as sp
    import torch
    import paper_1705_07112_amd as cpa
    u, v, rowptr, cols, vals = synth.completion()
    m, n = 20000, 4000
    S = sp.csr_matrix((vals.astype(np.float64), cols, rowptr), shape=(m, n))
    G = (S.T @ S).toarray()
    lam = float(obound.power_bound(G, seed=0, max_iter=300, tol=1e-10, cap=float(np.trace(G)))[0])
    tau = 0.5 * math.sqrt(lam)
    Y = _gpu_csr(m, n, rowptr, cols, vals, cpa.soft(tau), cpa.Opts(K=25, Lambda=lam, eval=ev))
    rows = np.r_[0:8, 777, 9996:10004, 19992:20000]
    got = Y[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
    ref = ocpa.cpa_rows_yform(G, S[rows].toarray(), Shrinkage(0, tau), lam, 25)
    parity.check(got, ref, TOL32, label=f"csr full size sampled rows {ev}")


def test_svt_completion_matches_oracle():
    import torch
    import paper_1705_07112_amd as cpa
    m, n, r = 240, 120, 3
    g = synth.rng(20600)
    M = g.standard_normal((m, r)) @ g.standard_normal((r, n))
    idx = np.sort(g.choice(m * n, size=int(0.2 * m * n), replace=False))
    rows, cols = idx // n, idx % n
    vals = M[rows, cols].astype(np.float32)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    tau, step, iters, K = 5 * math.sqrt(m * n), 1.2 * m * n / len(idx), 15, 25
    res = torch.zeros(iters, dtype=torch.float64, device="cuda")
    X, k0 = cpa.svt_complete(m, n, torch.from_numpy(rowptr).cuda(), torch.from_numpy(cols.astype(np.int32)).cuda(),
                             torch.from_numpy(vals).cuda(), tau, step, iters, cpa.Opts(K=K, warm_start=True),
                             resid=res)
    torch.cuda.synchronize()
    Xo, res_o, k0_o = drivers.svt_complete(m, n, rows, cols, vals.astype(np.float64), tau, step, iters, K)
    e = metrics.rel_fro(X.cpu().numpy(), Xo)
    print(f"svt k0 gpu={k0} oracle={k0_o} X drift={e:.2e} resid {res.cpu().numpy()[-3:]} vs {res_o[-3:]}", flush=True)
    assert k0 == k0_o
    assert e < 1e-3
    assert np.max(np.abs(res.cpu().numpy() - np.array(res_o))) < 1e-3


@pytest.mark.parametrize("ev", ["recurrence", "polynomial"])
@pytest.mark.parametrize("m,n,frac,K", [(300, 120, 0.05, 25), (257, 131, 0.03, 9), (64, 63, 0.2, 64),
                                        (500, 37, 0.02, 2), (129, 129, 0.1, 100)])
def test_csr_both_evaluation_routes(ev, m, n, frac, K):
    """The operator-form recurrence and the matrix-polynomial route (Gram S^T S,
    polynomial on the n x n side, one product S p) against the same oracle; odd n
    exercises the element-wise loads of p."""
    import paper_1705_07112_amd as cpa
    rowptr, cols, vals, S = _random_csr(m, n, frac, 4400 + m + n + K)
    G = S.T @ S
    lmax = float(np.linalg.eigvalsh(G)[-1])
    Lam, tau = 1.01 * lmax, 0.3 * math.sqrt(lmax)
    Y = _gpu_csr(m, n, rowptr, cols, vals, cpa.soft(tau), cpa.Opts(K=K, Lambda=Lam, eval=ev)).cpu().numpy()
    ref = ocpa.cpa_shrink(S, Shrinkage(0, tau), Lam, K)
    parity.check(Y.astype(np.float64), ref, TOL32, S, f"csr {m}x{n} K={K} eval={ev}")


def test_csr_damped_coefficients_match_oracle():
    import paper_1705_07112_amd as cpa
    m, n, K = 300, 120, 40
    rowptr, cols, vals, S = _random_csr(m, n, 0.05, 20400, empty_rows=(0,), empty_cols=(1,))
    lmax = float(np.linalg.eigvalsh(S.T @ S)[-1])
    Lam, tau = 1.01 * lmax, 0.3 * math.sqrt(lmax)
    for ev in ("recurrence", "polynomial"):
        Y = _gpu_csr(m, n, rowptr, cols, vals, cpa.hard(tau),
                     cpa.Opts(K=K, Lambda=Lam, eval=ev, damping="jackson")).cpu().numpy()
        ref = ocpa.cpa_shrink(S, Shrinkage(1, tau), Lam, K, damping="jackson")
        parity.check(Y, ref, TOL32, S, f"csr damped {ev}")


def _svt_problem(m, n, r, frac, seed):
    g = synth.rng(seed)
    M = g.standard_normal((m, r)) @ g.standard_normal((r, n))
    idx = np.sort(g.choice(m * n, size=int(frac * m * n), replace=False))
    rows, cols = idx // n, idx % n
    vals = M[rows, cols].astype(np.float32)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    return M, rows, cols, vals, rowptr


@pytest.mark.parametrize("ev,bound", [("auto", "power"), ("recurrence", "power"), ("auto", "lanczos")])
def test_svt_iterations_from_the_gpu_state(ev, bound):
    """Gated like the ADMM driver: the GPU's own iterate Y^t (on the observed set)
    after five iterations, then one and two more iterations continued from it;
    the oracle applies its shrink to the same Y^t at the bounds the GPU reports
    and the SVT update, and X (whole matrix) and Y (observed set) must agree to
    the FP32 tolerance.  On the matrix-polynomial route the first of the two
    iterations forms only the observed entries of X.  Every reported bound is at
    least the top eigenvalue of its iterate's Gram (the Lanczos rule warm-starts
    from the previous Ritz vector)."""
    import torch
    import paper_1705_07112_amd as cpa
    m, n, K = 600, 200, 25
    M, rows, cols, vals, rowptr = _svt_problem(m, n, 3, 0.2, 20700)
    tau, step = 5 * math.sqrt(m * n), 1.2 * m * n / len(vals)
    r_d = torch.from_numpy(rowptr).cuda()
    c_d = torch.from_numpy(cols.astype(np.int32)).cuda()
    v_d = torch.from_numpy(vals).cuda()
    opts = cpa.Opts(K=K, warm_start=True, eval=ev, bound=bound)
    y5 = torch.empty(len(vals), dtype=torch.float32, device="cuda")
    cpa.svt_complete(m, n, r_d, c_d, v_d, tau, step, 5, opts, y_end=y5)
    Y5 = np.zeros((m, n))
    Y5[rows, cols] = y5.cpu().numpy()
    sh = Shrinkage(0, tau)
    for extra in (1, 2):
        lam = torch.zeros(extra, dtype=torch.float64, device="cuda")
        yend = torch.empty_like(y5)
        X, _ = cpa.svt_complete(m, n, r_d, c_d, v_d, tau, step, extra, opts, y_start=y5, y_end=yend, lambdas=lam)
        torch.cuda.synchronize()
        Yo = Y5.copy()
        for t in range(extra):
            lmax = float(np.linalg.eigvalsh(Yo.T @ Yo)[-1])
            assert float(lam[t].item()) >= lmax * (1 - 1e-6), (bound, t, float(lam[t].item()), lmax)
            Xo = ocpa.cpa_shrink(Yo, sh, float(lam[t].item()), K)
            Yo[rows, cols] += step * (vals.astype(np.float64) - Xo[rows, cols])
        parity.check(X.cpu().numpy(), Xo, TOL32, label=f"svt X after {extra} from Y^5 ({ev})")
        parity.check(yend.cpu().numpy(), Yo[rows, cols], TOL32, label=f"svt Y on the observed set ({ev})")


def test_csr_polynomial_route_above_the_lds_rows():
    """n = 4100 > 4096: the Gram falls back to the product with the densified S
    (the row kernel's LDS rows hold 4096 floats); sampled rows against the oracle."""
    import scipy.sparse as sp
    import torch
    import paper_1705_07112_amd as cpa
    m, n = 4300, 4100
    rowptr, cols, vals, _ = _random_csr(m, n, 0.002, 20800)
    S = sp.csr_matrix((vals.astype(np.float64), cols, rowptr), shape=(m, n))
    G = (S.T @ S).toarray()
    lam = 1.01 * float(np.linalg.eigvalsh(G)[-1])
    tau = 0.3 * math.sqrt(lam)
    Y = _gpu_csr(m, n, rowptr, cols, vals, cpa.soft(tau), cpa.Opts(K=16, Lambda=lam, eval="polynomial"))
    rsel = np.r_[0:4, 2150, 4296:4300]
    got = Y[torch.from_numpy(rsel).cuda()].cpu().numpy().astype(np.float64)
    ref = ocpa.cpa_rows_yform(G, S[rsel].toarray(), Shrinkage(0, tau), lam, 16)
    parity.check(got, ref, TOL32, label="csr n=4100 polynomial (densified Gram)")


def test_csr_rejects_unsorted_or_repeated_columns():
    import paper_1705_07112_amd as cpa
    for cols in ([2, 1, 3], [1, 1, 3]):
        rowptr = np.array([0, 3, 3, 3, 3], dtype=np.int32)
        with pytest.raises(cpa.CpaError) as e:
            _gpu_csr(4, 4, rowptr, np.array(cols, np.int32), np.ones(3, np.float32), cpa.soft(0.1), cpa.Opts(K=5))
        assert e.value.status == cpa.ERR_ARG


@pytest.mark.parametrize("m,n,frac,steps,tol", [(2000, 400, 0.02, 12, 1e-7), (300, 120, 0.05, 32, 0.0),
                                                (64, 48, 0.1, 5, 0.0), (5000, 1500, 0.004, 12, 1e-7),
                                                (40, 3, 0.3, 12, 0.0)])
def test_csr_lanczos_bound_matches_oracle(m, n, frac, steps, tol):
    """The Lanczos bound on the operator form S^T S (two sparse products per step)
    against the oracle's lanczos_bound on the densified Gram with the same cap
    (tr G = ||S||_F^2), and the shrink at the device's bound against the oracle's
    CPA.  S holds FP32 values and both sides accumulate in FP64: the bounds agree
    to rounding (1e-8 relative; 2e-6 where the early stop lands one step apart)."""
    import paper_1705_07112_amd as cpa
    print(f"case csr lanczos {m}x{n} steps={steps} tol={tol}", flush=True)
    rowptr, cols, vals, S = _random_csr(m, n, frac, 20800 + m + n, empty_rows=(0,), empty_cols=(1,))
    G = S.T @ S
    Lo, th_o, r_o, k_o, *_ = obound.lanczos_bound(G, seed=0, steps=steps, tol=tol, cap=float(np.trace(G)))
    lmax = float(np.linalg.eigvalsh(G)[-1])
    tau = 0.3 * math.sqrt(lmax)
    Y, info = _gpu_csr(m, n, rowptr, cols, vals, cpa.soft(tau),
                       cpa.Opts(K=16, bound="lanczos", lanczos_steps=steps, power_tol=tol), info=True)
    print(f"  gpu {info['Lambda']:.15g} oracle {Lo:.15g} steps {info['power_iters_done']}/{k_o}", flush=True)
    if tol == 0.0:
        assert info["power_iters_done"] == k_o
    else:
        assert abs(info["power_iters_done"] - k_o) <= 1
    assert abs(info["Lambda"] - Lo) <= (1e-8 if info["power_iters_done"] == k_o else 2e-6) * Lo
    if steps >= 12:
        assert info["Lambda"] >= lmax * (1 - 1e-6)
    ref = ocpa.cpa_shrink(S, Shrinkage(0, tau), info["Lambda"], 16)
    parity.check(Y.cpu().numpy(), ref, TOL32, S, f"csr lanczos {m}x{n}")
