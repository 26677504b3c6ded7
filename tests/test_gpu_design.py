"""GPU parity of caller-given coefficients (opts.coeffs): other polynomial designs
of Sec. IV-B (least squares and minimax, eq. (l_p_norm_for_approximation)) run
through the same device evaluation as CPA.  The expected value is the oracle's
Chebyshev matrix sum (Algorithm 1, steps 5-10) of the oracle's design; the device
receives the library's design (host FP64), so the whole path is covered.  FP32
tolerance as the dense path: relative Frobenius error <= 1e-5."""
import math

import numpy as np
import pytest

import synth
from tests import parity
from oracle import cpa as ocpa
from oracle import design as odesign
from oracle.shrinkage import soft

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def _problem(m, n, seed):
    X = synth.as_f32_exact(synth.dense_lowrank(m, n, rank=min(4, m, n), noise=0.2, seed=seed))
    G = X.T @ X if m >= n else X @ X.T
    lmax = float(np.linalg.eigvalsh(G)[-1])
    return X, 1.01 * lmax, 0.4 * math.sqrt(lmax)


def _oracle(X, c, Lam):
    Phi, side = ocpa.gram(X)
    H = ocpa.chebyshev_matrix_sum(Phi, c, Lam)
    return X @ H if side == "right" else H @ X


def _designs(tau, Lam, K, kind):
    import paper_1705_07112_amd as cpa
    if kind == "lsq":
        ref = odesign.lsq(soft(tau), Lam, K, 2000)
    else:
        ref = odesign.minimax(soft(tau), Lam, K, 8000)[0]
    lib_c, _ = cpa.design_coeffs(cpa.soft(tau), Lam, K, kind)
    return ref, lib_c


@pytest.mark.parametrize("kind", ["lsq", "minimax"])
@pytest.mark.parametrize("ev", ["recurrence", "polynomial"])
@pytest.mark.parametrize("m,n,K", [(300, 200, 10), (300, 200, 30), (150, 400, 17), (130, 70, 1), (65, 64, 2)])
def test_designs_match_oracle(kind, ev, m, n, K):
    import torch
    import paper_1705_07112_amd as cpa
    print(f"case design={kind} eval={ev} m={m} n={n} K={K}", flush=True)
    X, Lam, tau = _problem(m, n, seed=7 + K)
    ref_c, lib_c = _designs(tau, Lam, K, kind)
    ref = _oracle(X, ref_c, Lam)
    c = torch.from_numpy(lib_c).cuda()
    Y = cpa.shrink_dense(torch.from_numpy(X.astype(np.float32)).cuda(), cpa.soft(tau),
                         cpa.Opts(K=K, bound="given", Lambda=Lam, eval=ev, coeffs=c))
    torch.cuda.synchronize()
    parity.check(Y.cpu().numpy(), ref, TOL32, X, f"{kind} {ev} {m}x{n} K={K}")


@pytest.mark.parametrize("kind", ["lsq", "minimax"])
def test_designs_full_size(kind):
    """The 1024 x 1024 frames of the RPCA workload at K = 20, matrix-polynomial route
    (the launch configuration of the design comparison)."""
    import torch
    import paper_1705_07112_amd as cpa
    print(f"case design={kind} 1024x1024 K=20", flush=True)
    I = synth.as_f32_exact(synth.rpca_frames(1024, 1024, seed=3)[0])
    G = I.T @ I
    Lam = 1.01 * float(np.linalg.eigvalsh(G)[-1])
    tau = 0.05 * math.sqrt(Lam)
    ref_c, lib_c = _designs(tau, Lam, 20, kind)
    ref = I @ ocpa.chebyshev_matrix_sum(G, ref_c, Lam)
    Y = cpa.shrink_dense(torch.from_numpy(I.astype(np.float32)).cuda(), cpa.soft(tau),
                         cpa.Opts(K=20, bound="given", Lambda=Lam, eval="polynomial",
                                  coeffs=torch.from_numpy(lib_c).cuda()))
    torch.cuda.synchronize()
    parity.check(Y.cpu().numpy(), ref, TOL32, I, f"{kind} full size")


def test_given_coefficients_on_the_csr_and_noalloc_paths():
    import torch
    import paper_1705_07112_amd as cpa
    print("case csr + noalloc with minimax coefficients", flush=True)
    g = synth.rng(11)
    m, n, frac, K = 400, 150, 0.05, 12
    mask = g.random((m, n)) < frac
    S = np.where(mask, g.standard_normal((m, n)), 0.0).astype(np.float32).astype(np.float64)
    lmax = float(np.linalg.eigvalsh(S.T @ S)[-1])
    Lam, tau = 1.01 * lmax, 0.3 * math.sqrt(lmax)
    ref_c, lib_c = _designs(tau, Lam, K, "minimax")
    ref = _oracle(S, ref_c, Lam)
    rows, cols = np.nonzero(mask)
    rowptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=m))]).astype(np.int32)
    vals = S[rows, cols].astype(np.float32)
    c = torch.from_numpy(lib_c).cuda()
    for ev in ("recurrence", "polynomial"):
        opts = cpa.Opts(K=K, bound="given", Lambda=Lam, eval=ev, coeffs=c)
        Y = cpa.shrink_csr(m, n, torch.from_numpy(rowptr).cuda(), torch.from_numpy(cols.astype(np.int32)).cuda(),
                           torch.from_numpy(vals).cuda(), cpa.soft(tau), opts)
        torch.cuda.synchronize()
        parity.check(Y.cpu().numpy(), ref, TOL32, S, f"csr {ev}")
    Xd = torch.from_numpy(S.astype(np.float32)).cuda()
    opts = cpa.Opts(K=K, bound="given", Lambda=Lam, coeffs=c)
    Y1 = cpa.shrink_dense(Xd, cpa.soft(tau), opts)
    Y2 = cpa.shrink_dense_noalloc(Xd, cpa.soft(tau), opts, torch.empty_like(Xd))
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)


def test_given_coefficients_argument_checks():
    import torch
    import paper_1705_07112_amd as cpa
    print("case coefficient argument checks", flush=True)
    X = torch.randn(64, 48, device="cuda")
    c = torch.zeros(8, dtype=torch.float64, device="cuda")
    sh = cpa.soft(0.1)
    with pytest.raises(cpa.CpaError) as e:          # the coefficients belong to one Lambda
        cpa.shrink_dense(X, sh, cpa.Opts(K=8, bound="power", coeffs=c))
    assert e.value.status == cpa.ERR_ARG
    for kw in ({"check": True}, {"damping": "jackson"}):
        with pytest.raises(cpa.CpaError) as e:
            cpa.shrink_dense(X, sh, cpa.Opts(K=8, Lambda=300.0, coeffs=c, **kw))
        assert e.value.status == cpa.ERR_UNSUPPORTED
    with pytest.raises(cpa.CpaError) as e:          # the FP64 path computes its own
        cpa.shrink_dense(X.double(), sh, cpa.Opts(K=8, Lambda=300.0, coeffs=c))
    assert e.value.status == cpa.ERR_UNSUPPORTED
    with pytest.raises(cpa.CpaError) as e:          # and so do the drivers
        cpa.rpca_admm(X, 0.1, 1.0, 2, 1e-7, cpa.Opts(K=8, Lambda=300.0, coeffs=c))
    assert e.value.status == cpa.ERR_UNSUPPORTED
    with pytest.raises(ValueError):                 # K entries of float64 on the device
        cpa.Opts(K=9, Lambda=300.0, coeffs=c).to_c()
    with pytest.raises(ValueError):
        cpa.Opts(K=8, Lambda=300.0, coeffs=c.float()).to_c()
    # the given coefficients are what is evaluated: zeros give Y = 0, c_0 = 2 gives Y = X
    Y = cpa.shrink_dense(X, sh, cpa.Opts(K=8, Lambda=300.0, coeffs=c))
    assert float(Y.abs().max()) == 0.0
    c[0] = 2.0
    Y = cpa.shrink_dense(X, sh, cpa.Opts(K=8, Lambda=300.0, coeffs=c))
    torch.cuda.synchronize()
    assert torch.allclose(Y, X, rtol=0, atol=1e-6)
