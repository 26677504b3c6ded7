"""Pins for the driver oracles (RPCA ADMM of Appendix B, SVT completion), each
against what the optimisation problem fixes, not against the oracle's own
algebra:

* RPCA (principal component pursuit, min ||L||_* + eta ||S||_1 s.t. L + S = I):
  with the exact nuclear-norm prox substituted for the CPA shrink, the ADMM
  fixed point must satisfy the problem's optimality conditions -- primal
  feasibility L + S = I, the x-update's stationarity K^T u = 0 (u1 = u2 = -u3),
  rho u1 a subgradient of ||.||_* at L (U^T W V = I on the range, spectral norm
  of the rest below 1) and rho u2 a subgradient of eta ||.||_1 at S -- and
  recover the planted low-rank and sparse parts of an exactly recoverable
  instance; with the CPA shrink at a high order it recovers them to the order's
  accuracy.
* SVT (Cai, Candes, Shen): k0 is the smallest integer with k0 delta ||P_Omega M||_2
  >= tau, checked on an input whose spectral norm is known in closed form
  (observed entries on a diagonal); with the exact prox the iteration recovers an
  exactly recoverable rank-2 matrix to rounding, and with the CPA shrink to the
  order's accuracy.
"""
import math

import numpy as np
import pytest

import synth
from oracle import cpa, drivers, exact


def _exact_prox(B, shrink, Lambda, K, damping="none"):
    """The definition of the nuclear-norm prox (SVD), in place of the CPA shrink."""
    return exact.svt_svd(B, shrink)


def _rpca_instance():
    I, L0, S0 = synth.rpca_frames(64, 64, rank=2, outlier_frac=0.01, seed=11)
    return I.astype(np.float64), L0.astype(np.float64), S0.astype(np.float64)


def _rpca_run(I, inv_rho, eta_over_rho, iters, K):
    state = drivers.rpca_start(I)
    v = None
    for _ in range(iters):
        state, info = drivers.rpca_step(state, I, inv_rho, eta_over_rho, K, v=v)
        v = info["v"]
    return state


def test_rpca_exact_prox_meets_pcp_optimality(monkeypatch):
    monkeypatch.setattr(cpa, "cpa_shrink", _exact_prox)
    I, L0, S0 = _rpca_instance()
    inv_rho, eta = 1.0, 1.0 / 8.0
    st = _rpca_run(I, inv_rho, eta * inv_rho, 400, 30)
    rho = 1.0 / inv_rho
    L, S = st["z1"], st["z2"]
    nI = np.linalg.norm(I)
    # primal feasibility and agreement of the x-update with z
    assert np.linalg.norm(L + S - I) / nI <= 1e-5
    assert np.linalg.norm(st["l"] - L) / nI <= 1e-5
    assert np.linalg.norm(st["s"] - S) / nI <= 1e-5
    # stationarity of the least-squares step: K^T u = (u1 + u3, u2 + u3) = 0
    assert np.max(np.abs(st["u1"] + st["u3"])) <= 1e-6
    assert np.max(np.abs(st["u2"] + st["u3"])) <= 1e-6
    # rho u1 in the nuclear norm's subdifferential at L
    W = rho * st["u1"]
    U, sv, Vt = np.linalg.svd(L)
    r = int(np.sum(sv > 1e-8 * sv[0]))
    Ur, Vr = U[:, :r], Vt[:r].T
    assert np.max(np.abs(Ur.T @ W @ Vr - np.eye(r))) <= 1e-6
    Wperp = (np.eye(64) - Ur @ Ur.T) @ W @ (np.eye(64) - Vr @ Vr.T)
    assert np.linalg.norm(Wperp, 2) < 1.0
    # rho u2 in eta times the l1 norm's subdifferential at S
    W2 = rho * st["u2"]
    supp = S != 0
    assert np.max(np.abs(W2[supp] - eta * np.sign(S[supp]))) <= 1e-6
    assert np.max(np.abs(W2[~supp])) < eta
    # the planted parts are recovered (the instance is exactly recoverable)
    assert np.array_equal(supp, S0 != 0)
    assert np.linalg.norm(L - L0) / np.linalg.norm(L0) <= 1e-5
    assert np.linalg.norm(S - S0) / np.linalg.norm(S0) <= 1e-4


def test_rpca_cpa_recovers_planted_parts():
    I, L0, S0 = _rpca_instance()
    l, s, E, lams = drivers.rpca_admm(I, inv_rho=1.0, eta_over_rho=1.0 / 8.0, iters=200, K=60)
    assert np.linalg.norm(l + s - I) / np.linalg.norm(I) <= 5e-4
    assert np.linalg.norm(l - L0) / np.linalg.norm(L0) <= 2e-3
    assert np.linalg.norm(s - S0) / np.linalg.norm(S0) <= 1e-2
    assert E[-1] <= 1e-4


def test_svt_k0_closed_form():
    """Observed entries on the diagonal: ||P_Omega M||_2 is the largest |entry|."""
    m, n = 6, 4
    d = np.array([3.0, -2.0, 1.0, 0.5])
    rows = np.arange(4)
    cols = np.arange(4)
    # tau / (delta * 3) = 10 / 3.6 = 2.78 -> k0 = 3
    _, _, k0 = drivers.svt_complete(m, n, rows, cols, d, tau=10.0, step=1.2, iters=1, K=5)
    assert k0 == 3
    # tau / (delta * 3) = 6.3 / 2.1 = 3.0000000001 -> 4 (just above an integer)
    _, _, k0 = drivers.svt_complete(m, n, rows, cols, d, tau=6.3 + 3e-10, step=0.7, iters=1, K=5)
    assert k0 == 4
    # tau / (delta * 3) = 0.05 -> 1
    _, _, k0 = drivers.svt_complete(m, n, rows, cols, d, tau=0.15, step=1.0, iters=1, K=5)
    assert k0 == 1


def _svt_instance():
    g = synth.rng(40)
    m, n, r = 60, 30, 2
    M = g.standard_normal((m, r)) @ g.standard_normal((r, n))
    idx = np.sort(g.choice(m * n, size=900, replace=False))
    rows, cols = idx // n, idx % n
    return m, n, M, rows, cols, 5 * math.sqrt(m * n), 1.2 * m * n / len(idx)


def test_svt_k0_defining_inequality():
    m, n, M, rows, cols, tau, step = _svt_instance()
    P = np.zeros((m, n))
    P[rows, cols] = M[rows, cols]
    s1 = np.linalg.norm(P, 2)
    _, _, k0 = drivers.svt_complete(m, n, rows, cols, M[rows, cols], tau, step, 1, 5)
    assert (k0 - 1) * step * s1 < tau <= k0 * step * s1


def test_svt_exact_prox_recovers(monkeypatch):
    monkeypatch.setattr(cpa, "cpa_shrink", _exact_prox)
    m, n, M, rows, cols, tau, step = _svt_instance()
    X, res, _ = drivers.svt_complete(m, n, rows, cols, M[rows, cols], tau, step, 600, 25)
    assert res[-1] <= 1e-9
    assert np.linalg.norm(X - M) / np.linalg.norm(M) <= 1e-8
    assert res[-1] < res[100] < res[0]


def test_svt_cpa_recovers():
    m, n, M, rows, cols, tau, step = _svt_instance()
    X, res, _ = drivers.svt_complete(m, n, rows, cols, M[rows, cols], tau, step, 300, 25)
    assert np.linalg.norm(X - M) / np.linalg.norm(M) <= 1e-2
    assert res[-1] <= 2e-3
