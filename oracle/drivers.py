"""Iteration drivers around the shrinkage (oracle; test infrastructure only).

RPCA background modelling by ADMM, Appendix B, eq. (admm_algorithm_mod), for
min ||L||_* + eta ||S||_1 s.t. I = L + S with z = K [l; s],
K = [[Id, O], [O, Id], [Id, Id]]:
  l' = (K^T K)^{-1} K^T (z - u):   with a = (z1-u1) + (z3-u3), b = (z2-u2) + (z3-u3),
                                   (K^T K)^{-1} = (1/3) [[2, -1], [-1, 2]] gives
                                   l = (2a - b)/3, s = (2b - a)/3
  z1 = prox_{(1/rho)||.||_*}(l + u1)   singular value soft shrinkage, tau = 1/rho,
                                       by CPA (Sec. V-B.1: the nuclear-norm prox is
                                       singular value shrinkage)
  z2 = prox_{(eta/rho)||.||_1}(s + u2) = sgn(x) max(|x| - eta/rho, 0)
  z3 = Pi_I(l + s + u3) = I            (every pixel observed)
  u  = u + K l' - z
  E_t = ||l_{t+1} - l_t||_2 / ||l_{t+1}||_2   (stopping quantity, Sec. V-B.2)
Initialisation: l_0 = s_0 = u_0 = all ones (Sec. V-D).  The paper leaves z_0
unstated; the reading here is z_0 = [l_0; s_0; I]: the first two blocks equal
K [l_0; s_0], and the third block is the projection onto the observed data,
which is I at every iteration, so it starts at I as well.
The spectral bound of each shrink is a power-iteration bound warm-started from
the previous iteration's vector.

SVT matrix completion (Cai, Candes, Shen 2010; the paper cites completion but
gives no algorithm): X^t = shrink_tau(Y^{t-1}); Y^t = Y^{t-1} + delta P_Omega(M - X^t),
Y^0 = k0 delta P_Omega(M).

Pins: (K^T K)^{-1} K^T checked by substitution; l1 prox against its closed
form; E_t falls on a low-rank-plus-sparse input.  Parity: pinned for the
closed-form pieces; the ADMM hyper-parameters are project choices (parity
does not depend on them, both sides take the same values).
"""
from __future__ import annotations

import math

import numpy as np

from . import bound, cpa
from .shrinkage import soft


def soft_elementwise(x, t):
    """prox of t||.||_1: sgn(x) max(|x| - t, 0)."""
    x = np.asarray(x, dtype=np.float64)
    return np.sign(x) * np.maximum(np.abs(x) - t, 0.0)


def admm_lsolve(z1, z2, z3, u1, u2, u3):
    """(K^T K)^{-1} K^T (z - u) for K = [[I,0],[0,I],[I,I]]."""
    a = (z1 - u1) + (z3 - u3)
    b = (z2 - u2) + (z3 - u3)
    return (2.0 * a - b) / 3.0, (2.0 * b - a) / 3.0


def rpca_admm(I, inv_rho: float, eta_over_rho: float, iters: int, K: int,
              seed: int = 0, power_iters: int = 100, warm_power_iters: int = 100,
              tol_power: float = 1e-7, delta: float = 0.01, record=None):
    """Runs ``iters`` ADMM iterations; returns (l, s, E_hist, Lambda_hist).

    ``record`` (optional list) receives (t, shrink_input, Lambda) per iteration
    so tests can check single shrinks on identical inputs."""
    I = np.asarray(I, dtype=np.float64)
    ones = np.ones_like(I)
    l, s = ones.copy(), ones.copy()
    u1, u2, u3 = ones.copy(), ones.copy(), ones.copy()
    z1, z2, z3 = l.copy(), s.copy(), I
    v = None
    E = []
    lams = []
    sh = soft(inv_rho)
    for t in range(iters):
        l_new, s_new = admm_lsolve(z1, z2, z3, u1, u2, u3)
        x = l_new + u1
        Phi, _ = cpa.gram(x)
        Lam, _, _, _, v = bound.power_bound(
            Phi, seed=seed, max_iter=(power_iters if v is None else warm_power_iters),
            tol=tol_power, delta=delta, v0=v)
        if record is not None:
            record.append((t, x.copy(), Lam))
        z1 = cpa.cpa_shrink(x, sh, Lam, K)
        z2 = soft_elementwise(s_new + u2, eta_over_rho)
        z3 = I
        u1 = u1 + l_new - z1
        u2 = u2 + s_new - z2
        u3 = u3 + l_new + s_new - z3
        num = math.sqrt(float(np.sum((l_new - l) ** 2)))
        den = math.sqrt(float(np.sum(l_new ** 2)))
        E.append(num / den if den > 0 else 0.0)
        lams.append(Lam)
        l, s = l_new, s_new
    return l, s, E, lams


def svt_complete(m, n, rows, cols, vals, tau: float, step: float, iters: int, K: int,
                 k0: int = 1, seed: int = 0, power_iters: int = 100):
    """SVT completion with CPA shrinkage on the dense iterate (small sizes only).
    Returns (X, residual history)."""
    Y = np.zeros((m, n))
    Y[rows, cols] = k0 * step * np.asarray(vals, dtype=np.float64)
    sh = soft(tau)
    X = np.zeros((m, n))
    res = []
    nrm = math.sqrt(float(np.sum(np.asarray(vals, dtype=np.float64) ** 2)))
    v = None
    for _ in range(iters):
        Phi, _ = cpa.gram(Y)
        Lam, _, _, _, v = bound.power_bound(Phi, seed=seed, max_iter=power_iters, v0=v)
        X = cpa.cpa_shrink(Y, sh, Lam, K)
        r = np.asarray(vals, dtype=np.float64) - X[rows, cols]
        Y[rows, cols] += step * r
        res.append(math.sqrt(float(r @ r)) / nrm)
    return X, res
