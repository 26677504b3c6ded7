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
the previous iteration's vector, or (bound_rule="lanczos") the k-step Lanczos
bound of oracle/bound.py warm-started from the previous Ritz vector.

SVT matrix completion (Cai, Candes, Shen 2010; the paper cites completion but
gives no algorithm): X^t = shrink_tau(Y^{t-1}); Y^t = Y^{t-1} + delta P_Omega(M - X^t),
Y^0 = k0 delta P_Omega(M).

Texture inpainting (Sec. V-C, eq. texture_repaire4; Appendix A, eqs. texture_repaire5,
z_insert, admm_eq, admm_algorithm_inp): ADMM on z = K l with
K = [Id; Psi; Omega; Id; Omega_bar], Psi the orthonormal 2-D DCT of the m x n image
(Psi l = vec(D_m L D_n^T)), Omega the observed-pixel mask and Omega_bar its complement:
  l = (K^T K)^{-1} K^T (z - u)              K^T K = 4 Id (Psi orthogonal, Omega + Omega_bar = Id)
  z1 = prox_{(1/rho)||.||_*}(l + u1)        CPA singular value soft shrinkage
  z2 = soft(Psi l + u2, eta/rho)
  z3 = Pi_I(Omega l + u3) = Omega i         the observed pixels
  z4 = Pi_D(l + u4) = clip to [0, 1]
  z5 = Pi_M(Omega_bar l + u5)               the recovered region shifted to the mean of the
                                            surrounding observed pixels m_del
  u += K l - z;   E_t = ||l_{t+1} - l_t|| / ||l_{t+1}||.
Readings: the start is l_0 = u_0 = 1 (Sec. V-C) and z_0 = K l_0 (unstated); the recovered
region is the unobserved set (Omega_bar) and the surrounding pixels m_del are a mask the
caller gives; Pi_M adds (mean of I over m_del) - (mean of y over the region) to y on the
region and leaves y elsewhere; without the mean term (the random-corruption experiment of
Sec. V-F) z5 and u5 are dropped and K^T K = 3 Id + Omega.

With the sparsifying transform (Sec. III-B and the experiments of Table IV), z1 is
the sparsified shrink of oracle.sparsify with K(|Phi|, k) and k from the previous
iteration's E_t by eq. (recommendation_epsilon) (oracle.sparsify.keep_schedule).

Pins: (K^T K)^{-1} K^T checked by substitution; l1 prox against its closed
form; with the exact nuclear-norm prox in place of the CPA shrink the RPCA
iteration reaches a point meeting principal component pursuit's optimality
conditions (L + S = I, u1 = u2 = -u3, rho u1 and rho u2 subgradients of the
two norms) and recovers the planted parts of an exactly recoverable input, and
with the CPA shrink at a high order it recovers them to that order's accuracy;
SVT: k0 against inputs whose ||P_Omega M||_2 is known in closed form and the
defining inequality (k0 - 1) delta ||P_Omega M||_2 < tau <= k0 delta ||P_Omega M||_2,
recovery of an exactly recoverable rank-2 matrix (to rounding with the exact
prox, to the order's accuracy with CPA).  Planted slips (z1 from l, u3 without
-I, l and s swapped, the l1 threshold, k0 rounded down, the step's sign) each
fail a pin.  Parity: pinned; the ADMM hyper-parameters are project choices
(parity does not depend on them, both sides take the same values).
"""
from __future__ import annotations

import math

import numpy as np

from . import bound, cpa
from .shrinkage import soft
from .sparsify import (cpa_shrink_sparsified, dct_matrix, keep_schedule, kth_largest_abs, transformed_gram,
                       truncate)


def soft_elementwise(x, t):
    """prox of t||.||_1: sgn(x) max(|x| - t, 0)."""
    x = np.asarray(x, dtype=np.float64)
    return np.sign(x) * np.maximum(np.abs(x) - t, 0.0)


def admm_lsolve(z1, z2, z3, u1, u2, u3):
    """(K^T K)^{-1} K^T (z - u) for K = [[I,0],[0,I],[I,I]]."""
    a = (z1 - u1) + (z3 - u3)
    b = (z2 - u2) + (z3 - u3)
    return (2.0 * a - b) / 3.0, (2.0 * b - a) / 3.0


def _bound(Phi, rule, seed, power_iters, tol_power, delta, v0, lanczos_steps):
    """(Lambda, the next warm-start vector) by the power iteration or by the
    k-step Lanczos rule (oracle/bound.py), both from the same start."""
    if rule == "lanczos":
        r = bound.lanczos_bound(Phi, seed=seed, steps=lanczos_steps, delta=delta, v0=v0, tol=tol_power)
        return r[0], r[4]
    r = bound.power_bound(Phi, seed=seed, max_iter=power_iters, tol=tol_power, delta=delta, v0=v0)
    return r[0], r[4]


def rpca_step(state, I, inv_rho: float, eta_over_rho: float, K: int, v=None, seed: int = 0,
              power_iters: int = 100, tol_power: float = 1e-7, delta: float = 0.01, bound_rule: str = "power",
              lanczos_steps: int = 12):
    """One ADMM iteration from ``state`` = dict(l, s, z1, z2, u1, u2, u3) (z3 = I).
    Returns (new_state, info) with info = dict(x, Lambda, v, E)."""
    I = np.asarray(I, dtype=np.float64)
    l_new, s_new = admm_lsolve(state["z1"], state["z2"], I, state["u1"], state["u2"], state["u3"])
    x = l_new + state["u1"]
    Phi, _ = cpa.gram(x)
    Lam, v = _bound(Phi, bound_rule, seed, power_iters, tol_power, delta, v, lanczos_steps)
    z1 = cpa.cpa_shrink(x, soft(inv_rho), Lam, K)
    z2 = soft_elementwise(s_new + state["u2"], eta_over_rho)
    new = {
        "l": l_new, "s": s_new, "z1": z1, "z2": z2,
        "u1": state["u1"] + l_new - z1,
        "u2": state["u2"] + s_new - z2,
        "u3": state["u3"] + l_new + s_new - I,
    }
    num = math.sqrt(float(np.sum((l_new - state["l"]) ** 2)))
    den = math.sqrt(float(np.sum(l_new ** 2)))
    return new, {"x": x, "Lambda": Lam, "v": v, "E": (num / den if den > 0 else 0.0)}


def rpca_start(I):
    """l_0 = s_0 = u_0 = 1, z_0 = [l_0; s_0; I] (z3 = I is implicit)."""
    ones = np.ones(np.shape(I))
    return {k: ones.copy() for k in ("l", "s", "z1", "z2", "u1", "u2", "u3")}


def rpca_admm(I, inv_rho: float, eta_over_rho: float, iters: int, K: int,
              seed: int = 0, power_iters: int = 100, tol_power: float = 1e-7, delta: float = 0.01):
    """Runs ``iters`` ADMM iterations from the start state; returns
    (l, s, E_hist, Lambda_hist).  The power-iteration bound of each shrink is
    warm-started from the previous iteration's vector."""
    state = rpca_start(I)
    v = None
    E, lams = [], []
    for _ in range(iters):
        state, info = rpca_step(state, I, inv_rho, eta_over_rho, K, v=v, seed=seed,
                                power_iters=power_iters, tol_power=tol_power, delta=delta)
        v = info["v"]
        E.append(info["E"])
        lams.append(info["Lambda"])
    return state["l"], state["s"], E, lams


def svt_complete(m, n, rows, cols, vals, tau: float, step: float, iters: int, K: int,
                 seed: int = 0, power_iters: int = 100, tol_power: float = 1e-7, delta_bound: float = 0.01):
    """SVT completion with CPA shrinkage on the dense iterate (small sizes only).

    k0 = ceil(tau / (step ||P_Omega M||_2)) with the norm from a converged power
    iteration (200 products, tol 1e-9); Y^0 = k0 step P_Omega(M).  Each shrink's
    bound is a power bound capped by tr(Y^T Y) = ||Y||_F^2 (the operator-form cap),
    warm-started from the previous vector (the first from the k0 iteration).
    Returns (X, residual history, k0)."""
    vals = np.asarray(vals, dtype=np.float64)
    P = np.zeros((m, n))
    P[rows, cols] = vals
    G0 = P.T @ P if m >= n else P @ P.T
    _, mu0, _, _, v = bound.power_bound(G0, seed=seed, max_iter=200, tol=1e-9, delta=delta_bound,
                                        cap=float(np.trace(G0)))
    nrm2 = math.sqrt(max(mu0, 0.0))
    k0 = math.ceil(tau / (step * nrm2)) if nrm2 > 0 else 1
    Y = np.zeros((m, n))
    Y[rows, cols] = k0 * step * vals
    sh = soft(tau)
    X = np.zeros((m, n))
    res = []
    nrm = math.sqrt(float(vals @ vals))
    for _ in range(iters):
        Phi, _ = cpa.gram(Y)
        Lam, _, _, _, v = bound.power_bound(Phi, seed=seed, max_iter=power_iters, tol=tol_power,
                                            delta=delta_bound, v0=v, cap=float(np.trace(Phi)))
        X = cpa.cpa_shrink(Y, sh, Lam, K)
        r = vals - X[rows, cols]
        Y[rows, cols] += step * r
        res.append(math.sqrt(float(r @ r)) / nrm)
    return X, res, k0


def dct2(L, Dm=None, Dn=None):
    """Psi l as a matrix: D_m L D_n^T with the orthonormal DCT-II matrices."""
    L = np.asarray(L, dtype=np.float64)
    m, n = L.shape
    Dm = dct_matrix(m) if Dm is None else Dm
    Dn = dct_matrix(n) if Dn is None else Dn
    return Dm @ L @ Dn.T


def idct2(S, Dm=None, Dn=None):
    """Psi^T s as a matrix: D_m^T S D_n."""
    S = np.asarray(S, dtype=np.float64)
    m, n = S.shape
    Dm = dct_matrix(m) if Dm is None else Dm
    Dn = dct_matrix(n) if Dn is None else Dn
    return Dm.T @ S @ Dn


INPAINT_NAMES = ("l", "z1", "z2", "z3", "z4", "z5", "u1", "u2", "u3", "u4", "u5")


def inpaint_start(omega):
    """l_0 = u_0 = 1 and z_0 = K l_0 (with the mean term; z5, u5 unused without it)."""
    om = np.asarray(omega, dtype=np.float64)
    ones = np.ones(om.shape)
    st = {k: ones.copy() for k in INPAINT_NAMES}
    st["z2"] = dct2(ones)
    st["z3"] = om * ones
    st["z5"] = (1.0 - om) * ones
    return st


def inpaint_step(state, I, omega, border, inv_rho: float, eta_over_rho: float, K: int, v=None, seed: int = 0,
                 power_iters: int = 100, tol_power: float = 1e-7, delta: float = 0.01, sparsify=None,
                 bound_rule: str = "power", lanczos_steps: int = 12):
    """One ADMM iteration of eq. (admm_algorithm_inp).  omega: observed mask (1/0);
    border: mask of the surrounding pixels m_del, or None for no mean term.
    sparsify: None for the plain shrink, or dict(T, zero, keep): z1 by the
    sparsified shrink of Sec. III-B (transform T, the high-frequency mask zero or
    None, threshold K(|Phi|, keep)), its bound the power bound of the truncated
    matrix from a cold start.
    Returns (new_state, info) with info = dict(x, Lambda, v, E)."""
    I = np.asarray(I, dtype=np.float64)
    om = np.asarray(omega, dtype=np.float64)
    ob = 1.0 - om
    ave = border is not None
    st = state
    r = (st["z1"] - st["u1"]) + idct2(st["z2"] - st["u2"]) + om * (st["z3"] - st["u3"]) + (st["z4"] - st["u4"])
    if ave:
        r = r + ob * (st["z5"] - st["u5"])
    diag = 3.0 + om + (ob if ave else 0.0)
    l_new = r / diag
    x = l_new + st["u1"]
    if sparsify is None:
        Phi, _ = cpa.gram(x)
        Lam, v = _bound(Phi, bound_rule, seed, power_iters, tol_power, delta, v, lanczos_steps)
        z1 = cpa.cpa_shrink(x, soft(inv_rho), Lam, K)
    else:
        T, zero, keep = sparsify["T"], sparsify.get("zero"), sparsify["keep"]
        Phi, _ = transformed_gram(x, T)
        if zero is not None:
            Phi[zero, :] = 0.0
            Phi[:, zero] = 0.0
        Phil = truncate(Phi, kth_largest_abs(Phi, keep))
        Lam, _, _, _, v = bound.power_bound(Phil, seed=seed, max_iter=power_iters, tol=tol_power, delta=delta)
        z1 = cpa_shrink_sparsified(x, soft(inv_rho), Lam, K, T, keep, zero=zero)[0]
    P = dct2(l_new)
    z2 = soft_elementwise(P + st["u2"], eta_over_rho)
    z3 = om * I
    z4 = np.clip(l_new + st["u4"], 0.0, 1.0)
    new = {"l": l_new, "z1": z1, "z2": z2, "z3": z3, "z4": z4,
           "u1": st["u1"] + l_new - z1, "u2": st["u2"] + P - z2, "u3": st["u3"] + om * l_new - z3,
           "u4": st["u4"] + l_new - z4}
    if ave:
        bd = np.asarray(border, dtype=bool)
        reg = om == 0.0
        y = ob * l_new + st["u5"]
        z5 = y.copy()
        z5[reg] += float(np.mean(I[bd])) - float(np.mean(y[reg]))
        new["z5"] = z5
        new["u5"] = st["u5"] + ob * l_new - z5
    else:
        new["z5"] = st["z5"]
        new["u5"] = st["u5"]
    num = math.sqrt(float(np.sum((l_new - st["l"]) ** 2)))
    den = math.sqrt(float(np.sum(l_new ** 2)))
    return new, {"x": x, "Lambda": Lam, "v": v, "E": (num / den if den > 0 else 0.0)}


def inpaint_admm(I, omega, border, inv_rho: float, eta_over_rho: float, iters: int, K: int, seed: int = 0,
                 power_iters: int = 100, tol_power: float = 1e-7, delta: float = 0.01, schedule=None, state=None):
    """``iters`` iterations of eq. (admm_algorithm_inp) from inpaint_start (or from
    ``state``); returns (l, E_hist), or (state, E_hist, keeps) with a schedule.
    The power bound of each plain shrink is warm-started.
    schedule: None, or dict(T, zero, E_l, E_m, E_prev): z1 by the sparsified shrink
    with keep = keep_schedule(E, d) of the previous iteration's E (E_prev before
    the first), d the side of the Gram (eq. recommendation_epsilon)."""
    state = inpaint_start(omega) if state is None else state
    v = None
    E = []
    keeps = []
    for _ in range(iters):
        sp = None
        if schedule is not None:
            d = min(np.shape(I))
            e_prev = E[-1] if E else schedule.get("E_prev", math.inf)
            sp = {"T": schedule["T"], "zero": schedule.get("zero"),
                  "keep": keep_schedule(e_prev, d, schedule.get("E_l", 0.03), schedule.get("E_m", 6e-4))}
            keeps.append(sp["keep"])
        state, info = inpaint_step(state, I, omega, border, inv_rho, eta_over_rho, K, v=v, seed=seed,
                                   power_iters=power_iters, tol_power=tol_power, delta=delta, sparsify=sp)
        v = info["v"]
        E.append(info["E"])
    if schedule is not None:
        return state, E, keeps
    return state["l"], E
