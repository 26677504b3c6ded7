"""Spectral bound Lambda >= lambda_max(Phi) (oracle; test infrastructure only).

Paper passage: Algorithm 1 (Sec. III-B), the step that computes the maximum
eigenvalue Lambda_max of the (truncated) Gram, which is also the scale of
hat B = (2/Lambda_max) Phi - Id.  The paper does not say how it is computed.

Reading (documented as a project choice):
  * power iteration on Phi from a start vector drawn by SplitMix64 (Steele,
    Lea, Flood, OOPSLA 2014) used as a counter-based generator: entry i is the
    SplitMix64 output for state seed + (i+1) * 0x9E3779B97F4A7C15, mapped to
    2u - 1 with u = (out >> 11) * 2^-53;
  * v <- v / ||v||; repeat: w = Phi v, mu = v.w, stop once
    |mu_t - mu_{t-1}| <= tol * mu_t (t >= 2) or after max_iter products;
    otherwise v <- w / ||w||;
  * residual norm ||r|| = sqrt(max(||w||^2 - mu^2, 0)) for the last (v, w, mu);
  * Lambda = min(mu + max(delta * mu, ||r||), (1 + delta) ||Phi||_F).
    ||Phi||_F >= lambda_max for a PSD matrix, so the cap never cuts below the
    largest eigenvalue, and it keeps the relative margin: a bound equal to
    lambda_max would put the top eigenvalue on the endpoint of [-1, 1], where
    T_k has slope k^2 and rounding is amplified about K^2-fold;
  * ||Phi||_F == 0 gives Lambda = 0; a vanishing product (w == 0 while
    ||Phi||_F > 0) gives Lambda = ||Phi||_F.

For a sparse S the operator form caps with tr(Phi) = ||S||_F^2 instead of
||Phi||_F (both bound lambda_max of a PSD matrix).

k-step Lanczos (a second reading of the same step; the paper names no method):
  * q_1 = v_0 / ||v_0|| (the same start vector), beta_0 = 0; for j = 1..k:
    u = Phi q_j - beta_{j-1} q_{j-1}, alpha_j = q_j.u, u <- u - alpha_j q_j,
    beta_j = ||u||, q_{j+1} = u / beta_j (plain three-term recurrence, no
    reorthogonalisation; an exactly vanishing beta_j ends the run at step j,
    and with tol > 0 so does the first step j >= 2 whose Ritz value theta_j,
    the largest eigenvalue of T_j, satisfies |theta_j - theta_{j-1}| <= tol theta_j,
    the power iteration's test with the Ritz values in place of the quotients);
  * T_k = tridiagonal (alpha on the diagonal, beta_1..beta_{k-1} beside it),
    theta = its largest eigenvalue, s its unit eigenvector, Ritz vector
    y = sum_i s_i q_i, residual norm ||Phi y - theta y|| = beta_k |s_k|;
  * Lambda = min(theta + max(delta * theta, ||r||), (1 + delta) ||Phi||_F), the
    rule of the power iteration with (theta, ||r||) in place of (mu, ||r||);
    k = min(steps, d).  theta never exceeds lambda_max (interlacing), and one
    step is one power product: theta_1 = mu_1, ||r||_1 = the power residual.

Pins: the bound is >= the true largest eigenvalue (from eigh) on seeded
matrices; on diagonal matrices it converges to the known maximum; the start
vector reproduces SplitMix64's published first outputs for seed 0.  Lanczos:
on the [-1, 2, -1] Toeplitz matrix from e_1 the recurrence returns the matrix's
own leading block, so theta and ||r|| have closed forms; with as many steps as
distinct eigenvalues it finds the largest one exactly; one step equals one
power product; the Ritz pair's residual equals beta_k |s_k|; theta <= lambda_max.
Parity: pinned (the margin delta is a project choice, stated above).
"""
from __future__ import annotations

import math

import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(state: int) -> int:
    """Output function of SplitMix64 applied to a 64-bit state."""
    z = state & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def start_vector(d: int, seed: int) -> np.ndarray:
    v = np.empty(d)
    for i in range(d):
        out = splitmix64((seed + (i + 1) * _GAMMA) & _MASK)
        u = (out >> 11) * (1.0 / 9007199254740992.0)
        v[i] = 2.0 * u - 1.0
    return v


def power_bound(Phi: np.ndarray, seed: int = 0, max_iter: int = 100, tol: float = 1e-7,
                delta: float = 0.01, v0=None, cap=None):
    """Returns (Lambda, mu, resid, iters, v_last).

    ``cap`` replaces ||Phi||_F as the guaranteed upper bound when given (the
    operator form knows only tr(Phi) = ||S||_F^2, which is also >= lambda_max)."""
    Phi = np.asarray(Phi, dtype=np.float64)
    d = Phi.shape[0]
    fro = math.sqrt(float(np.sum(Phi * Phi))) if cap is None else float(cap)
    if d == 0 or fro == 0.0:
        return 0.0, 0.0, 0.0, 0, np.zeros(d)
    v = start_vector(d, seed) if v0 is None else np.asarray(v0, dtype=np.float64).copy()
    nv = math.sqrt(float(v @ v))
    if nv == 0.0:
        return fro, 0.0, 0.0, 0, v
    v = v / nv
    mu_prev = None
    mu = 0.0
    wn2 = 0.0
    it = 0
    for it in range(1, max_iter + 1):
        w = Phi @ v
        mu = float(v @ w)
        wn2 = float(w @ w)
        if wn2 == 0.0:
            return fro, 0.0, 0.0, it, v
        if mu_prev is not None and abs(mu - mu_prev) <= tol * mu:
            break
        mu_prev = mu
        if it < max_iter:
            v = w / math.sqrt(wn2)
    resid = math.sqrt(max(wn2 - mu * mu, 0.0))
    Lam = min(mu + max(delta * mu, resid), (1.0 + delta) * fro)
    return Lam, mu, resid, it, v


def lanczos_bound(Phi: np.ndarray, seed: int = 0, steps: int = 12, delta: float = 0.01, v0=None, cap=None,
                  tol: float = 0.0):
    """Returns (Lambda, theta, resid, steps_done, y, alpha, beta)."""
    Phi = np.asarray(Phi, dtype=np.float64)
    d = Phi.shape[0]
    fro = math.sqrt(float(np.sum(Phi * Phi))) if cap is None else float(cap)
    if d == 0 or fro == 0.0:
        return 0.0, 0.0, 0.0, 0, np.zeros(d), np.zeros(0), np.zeros(0)
    v = start_vector(d, seed) if v0 is None else np.asarray(v0, dtype=np.float64).copy()
    nv = math.sqrt(float(v @ v))
    if nv == 0.0:
        return fro, 0.0, 0.0, 0, v, np.zeros(0), np.zeros(0)
    k = min(int(steps), d)
    Q = np.zeros((k, d))
    alpha, beta = [], []
    q, q_prev, b_prev = v / nv, np.zeros(d), 0.0
    th_prev = None
    for j in range(k):
        Q[j] = q
        u = Phi @ q - b_prev * q_prev
        a = float(q @ u)
        u = u - a * q
        b = math.sqrt(float(u @ u))
        alpha.append(a)
        beta.append(b)
        if b == 0.0:
            break
        if tol > 0.0:
            m = len(alpha)
            Tj = np.diag(alpha) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
            th = float(np.linalg.eigvalsh(Tj)[-1])
            if th_prev is not None and abs(th - th_prev) <= tol * th:
                break
            th_prev = th
        q_prev, q, b_prev = q, u / b, b
    m = len(alpha)
    if m == 1 and alpha[0] == 0.0 and beta[0] == 0.0:
        return fro, 0.0, 0.0, 1, Q[0], np.array(alpha), np.array(beta)   # the product vanished
    T = np.diag(alpha) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
    ev, S = np.linalg.eigh(T)
    theta, s = float(ev[-1]), S[:, -1]
    resid = beta[m - 1] * abs(float(s[m - 1]))
    y = s @ Q[:m]
    Lam = min(theta + max(delta * theta, resid), (1.0 + delta) * fro)
    return Lam, theta, resid, m, y, np.array(alpha), np.array(beta)
