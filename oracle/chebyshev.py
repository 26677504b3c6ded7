"""Scalar Chebyshev machinery (oracle; test infrastructure only).

Paper passages:
  * truncated Chebyshev series, Sec. II-B, eq. (chebychev_series)
  * Chebyshev polynomial cos-form, Sec. II-B, eq. (chebychev_polynomial)
  * three-term recurrence, Sec. II-B, eq. (chebyche2)
  * discrete coefficients, Sec. II-B, eq. (chebychev_coeff_discrete)
  * shifted coefficients for [0, lambda_max], Sec. III-A, eq. (chebychev_coeff_shifted)

Reading of "order": the paper's alpha is the number of coefficients
c_0..c_{alpha-1} and also the number of nodes, so the polynomial degree is
alpha-1.  Here K == alpha.

Damping (not in the paper; an optional ripple reducer for steep responses such
as the high-order hard threshold): the series sum_k g_k c_k T_k with, for degree
N = K - 1,
  Jackson  g_k = ((N - k + 1) cos(pi k/(N+1)) + sin(pi k/(N+1)) cot(pi/(N+1))) / (N + 1)
  Lanczos  g_k = sin(pi k/(N+1)) / (pi k/(N+1)),  g_0 = 1
(Weisse, Wellein, Alvermann, Fehske, Rev. Mod. Phys. 78 (2006), Sec. II.C: the
kernel polynomial method's damping factors).  Pinned in tests/test_oracle_damping.py
(g_0 = 1, Jackson g_1 = cos(pi/K), the Jackson-damped step stays in [0, 1] while
the undamped one overshoots by more than 10%, Lanczos by less than 3%).

Pins (tests/test_oracle_pins.py): cos-form == recurrence (T_k(cos t) = cos kt);
coefficients exact for polynomial h of degree < K, aliasing of T_K to zero;
interpolation at the K nodes; discrete orthogonality.  Parity: pinned.
"""
from __future__ import annotations

import math

import numpy as np


def cheb_cos(k: int, x):
    """psi_k(x) = cos(k * arccos(x)) for x in [-1, 1] (eq. chebychev_polynomial)."""
    x = np.clip(np.asarray(x, dtype=np.float64), -1.0, 1.0)
    return np.cos(k * np.arccos(x))


def cheb_recurrence(k: int, x):
    """psi_k by psi_k = 2 x psi_{k-1} - psi_{k-2}, psi_0 = 1, psi_1 = x (eq. chebyche2)."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if k == 0:
        return p0
    p1 = x.copy()
    for _ in range(2, k + 1):
        p0, p1 = p1, 2.0 * x * p1 - p0
    return p1


def node_angles(K: int) -> np.ndarray:
    """theta(l) = pi (l - 1/2) / K for l = 1..K (after eq. chebychev_coeff_discrete)."""
    return np.array([math.pi * (l - 0.5) / K for l in range(1, K + 1)])


def coefficients_unit(h, K: int) -> np.ndarray:
    """c_k = (2/K) sum_{l=1..K} cos(k theta_l) h(cos theta_l), k = 0..K-1, for h on [-1,1]
    (eq. chebychev_coeff_discrete).  Sum over l in ascending order; cos evaluated directly."""
    th = node_angles(K)
    c = np.zeros(K)
    for k in range(K):
        s = 0.0
        for l in range(K):
            s += math.cos(k * th[l]) * float(h(math.cos(th[l])))
        c[k] = 2.0 / K * s
    return c


def coefficients_shifted(h, Lambda: float, K: int) -> np.ndarray:
    """hat c_k = (2/K) sum_l cos(k theta_l) h( Lambda/2 (cos theta_l + 1) ), k = 0..K-1
    (eq. chebychev_coeff_shifted; Algorithm 1, coefficient step).  h is defined on
    [0, Lambda]; the nodes map back from [-1, 1] to that interval."""
    th = node_angles(K)
    c = np.zeros(K)
    for k in range(K):
        s = 0.0
        for l in range(K):
            x = Lambda / 2.0 * (math.cos(th[l]) + 1.0)
            s += math.cos(k * th[l]) * float(h(x))
        c[k] = 2.0 / K * s
    return c


def series_unit(c, x):
    """hat h(x) = c_0/2 + sum_{k=1}^{K-1} c_k psi_k(x) on [-1,1] (eq. chebychev_series)."""
    x = np.asarray(x, dtype=np.float64)
    out = 0.5 * c[0] * np.ones_like(x)
    for k in range(1, len(c)):
        out = out + c[k] * cheb_cos(k, x)
    return out


def series_shifted(c, Lambda: float, x):
    """The interpolant as a function of the original variable x in [0, Lambda]:
    hat h(x) = c_0/2 + sum_k c_k psi_k(2x/Lambda - 1) (eqs. transform_lamB and
    chebychev_series_matrix_shift2, read on one eigenvalue)."""
    x = np.asarray(x, dtype=np.float64)
    return series_unit(c, 2.0 * x / Lambda - 1.0)


def damping_factors(K: int, kind: str = "none") -> np.ndarray:
    """g_0..g_{K-1} of the kind "none", "jackson" or "lanczos" (see the header)."""
    if kind == "none":
        return np.ones(K)
    N = K - 1
    g = np.ones(K)
    if N == 0:
        return g
    for k in range(1, K):
        a = math.pi * k / (N + 1)
        if kind == "jackson":
            g[k] = ((N - k + 1) * math.cos(a) + math.sin(a) / math.tan(math.pi / (N + 1))) / (N + 1)
        elif kind == "lanczos":
            g[k] = math.sin(a) / a
        else:
            raise ValueError("unknown damping")
    return g
