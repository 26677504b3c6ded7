"""Polynomial designs compared with CPA in Sec. IV-B (the comparison of Fig. 4;
eq. (l_p_norm_for_approximation)) -- oracle; test infrastructure only.

All designs return a polynomial of degree K - 1 on [0, Lambda] as coefficients in
the convention of the shrinkage, p(x) = c_0/2 + sum_{k>=1} c_k T_k(2x/Lambda - 1),
so that the same matrix evaluation applies to each of them.

* ``lsq_vandermonde``  the paper's least-squares coefficients c = Upsilon^+ h with
  the Vandermonde matrix of the monomials 1, u, ..., u^{K-1} at the sample points
  (the printed matrix lacks the column of first powers; read as a typesetting
  slip), in the variable u = x / Lambda, numpy's pseudo-inverse; converted to the
  Chebyshev convention.  Usable while the Vandermonde matrix is well conditioned
  (small K).
* ``lsq``  the same least-squares polynomial (the minimiser over polynomials of
  degree < K on the sample set is unique, whatever the basis) computed in the
  Chebyshev basis with numpy's least-squares solver: stable for every K.
* ``minimax``  the best uniform approximation on a grid by the Remez exchange:
  on a reference of K + 1 grid points solve p(x_j) + (-1)^j E = h(x_j), move the
  reference to the extrema of the error (one per maximal run of constant sign,
  trimmed to K + 1 alternating points), until the largest grid error exceeds |E|
  by at most a relative 1e-10 (plus 1e-14 of max |h|, the rounding of an exact fit).

Sample points of the least-squares fits: x_i = Lambda i / (n - 1), i = 0..n-1
(uniform; the paper does not fix them).  Remez grid: the n points
x_i = (Lambda / 2)(1 - cos(pi i / (n - 1))) (clustered at both ends, where the
Chebyshev polynomials vary fastest); initial reference: the grid points nearest to
the extrema (Lambda / 2)(1 - cos(pi j / K)), j = 0..K, of T_K.

Pins: exact reproduction of polynomial responses of degree < K by every design;
the best approximation of T_K by lower degrees is the zero polynomial with error
2^0 = 1 (Chebyshev's alternation theorem, for the monic form 2^{1-K} T_K);
equioscillation of the minimax error on its final reference; orthogonality of the
least-squares residual to every basis polynomial on the samples; the Vandermonde
and Chebyshev-basis least-squares polynomials agree where both are well
conditioned.  Parity: pinned.
"""
from __future__ import annotations

import numpy as np

from . import chebyshev


def _cheb_matrix(t, K):
    """V[i, k] = T_k(t_i), k = 0..K-1 (cos form on [-1, 1])."""
    t = np.clip(np.asarray(t, dtype=np.float64), -1.0, 1.0)
    th = np.arccos(t)
    return np.cos(np.outer(th, np.arange(K)))


def _to_convention(a):
    """Plain Chebyshev coefficients (p = sum a_k T_k) -> the c_0/2 convention."""
    c = np.array(a, dtype=np.float64)
    c[0] *= 2.0
    return c


def _hvals(h, x):
    return np.array([h(float(v)) for v in x])


def sample_points(Lambda: float, n: int) -> np.ndarray:
    return Lambda * np.arange(n) / (n - 1)


def remez_grid(Lambda: float, n: int) -> np.ndarray:
    return 0.5 * Lambda * (1.0 - np.cos(np.pi * np.arange(n) / (n - 1)))


def lsq_vandermonde(h, Lambda: float, K: int, n: int = 2000) -> np.ndarray:
    x = sample_points(Lambda, n)
    u = x / Lambda
    U = np.vander(u, K, increasing=True)           # 1, u, ..., u^{K-1}
    a = np.linalg.pinv(U) @ _hvals(h, x)           # monomial coefficients in u
    poly = lambda xx: float(np.polyval(a[::-1], xx / Lambda))
    return chebyshev.coefficients_shifted(poly, Lambda, K)   # exact for degree < K


def lsq(h, Lambda: float, K: int, n: int = 2000) -> np.ndarray:
    x = sample_points(Lambda, n)
    V = _cheb_matrix(2.0 * x / Lambda - 1.0, K)
    a, *_ = np.linalg.lstsq(V, _hvals(h, x), rcond=None)
    return _to_convention(a)


def minimax(h, Lambda: float, K: int, n: int = 8000, max_iter: int = 200, tol: float = 1e-10):
    """(coefficients, levelled error E, reference indices into the grid)."""
    x = remez_grid(Lambda, n)
    t = 2.0 * x / Lambda - 1.0
    hv = _hvals(h, x)
    hscale = max(1.0, float(np.max(np.abs(hv))))
    V = _cheb_matrix(t, K)
    target = 0.5 * Lambda * (1.0 - np.cos(np.pi * np.arange(K + 1) / K))
    ref = np.unique(np.abs(x[:, None] - target[None, :]).argmin(axis=0))
    if ref.size != K + 1:
        raise ValueError("grid too coarse for the reference")
    sign = (-1.0) ** np.arange(K + 1)
    a = np.zeros(K)
    E = 0.0
    for _ in range(max_iter):
        A = np.hstack([V[ref], sign[:, None]])
        sol = np.linalg.solve(A, hv[ref])
        a, E = sol[:K], sol[K]
        e = hv - V @ a
        emax = float(np.max(np.abs(e)))
        # converged: the grid error is levelled, or it is rounding of an exact fit
        if emax <= abs(E) * (1.0 + tol) + 1e-14 * hscale:
            break
        # one extremum per maximal run of constant sign
        s = np.sign(e)
        s[s == 0] = 1.0
        cand = []
        start = 0
        for i in range(1, n + 1):
            if i == n or s[i] != s[start]:
                seg = np.arange(start, i)
                cand.append(seg[np.argmax(np.abs(e[seg]))])
                start = i
        cand = list(cand)
        # trim to K + 1 alternating points, dropping the smaller end each time
        while len(cand) > K + 1:
            if abs(e[cand[0]]) < abs(e[cand[-1]]):
                cand.pop(0)
            else:
                cand.pop()
        if len(cand) < K + 1:
            break
        new = np.array(cand)
        if np.array_equal(new, ref):
            break
        ref = new
        sign = np.sign(e[ref])
    return _to_convention(a), abs(float(E)), ref


def sup_error(h, c, Lambda: float, n: int = 20001) -> float:
    """max |h(x) - p(x)| on a fine uniform grid of [0, Lambda]."""
    x = Lambda * np.arange(n) / (n - 1)
    return float(np.max(np.abs(_hvals(h, x) - chebyshev.series_shifted(c, Lambda, x))))
