"""CPA-based singular value shrinkage (oracle; test infrastructure only).

Main routine ``cpa_shrink`` follows Algorithm 1 (Sec. III-B) with the
sparsifying transform T = Id and no component truncation (epsilon = 0), so
Phi = underline(Phi) = B^T B:
  step 1   Phi <- B^T B
  step 3   Lambda_max (passed in; see oracle.bound for the estimate)
  step 4   hat c_k    (eq. chebychev_coeff_shifted, oracle.chebyshev)
  step 5   hat B <- (2 / Lambda_max) Phi - Id          (eq. transform_lamB)
  step 6-7 Psi_0 = Id, Psi_1 = hat B, H = c_0/2 Psi_0 + c_1 Psi_1
  step 8-10 Psi_k = 2 hat B Psi_{k-1} - Psi_{k-2}, H += c_k Psi_k
           (eqs. cheby_matrix_eigen_saiki3, recurrence_our_method)
  step 12  hat G(B) = B H
The identity G(B) = B H(B^T B) with h(x) = g(sqrt x)/sqrt x is
eq. (sing_shrink_from_eig_shrink).

Readings where the paper is silent:
  * the paper treats m > n.  For m < n the oracle uses the transposed
    identity  G(B) = H(B B^T) B  (the shrinkage of B^T, transposed back);
    m == n uses the B^T B side.
  * K == alpha == number of coefficients (degree K-1); K = 1 gives c_0/2 * B.
  * Lambda == 0 (B == 0) returns the zero matrix without dividing.

Cross-check forms (used only in tests, all equal to ``cpa_shrink`` in exact
arithmetic):
  * ``cpa_shrink_yform``  - the same sum distributed over B:
        Y_0 = B, Y_1 = B hat B, Y_k = 2 Y_{k-1} hat B - Y_{k-2}, result sum c_k Y_k
  * ``cpa_shrink_spectral`` - B V diag(hat h(lambda_i)) V^T from an EVD of the
        Gram (eq. chebychev_series_matrix_shift2)
  * ``cpa_shrink_operator`` - for the m >= n case written with the left Gram:
        Y_{k+1} = 2 ((2/Lambda) B (B^T Y_k) - Y_k) - Y_{k-1}, which never forms
        an n x n or m x m matrix product with a dense operand other than B.

Pins: polynomial h (h = 1, h = x, h = T_j) give closed forms; the four forms
agree; shrinkage of diagonal and rotated-diagonal inputs equals the scalar
interpolant on their singular values; invariances (transpose, orthogonal
rotation, homogeneity).  Parity: pinned.
"""
from __future__ import annotations

import numpy as np

from . import chebyshev


def gram(B: np.ndarray):
    """Algorithm 1 step 1 with T = Id.  Returns (Phi, side) with side 'right'
    (Phi = B^T B, m >= n) or 'left' (Phi = B B^T, m < n)."""
    m, n = B.shape
    if m >= n:
        return B.T @ B, "right"
    return B @ B.T, "left"


def chebyshev_matrix_sum(Phi: np.ndarray, c: np.ndarray, Lambda: float) -> np.ndarray:
    """Algorithm 1 steps 5-10: hat H(Phi) = c_0/2 Id + sum_{k>=1} c_k Psi_k(hat B),
    hat B = (2/Lambda) Phi - Id, Psi by the matrix three-term recurrence."""
    d = Phi.shape[0]
    K = len(c)
    Id = np.eye(d)
    Bh = (2.0 / Lambda) * Phi - Id
    psi_prev = Id
    H = 0.5 * c[0] * psi_prev
    if K == 1:
        return H
    psi = Bh
    H = H + c[1] * psi
    for k in range(2, K):
        psi_next = 2.0 * (Bh @ psi) - psi_prev
        H = H + c[k] * psi_next
        psi_prev, psi = psi, psi_next
    return H


def cpa_shrink(B: np.ndarray, shrink, Lambda: float, K: int, damping: str = "none") -> np.ndarray:
    """hat G(B) by Algorithm 1 (T = Id, epsilon = 0).  ``shrink`` is a callable h(x)
    (e.g. oracle.shrinkage.Shrinkage).  Lambda must bound the Gram's largest
    eigenvalue; it is taken as given.  ``damping`` multiplies the coefficients by
    chebyshev.damping_factors (not in the paper)."""
    B = np.asarray(B, dtype=np.float64)
    if K < 1:
        raise ValueError("K must be >= 1")
    m, n = B.shape
    if m == 0 or n == 0:
        return np.zeros((m, n))
    if Lambda <= 0.0:
        return np.zeros((m, n))
    Phi, side = gram(B)
    c = chebyshev.coefficients_shifted(shrink, Lambda, K) * chebyshev.damping_factors(K, damping)
    H = chebyshev_matrix_sum(Phi, c, Lambda)
    if side == "right":
        return B @ H
    return H @ B


def cpa_shrink_yform(B: np.ndarray, shrink, Lambda: float, K: int, c=None) -> np.ndarray:
    """The Algorithm 1 sum distributed over B (cross-check form)."""
    B = np.asarray(B, dtype=np.float64)
    m, n = B.shape
    if m == 0 or n == 0 or Lambda <= 0.0:
        return np.zeros((m, n))
    Phi, side = gram(B)
    if c is None:
        c = chebyshev.coefficients_shifted(shrink, Lambda, K)
    d = Phi.shape[0]
    Bh = (2.0 / Lambda) * Phi - np.eye(d)

    def apply(Y):
        return Y @ Bh if side == "right" else Bh @ Y

    y_prev = B
    acc = 0.5 * c[0] * y_prev
    if len(c) == 1:
        return acc
    y = apply(B)
    acc = acc + c[1] * y
    for k in range(2, len(c)):
        y_next = 2.0 * apply(y) - y_prev
        acc = acc + c[k] * y_next
        y_prev, y = y, y_next
    return acc


def cpa_shrink_spectral(B: np.ndarray, shrink, Lambda: float, K: int) -> np.ndarray:
    """B V diag(hat h(lambda_i)) V^T (right) or U diag(hat h) U^T B (left), the
    closed form of the CPA result on the Gram's eigenpairs (cross-check form)."""
    B = np.asarray(B, dtype=np.float64)
    m, n = B.shape
    if m == 0 or n == 0 or Lambda <= 0.0:
        return np.zeros((m, n))
    Phi, side = gram(B)
    lam, V = np.linalg.eigh(Phi)
    c = chebyshev.coefficients_shifted(shrink, Lambda, K)
    hh = chebyshev.series_shifted(c, Lambda, lam)
    H = (V * hh) @ V.T
    return B @ H if side == "right" else H @ B


def cpa_shrink_operator(B: np.ndarray, shrink, Lambda: float, K: int) -> np.ndarray:
    """Y-form with the Gram applied as an operator through B (cross-check form
    for sparse inputs): for m >= n, B p(B^T B) = p(B B^T) B, and
    (B B^T) Y = B (B^T Y) never needs the m x m product."""
    B = np.asarray(B, dtype=np.float64)
    m, n = B.shape
    if m == 0 or n == 0 or Lambda <= 0.0:
        return np.zeros((m, n))
    c = chebyshev.coefficients_shifted(shrink, Lambda, K)

    def apply(Y):
        if m >= n:
            return (2.0 / Lambda) * (B @ (B.T @ Y)) - Y
        return (2.0 / Lambda) * ((Y @ B.T) @ B) - Y

    y_prev = B
    acc = 0.5 * c[0] * y_prev
    if K == 1:
        return acc
    y = apply(B)
    acc = acc + c[1] * y
    for k in range(2, K):
        y_next = 2.0 * apply(y) - y_prev
        acc = acc + c[k] * y_next
        y_prev, y = y, y_next
    return acc


def cpa_rows_yform(Phi: np.ndarray, Brows: np.ndarray, shrink, Lambda: float, K: int) -> np.ndarray:
    """Rows of the m >= n Y-form result from the full Gram Phi = B^T B and the
    selected rows of B (row r of Y_{k+1} = 2 Y_k[r] hat B - Y_{k-1}[r] needs only
    row r).  For inputs whose Gram is cheap to form but whose H-form is not."""
    Phi = np.asarray(Phi, dtype=np.float64)
    Brows = np.asarray(Brows, dtype=np.float64)
    if Lambda <= 0.0:
        return np.zeros(Brows.shape)
    c = chebyshev.coefficients_shifted(shrink, Lambda, K)
    Bh = (2.0 / Lambda) * Phi - np.eye(Phi.shape[0])
    y_prev = Brows
    acc = 0.5 * c[0] * y_prev
    if K == 1:
        return acc
    y = Brows @ Bh
    acc = acc + c[1] * y
    for k in range(2, K):
        y_next = 2.0 * (y @ Bh) - y_prev
        acc = acc + c[k] * y_next
        y_prev, y = y, y_next
    return acc


def cpa_rows(B: np.ndarray, shrink, Lambda: float, K: int, rows) -> np.ndarray:
    """Selected output rows of ``cpa_shrink`` for the m >= n side: hat H is
    formed once (Algorithm 1 steps 1-10) and only B[rows] H is multiplied out
    (rows of B H depend only on the same rows of B).  Used to check full-size
    results on a sample of outputs."""
    B = np.asarray(B, dtype=np.float64)
    m, n = B.shape
    assert m >= n
    if Lambda <= 0.0:
        return np.zeros((len(rows), n))
    Phi, _ = gram(B)
    c = chebyshev.coefficients_shifted(shrink, Lambda, K)
    H = chebyshev_matrix_sum(Phi, c, Lambda)
    return B[np.asarray(rows)] @ H
