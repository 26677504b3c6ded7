"""Sparsifying transform and component truncation of Algorithm 1 (oracle; test
infrastructure only).

Sec. III-B writes the shrinkage with an orthogonal forward transform T:
  Phi = T B^T B T^T                                   (eq. sing_shrink_exact_sparse)
  underline Phi_ij = Phi_ij if |Phi_ij| >= eps, else 0 (eq. threshold_components)
  hat G(B) = B T^T hat H(underline Phi) T             (Algorithm 1, last step)
with hat H by Algorithm 1's three-term recurrence (oracle.cpa.chebyshev_matrix_sum).
The threshold is eps = K(|Phi|, k), the k-th largest entry of |Phi|
(Sec. V, eq. recommendation_epsilon, where k is a fraction of n^2).

Readings where the paper is silent:
  * K(|underline Phi|, k) in eq. (recommendation_epsilon) is read as K(|Phi|, k):
    the threshold is taken on the transformed Gram before truncation (the
    truncated matrix cannot define its own threshold).
  * entries equal to eps are kept (>=), so ties at the k-th value keep more
    than k entries -- Phi is symmetric, so an off-diagonal k-th value always
    brings its mirror entry (k or k + 1 entries are kept when no other values tie);
  * m < n uses the transposed identity, hat G(B) = T^T hat H(T B B^T T^T) T B.
  * the computed product T G T^T is symmetrised, (Phi + Phi^T)/2, before the
    threshold: rounding makes it slightly asymmetric, and an entry and its mirror
    could then land on different sides of eps and give a non-symmetric matrix.

Transforms (forward, orthonormal rows):
  dct_matrix(n)    D[k, j] = s_k cos(pi (2 j + 1) k / (2 n)), s_0 = sqrt(1/n),
                   s_k = sqrt(2/n) (DCT-II)
  block_dct(n, b)  kron(I_{n/b}, dct_matrix(b)): the b x b block DCT, b = 8 in the paper
  haar_matrix(n)   one-level Haar DWT: row q < n/2 is (e_2q + e_2q+1)/sqrt 2 (low
                   pass), row n/2 + q is (e_2q - e_2q+1)/sqrt 2 (high pass).  The
                   experiments of Sec. V use it with every high-frequency
                   component set to zero: `zero` below marks those components,
                   whose rows and columns of Phi are zeroed before the threshold.

Pins (tests/test_oracle_sparsify.py): the DCT matrix equals scipy's orthonormal
DCT-II and is orthogonal; without truncation (k = n^2) the result equals the
T = Id shrinkage for every orthogonal T (an orthogonal similarity); with
truncation it equals the spectral form built from an eigendecomposition of the
truncated matrix; eps equals the k-th value of a full sort; the Haar matrix
maps hand-computed vectors to their sums and differences; with the high
frequencies zeroed the result equals B T_L^T hat h(Phi_LL) T_L + hat h(0) B T_H^T T_H
from an eigendecomposition of the low-pass block.  Parity: pinned.

Adaptive keep count (eq. recommendation_epsilon, with the thresholds E_l = 0.03
and E_m = 6e-4 and the counts k_1, k_2, k_3 of Table IV):
  k = (0.5e-4) n^2 if E_t > E_l;  (1.5e-4) n^2 if E_l >= E_t > E_m;  (0.5e-3) n^2 otherwise.
Readings: a fractional count is rounded up, in exact rational arithmetic (the
fractions are 1/20000, 3/20000 and 1/2000 of n^2), and clamped to [1, n^2]; E_t is
the previous iteration's ADMM change, and the first iteration, which has none,
takes E_t = +inf (the first case).  Pins: Table IV's caption gives k_1 = 50,
k_2 = 150, k_3 = 500 at n = 1000; the case edges E_t = E_l and E_t = E_m.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from . import chebyshev
from .cpa import chebyshev_matrix_sum


def dct_matrix(n: int) -> np.ndarray:
    """Orthonormal DCT-II matrix (rows are the basis functions; D @ x transforms x)."""
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    D = np.cos(math.pi * (2 * j + 1) * k / (2.0 * n))
    D[0, :] *= math.sqrt(1.0 / n)
    D[1:, :] *= math.sqrt(2.0 / n)
    return D


def block_dct(n: int, b: int = 8) -> np.ndarray:
    """kron(I_{n/b}, D_b): the b x b block DCT of length-n vectors (n a multiple of b)."""
    if n % b:
        raise ValueError("n must be a multiple of the block size")
    return np.kron(np.eye(n // b), dct_matrix(b))


def haar_matrix(n: int) -> np.ndarray:
    """One-level orthonormal Haar DWT of length-n vectors (n even): low-pass
    outputs first, then high-pass."""
    if n % 2:
        raise ValueError("n must be even")
    H = np.zeros((n, n))
    r = math.sqrt(0.5)
    for q in range(n // 2):
        H[q, 2 * q] = H[q, 2 * q + 1] = r
        H[n // 2 + q, 2 * q] = r
        H[n // 2 + q, 2 * q + 1] = -r
    return H


def transformed_gram(B: np.ndarray, T: np.ndarray):
    """Algorithm 1 step 1: (Phi, side) with Phi = T B^T B T^T (m >= n, 'right') or
    T B B^T T^T (m < n, 'left')."""
    B = np.asarray(B, dtype=np.float64)
    m, n = B.shape
    G = B.T @ B if m >= n else B @ B.T
    Phi = T @ G @ T.T
    # exactly symmetric, like the true Phi: otherwise an entry and its mirror can
    # fall on different sides of the threshold
    return 0.5 * (Phi + Phi.T), ("right" if m >= n else "left")


def kth_largest_abs(Phi: np.ndarray, k: int) -> float:
    """K(|Phi|, k): the k-th largest entry of |Phi| (1 <= k <= Phi.size)."""
    a = np.abs(np.asarray(Phi, dtype=np.float64)).ravel()
    if not 1 <= k <= a.size:
        raise ValueError("k out of range")
    return float(np.partition(a, a.size - k)[a.size - k])


def truncate(Phi: np.ndarray, eps: float) -> np.ndarray:
    """eq. (threshold_components): keep the entries with |Phi_ij| >= eps."""
    Phi = np.asarray(Phi, dtype=np.float64)
    return np.where(np.abs(Phi) >= eps, Phi, 0.0)


def keep_count(n: int, fraction: float) -> int:
    """k for a kept fraction of the n x n entries (eq. recommendation_epsilon writes
    k = f n^2): ceil(f n^2), at least 1."""
    return max(1, int(math.ceil(fraction * n * n)))


def keep_schedule(E_t: float, n: int, E_l: float = 0.03, E_m: float = 6e-4) -> int:
    """eq. (recommendation_epsilon): the keep count k of K(|Phi|, k) for the ADMM
    change E_t, on an n x n transformed Gram."""
    if math.isnan(E_t):
        raise ValueError("E_t is NaN")
    if E_t > E_l:
        f = Fraction(1, 20000)     # 0.5e-4
    elif E_t > E_m:
        f = Fraction(3, 20000)     # 1.5e-4
    else:
        f = Fraction(1, 2000)      # 0.5e-3
    k = math.ceil(f * n * n)
    return min(max(k, 1), n * n)


def cpa_shrink_sparsified(B: np.ndarray, shrink, Lambda: float, K: int, T: np.ndarray, k, zero=None, eps=None):
    """hat G(B) by Algorithm 1 with transform T and threshold eps = K(|Phi|, k), or
    the given eps of eq. (threshold_components) (k = None; the experiments of Table
    III fix eps).
    zero (optional boolean mask over the transform's components): those rows and
    columns of Phi are set to zero first (the high frequencies of the DWT in
    Sec. V).  Lambda must bound the largest eigenvalue of the truncated matrix; it
    is taken as given.  Returns (result, eps, kept entries)."""
    B = np.asarray(B, dtype=np.float64)
    m, n = B.shape
    Phi, side = transformed_gram(B, T)
    if zero is not None:
        Phi = Phi.copy()
        Phi[zero, :] = 0.0
        Phi[:, zero] = 0.0
    if eps is None:
        eps = kth_largest_abs(Phi, k)
    Phil = truncate(Phi, eps)
    nnz = int(np.count_nonzero(np.abs(Phi) >= eps))
    # nothing kept: the truncated matrix is zero and so is its largest eigenvalue;
    # every shrink function here has h(0) = 0, so the result is zero whatever Lambda
    if Lambda <= 0.0 or nnz == 0:
        return np.zeros((m, n)), eps, nnz
    c = chebyshev.coefficients_shifted(shrink, Lambda, K)
    H = chebyshev_matrix_sum(Phil, c, Lambda)
    M = T.T @ H @ T
    return (B @ M if side == "right" else M @ B), eps, nnz
