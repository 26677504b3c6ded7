"""Exact singular value shrinkage (oracle; test infrastructure only).

  * ``svt_svd``  - G(B) = U diag(g(sigma_i)) V^T, the definition of Sec. III-B,
                   eq. (sing_shrink_exact), with numpy's SVD as the primitive.
  * ``svt_evd``  - the EVD-based exact method of Sec. V-A: eigenpairs of the
                   Gram, shrink lambda_i -> h(lambda_i), B V diag(h) V^T
                   (eqs. sing_shrink_exact_from_eig, sing_shrink_exact_from_eig2).
                   Negative rounding-level eigenvalues are clamped to 0, h(0) = 0.
  * ``cpa_error_from_spectrum`` - the exact CPA-vs-exact error from singular
                   values alone: both results share the singular vectors of B,
                   so ||CPA - exact||_F^2 = sum_i (sigma_i hat h(sigma_i^2) - g(sigma_i))^2.
  * ``eig3_sym``  - eigenvalues of a symmetric 3x3 matrix by the trigonometric
                   closed form of the characteristic cubic (Smith, CACM 1961),
                   used as a brute-force pin for tiny inputs.

Pins: diagonal and rotated-diagonal inputs (closed form), the block matrix of
Sec. V-F (closed-form spectrum), 4x3 inputs via the closed-form cubic.
Parity: pinned.
"""
from __future__ import annotations

import math

import numpy as np

from . import chebyshev


def svt_svd(B: np.ndarray, shrink) -> np.ndarray:
    B = np.asarray(B, dtype=np.float64)
    if B.size == 0:
        return np.zeros(B.shape)
    U, s, Vt = np.linalg.svd(B, full_matrices=False)
    gs = np.array([shrink.g(si) for si in s])
    return (U * gs) @ Vt


def svt_evd(B: np.ndarray, shrink) -> np.ndarray:
    B = np.asarray(B, dtype=np.float64)
    m, n = B.shape
    if B.size == 0:
        return np.zeros(B.shape)
    if m >= n:
        lam, V = np.linalg.eigh(B.T @ B)
    else:
        lam, V = np.linalg.eigh(B @ B.T)
    lam = np.maximum(lam, 0.0)
    hh = np.array([shrink.h(l) if l > 0.0 else 0.0 for l in lam])
    H = (V * hh) @ V.T
    return B @ H if m >= n else H @ B


def cpa_error_from_spectrum(sigmas, shrink, Lambda: float, K: int):
    """(abs_err, rel_err) of the CPA result against the exact shrinkage, from the
    singular values alone."""
    s = np.asarray(sigmas, dtype=np.float64)
    c = chebyshev.coefficients_shifted(shrink, Lambda, K)
    approx = s * chebyshev.series_shifted(c, Lambda, s * s)
    exact = np.array([shrink.g(si) for si in s])
    num = math.sqrt(float(np.sum((approx - exact) ** 2)))
    den = math.sqrt(float(np.sum(exact ** 2)))
    return num, (num / den if den > 0 else num)


def eig3_sym(A: np.ndarray) -> np.ndarray:
    """Eigenvalues (ascending) of a real symmetric 3x3 matrix, closed form."""
    a = np.asarray(A, dtype=np.float64)
    p1 = a[0, 1] ** 2 + a[0, 2] ** 2 + a[1, 2] ** 2
    q = np.trace(a) / 3.0
    if p1 == 0.0:
        return np.sort(np.diag(a))
    p2 = (a[0, 0] - q) ** 2 + (a[1, 1] - q) ** 2 + (a[2, 2] - q) ** 2 + 2.0 * p1
    p = math.sqrt(p2 / 6.0)
    b = (a - q * np.eye(3)) / p
    r = np.linalg.det(b) / 2.0
    r = min(1.0, max(-1.0, r))
    phi = math.acos(r) / 3.0
    e1 = q + 2.0 * p * math.cos(phi)
    e3 = q + 2.0 * p * math.cos(phi + 2.0 * math.pi / 3.0)
    e2 = 3.0 * q - e1 - e3
    return np.sort(np.array([e1, e2, e3]))


def null_vector3(M: np.ndarray) -> np.ndarray:
    """A unit vector spanning the null space of a rank-2 symmetric 3x3 matrix, from
    the largest cross product of its rows."""
    r = [M[0], M[1], M[2]]
    cands = [np.cross(r[0], r[1]), np.cross(r[0], r[2]), np.cross(r[1], r[2])]
    v = max(cands, key=lambda c: float(c @ c))
    return v / math.sqrt(float(v @ v))
