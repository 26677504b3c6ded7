"""Error metrics (oracle; test infrastructure only).

  * relative Frobenius error ||A - B||_F / ||B||_F, with ||A - B||_F / ||X||_F
    when ||B||_F vanishes (B == 0 is a legitimate exact result);
  * RMSE, the precision metric of Sec. V-A: sqrt(mean((A - B)^2)).
Sums are taken with math.fsum (exactly rounded), so the metric itself adds no
rounding that depends on order.  Parity: pinned by definition.
"""
from __future__ import annotations

import math

import numpy as np


def fro(A) -> float:
    a = np.asarray(A, dtype=np.float64).ravel()
    return math.sqrt(math.fsum((a * a).tolist()))


def rel_fro(A, B, X=None) -> float:
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    num = fro(A - B)
    den = fro(B)
    if den < 1e-300:
        den = fro(X) if X is not None else 1.0
        if den < 1e-300:
            return num
    return num / den


def rmse(A, B) -> float:
    d = (np.asarray(A, dtype=np.float64) - np.asarray(B, dtype=np.float64)).ravel()
    if d.size == 0:
        return 0.0
    return math.sqrt(math.fsum((d * d).tolist()) / d.size)
