"""Generic shrinkage response family (oracle; test infrastructure only).

Paper passage: Sec. IV-A, eq. (filter_response_ours):
    h(x; w(x)/rho, tau) = (sqrt(x) - w(x)/rho) / sqrt(x)   if sqrt(x) > tau
                        = 0                                  otherwise
with the three named members
    hard          h(x; 0, tau_hard)
    weighted soft h(x; w(x)/rho, w(x)/rho)
    soft          h(x; 1/rho, 1/rho)      =>  g(s) = max(s - 1/rho, 0)
and g(sqrt(x)) = sqrt(x) h(x) (Sec. III-B, after eq. sing_shrink_from_eig_shrink).

Readings where the paper is silent:
  * the threshold compares sqrt(x) (a singular value), strictly (> tau);
    sqrt(x) == tau gives 0.  The hard response of eq. (ideal_filter_response)
    is written on x in [0,1]; here it is applied to sqrt(x) as in
    eq. (filter_response_ours).
  * x <= 0 gives h = 0 (a zero singular value is not kept).
  * the weight function: a constant, or the reweighting
        w(x) = w_c / (sqrt(max(x - w_sigma, 0)) + w_eps)
    evaluated on x = sigma^2 (a weighted nuclear norm style weight; its
    constants are project choices, not the paper's).
Kinds are encoded as small integers shared by convention with the C header:
SOFT=0, HARD=1, WEIGHTED_CONST=2, WEIGHTED_FN=3 (the oracle re-declares them;
it includes nothing from the library).

Pins: soft response reproduces max(s - tau, 0) exactly; hard keeps s for
s > tau; weighted constant equals soft at tau = w; tie at the threshold.
Parity: pinned.
"""
from __future__ import annotations

import math

SOFT, HARD, WEIGHTED_CONST, WEIGHTED_FN = 0, 1, 2, 3


class Shrinkage:
    """Parameters of one member of the family.

    kind SOFT:            tau = 1/rho
    kind HARD:            tau = tau_hard
    kind WEIGHTED_CONST:  tau = w / rho (one constant weight)
    kind WEIGHTED_FN:     w(x) = w_c / (sqrt(max(x - w_sigma, 0)) + w_eps), threshold = w(x)
    """

    def __init__(self, kind: int = SOFT, tau: float = 0.0, w_c: float = 0.0,
                 w_sigma: float = 0.0, w_eps: float = 1e-6):
        self.kind = int(kind)
        self.tau = float(tau)
        self.w_c = float(w_c)
        self.w_sigma = float(w_sigma)
        self.w_eps = float(w_eps)

    def weight(self, x: float) -> float:
        return self.w_c / (math.sqrt(max(x - self.w_sigma, 0.0)) + self.w_eps)

    def h(self, x: float) -> float:
        """Eigenvalue response h(x), x = sigma^2 (eq. filter_response_ours)."""
        x = float(x)
        if x <= 0.0:
            return 0.0
        s = math.sqrt(x)
        if self.kind == SOFT or self.kind == WEIGHTED_CONST:
            w, t = self.tau, self.tau
        elif self.kind == HARD:
            w, t = 0.0, self.tau
        elif self.kind == WEIGHTED_FN:
            w = self.weight(x)
            t = w
        else:
            raise ValueError("unknown shrinkage kind")
        if s > t:
            return (s - w) / s
        return 0.0

    def g(self, s: float) -> float:
        """Singular value response g(s) = s h(s^2)."""
        s = float(s)
        return s * self.h(s * s)

    def __call__(self, x):
        return self.h(x)


def soft(tau: float) -> Shrinkage:
    return Shrinkage(SOFT, tau)


def hard(tau: float) -> Shrinkage:
    return Shrinkage(HARD, tau)


def weighted_const(w_over_rho: float) -> Shrinkage:
    return Shrinkage(WEIGHTED_CONST, w_over_rho)


def weighted_fn(w_c: float, w_sigma: float, w_eps: float = 1e-6) -> Shrinkage:
    return Shrinkage(WEIGHTED_FN, 0.0, w_c, w_sigma, w_eps)
