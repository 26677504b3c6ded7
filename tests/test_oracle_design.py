"""Pins for the polynomial designs compared with CPA in Sec. IV-B (least squares
and minimax, eq. (l_p_norm_for_approximation)), each against what approximation
theory fixes, not against the oracle's own algebra."""
import math

import numpy as np
import pytest

from oracle import chebyshev, design
from oracle.shrinkage import hard, soft, weighted_const


class Poly:
    def __init__(self, f):
        self.f = f

    def h(self, x):
        return self.f(x)

    def __call__(self, x):
        return self.f(x)


LAM = 7.3


def _tk(k, Lam=LAM):
    return Poly(lambda x: math.cos(k * math.acos(max(-1.0, min(1.0, 2.0 * x / Lam - 1.0)))))


@pytest.mark.parametrize("K", [3, 8, 17])
def test_designs_reproduce_polynomials(K):
    """A response that is a polynomial of degree < K is reproduced exactly by every
    design: coefficients delta_jk for T_j, and (Lambda, Lambda/2, 0, ...) for h = x."""
    for j in (0, 1, K - 1):
        e = np.zeros(K)
        e[j] = 2.0 if j == 0 else 1.0
        for c in (design.lsq(_tk(j), LAM, K, 500), design.minimax(_tk(j), LAM, K, 3000)[0]):
            assert np.max(np.abs(c - e)) < 1e-9, (j, c[:4])
    x = Poly(lambda v: v)
    ref = np.zeros(K)
    ref[0], ref[1] = LAM, LAM / 2
    assert np.max(np.abs(design.lsq(x, LAM, K, 500) - ref)) < 1e-9
    c, E, _ = design.minimax(x, LAM, K, 3000)
    assert np.max(np.abs(c - ref)) < 1e-9 and E < 1e-9


@pytest.mark.parametrize("K", [4, 7, 12])
def test_minimax_of_the_next_chebyshev_polynomial(K):
    """Chebyshev: the best uniform approximation of T_K by polynomials of degree < K is
    zero, with error max |T_K| = 1, attained with alternating signs at the K + 1
    extrema of T_K (on the Remez grid, which contains them: K divides n - 1)."""
    c, E, ref = design.minimax(_tk(K), LAM, K, 4201)
    assert np.max(np.abs(c)) < 1e-9
    assert abs(E - 1.0) < 1e-9
    x = design.remez_grid(LAM, 4201)[ref]
    t = 2.0 * x / LAM - 1.0
    ext = np.cos(np.pi * np.arange(K + 1) / K)
    assert np.max(np.abs(np.sort(t) - np.sort(ext))) < 1e-12


@pytest.mark.parametrize("sh,K", [(soft(0.8), 10), (soft(0.8), 20), (hard(1.1), 10), (weighted_const(0.5), 20)])
def test_minimax_equioscillates(sh, K):
    """The minimax error reaches its maximum on the grid at K + 1 reference points,
    with alternating signs (the alternation theorem), and no other design has a
    smaller maximum error on that grid."""
    n = 8000
    c, E, ref = design.minimax(sh, LAM, K, n)
    x = design.remez_grid(LAM, n)
    e = np.array([sh.h(v) for v in x]) - chebyshev.series_shifted(c, LAM, x)
    assert len(ref) == K + 1
    assert np.max(np.abs(np.abs(e[ref]) - E)) <= 1e-8 * max(E, 1e-300)
    assert np.all(np.sign(e[ref][1:]) == -np.sign(e[ref][:-1]))
    assert np.max(np.abs(e)) <= E * (1 + 1e-8)
    for other in (chebyshev.coefficients_shifted(sh, LAM, K), design.lsq(sh, LAM, K, 2000)):
        eo = np.array([sh.h(v) for v in x]) - chebyshev.series_shifted(other, LAM, x)
        assert np.max(np.abs(eo)) >= E * (1 - 1e-9)


@pytest.mark.parametrize("sh,K", [(soft(0.8), 10), (hard(1.1), 20), (weighted_const(0.5), 15)])
def test_lsq_residual_is_orthogonal(sh, K):
    """First-order optimality of least squares: on the samples, the residual is
    orthogonal to every polynomial of degree < K (checked against the monomials
    u^k, a different basis from the solver's)."""
    n = 2000
    c = design.lsq(sh, LAM, K, n)
    x = design.sample_points(LAM, n)
    r = np.array([sh.h(v) for v in x]) - chebyshev.series_shifted(c, LAM, x)
    u = x / LAM
    for k in range(K):
        assert abs(float(np.sum(r * u ** k))) <= 1e-9 * math.sqrt(n) * float(np.linalg.norm(u ** k))


@pytest.mark.parametrize("sh,K", [(soft(0.8), 6), (hard(1.1), 8), (weighted_const(0.5), 10)])
def test_lsq_matches_the_vandermonde_pseudo_inverse(sh, K):
    """The paper's route, c = Upsilon^+ h with monomials, gives the same polynomial as
    the Chebyshev-basis solver where the Vandermonde matrix is well conditioned."""
    a = design.lsq_vandermonde(sh, LAM, K, 400)
    b = design.lsq(sh, LAM, K, 400)
    assert np.max(np.abs(a - b)) <= 1e-7 * max(1.0, float(np.max(np.abs(b))))


def test_error_orders_of_the_designs():
    """On each design's own measure it is the best of the three: least squares has
    the smallest sum of squares on its samples, minimax the smallest maximum on its
    grid (soft threshold, K = 20)."""
    sh, K = soft(0.8), 20
    cs = {"cpa": chebyshev.coefficients_shifted(sh, LAM, K), "lsq": design.lsq(sh, LAM, K, 2000),
          "minimax": design.minimax(sh, LAM, K, 8000)[0]}
    xs = design.sample_points(LAM, 2000)
    hs = np.array([sh.h(v) for v in xs])
    l2 = {k: float(np.sum((hs - chebyshev.series_shifted(c, LAM, xs)) ** 2)) for k, c in cs.items()}
    xg = design.remez_grid(LAM, 8000)
    hg = np.array([sh.h(v) for v in xg])
    linf = {k: float(np.max(np.abs(hg - chebyshev.series_shifted(c, LAM, xg)))) for k, c in cs.items()}
    assert l2["lsq"] <= min(l2.values()) * (1 + 1e-12)
    assert linf["minimax"] <= min(linf.values()) * (1 + 1e-9)


@pytest.mark.parametrize("K", [20, 50])
def test_stop_band_ripple_of_the_hard_threshold(K):
    """The comparison of Sec. IV-B: on the hard threshold CPA leaves less ripple in
    the stop band (x < tau^2, where h = 0) than least squares and minimax, which
    both keep about half the step height there (Gibbs-like, and levelled)."""
    sh, Lam = hard(0.3), 1.0
    x = np.linspace(0.0, Lam, 20001)
    stop = x < 0.3 ** 2
    cs = {"cpa": chebyshev.coefficients_shifted(sh, Lam, K), "lsq": design.lsq(sh, Lam, K, 2000),
          "minimax": design.minimax(sh, Lam, K, 8000)[0]}
    ripple = {k: float(np.max(np.abs(chebyshev.series_shifted(c, Lam, x)[stop]))) for k, c in cs.items()}
    assert ripple["cpa"] < 0.8 * min(ripple["lsq"], ripple["minimax"]), ripple
    assert min(ripple["lsq"], ripple["minimax"]) > 0.45
