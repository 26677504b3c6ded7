"""Pins for the optional damping of the Chebyshev coefficients (Jackson and
Lanczos factors of the kernel polynomial method; not in the paper): values
fixed in closed form and the ripple behaviour of a damped step (the hard
threshold's response)."""
import math

import numpy as np
import pytest

from oracle import chebyshev, cpa
from oracle.shrinkage import Shrinkage


@pytest.mark.parametrize("K", [1, 2, 5, 30, 64])
def test_damping_closed_forms(K):
    for kind in ("jackson", "lanczos"):
        g = chebyshev.damping_factors(K, kind)
        assert g[0] == 1.0 and len(g) == K
        assert np.all(g <= 1.0 + 1e-15) and np.all(g > -1e-15)
    if K > 1:
        # Jackson: g_1 = ((N) cos t + sin t cot t)/(N + 1) = cos t with t = pi/(N + 1)
        assert abs(chebyshev.damping_factors(K, "jackson")[1] - math.cos(math.pi / K)) <= 1e-15
        # Lanczos: sigma factors vanish at k = N + 1 = K; the last one is sin(pi (K-1)/K) / (pi (K-1)/K)
        assert abs(chebyshev.damping_factors(K, "lanczos")[-1] - math.sin(math.pi / K) / (math.pi * (K - 1) / K)) <= 1e-15
    assert np.array_equal(chebyshev.damping_factors(K, "none"), np.ones(K))


@pytest.mark.parametrize("K", [16, 30, 64, 128])
def test_jackson_damped_step_has_no_ripple(K):
    """The hard threshold's response is a step on [0, Lambda]: undamped it
    overshoots by more than 10% (Gibbs), Jackson-damped it stays in [0, 1] (a
    positive kernel), Lanczos-damped within 3%."""
    lam = 1.0
    x = np.linspace(0.0, lam, 4001)
    sh = Shrinkage(1, math.sqrt(0.3))
    c = chebyshev.coefficients_shifted(sh, lam, K)
    f0 = chebyshev.series_shifted(c, lam, x)
    fj = chebyshev.series_shifted(c * chebyshev.damping_factors(K, "jackson"), lam, x)
    fl = chebyshev.series_shifted(c * chebyshev.damping_factors(K, "lanczos"), lam, x)
    assert f0.max() > 1.1 and f0.min() < -0.1
    assert fj.min() >= -1e-12 and fj.max() <= 1.0 + 1e-12
    assert fl.max() < 1.03 and fl.min() > -0.03


def test_damped_shrink_of_a_diagonal_matrix():
    """Diagonal X: the damped shrink scales each diagonal entry s by the damped
    series at s^2 (times s), computed here from the scalar series."""
    s = np.array([0.2, 0.5, 0.9, 1.3, 2.0])
    X = np.diag(s)
    lam = 1.01 * s.max() ** 2
    sh = Shrinkage(1, 0.8)
    K = 24
    c = chebyshev.coefficients_shifted(sh, lam, K) * chebyshev.damping_factors(K, "jackson")
    ref = np.diag(s * chebyshev.series_shifted(c, lam, s ** 2))
    Y = cpa.cpa_shrink(X, sh, lam, K, damping="jackson")
    assert np.abs(Y - ref).max() <= 1e-12
