"""The library's host designs (cpa_design_coeffs) against the oracle's (least squares
and minimax of Sec. IV-B, eq. (l_p_norm_for_approximation)).  Both minimisers are
unique on their point sets, so two independent solvers must agree; no GPU needed."""
import numpy as np
import pytest

import paper_1705_07112_amd as cpa
from oracle import chebyshev, design
from oracle.shrinkage import hard, soft, weighted_const

LAM = 7.3
CASES = [(cpa.soft(0.8), soft(0.8)), (cpa.hard(1.1), hard(1.1)), (cpa.weighted_const(0.5), weighted_const(0.5))]


@pytest.mark.parametrize("i", range(3))
@pytest.mark.parametrize("K", [1, 10, 30, 50])
def test_lsq_matches_the_oracle(i, K):
    lib_sh, ora_sh = CASES[i]
    c, err = cpa.design_coeffs(lib_sh, LAM, K, "lsq", 2000)
    ref = design.lsq(ora_sh, LAM, K, 2000)
    assert np.max(np.abs(c - ref)) <= 1e-9 * max(1.0, float(np.max(np.abs(ref))))
    x = design.sample_points(LAM, 2000)
    e = np.array([ora_sh.h(v) for v in x]) - chebyshev.series_shifted(ref, LAM, x)
    assert abs(err - float(np.max(np.abs(e)))) <= 1e-12 + 1e-9 * err


@pytest.mark.parametrize("i", range(3))
@pytest.mark.parametrize("K", [2, 10, 20, 30])
def test_minimax_matches_the_oracle(i, K):
    lib_sh, ora_sh = CASES[i]
    c, err = cpa.design_coeffs(lib_sh, LAM, K, "minimax", 8000)
    ref, E, _ = design.minimax(ora_sh, LAM, K, 8000)
    x = design.remez_grid(LAM, 8000)
    h = np.array([ora_sh.h(v) for v in x])
    e_lib = float(np.max(np.abs(h - chebyshev.series_shifted(c, LAM, x))))
    # both are the grid's best approximation within the stopping rule's 1e-10
    assert abs(e_lib - E) <= 1e-8 * E + 1e-13
    assert abs(err - e_lib) <= 1e-12 + 1e-9 * e_lib
    assert np.max(np.abs(c - ref)) <= 1e-5 * max(1.0, float(np.max(np.abs(ref))))


def test_chebyshev_design_is_the_cpa_coefficients():
    c, err = cpa.design_coeffs(cpa.soft(0.8), LAM, 25, "chebyshev")
    assert np.array_equal(c, cpa.chebyshev_coeffs(cpa.soft(0.8), LAM, 25))
    assert err < 1e-12   # the interpolant is exact at its own nodes


def test_zero_lambda_and_arguments():
    c, err = cpa.design_coeffs(cpa.soft(0.8), 0.0, 7, "minimax")
    assert np.all(c == 0) and err == 0
    for K, d, n in [(0, "lsq", 0), (1025, "lsq", 0), (20, "lsq", 19), (20, "minimax", 40), (2, "lsq", 1 << 21),
                    (1024, "minimax", 1 << 17)]:
        with pytest.raises(RuntimeError):
            cpa.design_coeffs(cpa.soft(0.8), LAM, K, d, n)
    with pytest.raises(RuntimeError):
        cpa.design_coeffs(cpa.soft(0.8), -1.0, 5, "lsq")
    with pytest.raises(RuntimeError):
        cpa._check(cpa.lib().cpa_design_coeffs(cpa.soft(0.8), LAM, 5, 3, 0, (cpa.ctypes.c_double * 5)(), None))
