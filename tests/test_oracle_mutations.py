"""Planted mistakes in the oracle (on the CPU only): every plausible slip below
must make at least one pin fail, which shows the pins constrain the code that
matters.  The oracle modules are patched in-process and restored afterwards."""
import math

import numpy as np
import pytest

from oracle import chebyshev, cpa
import oracle.shrinkage as shrinkage_mod
import tests.test_oracle_pins as pins

PIN_FUNCS = [
    pins.test_coefficients_exact_for_polynomials,
    pins.test_interpolation_at_nodes,
    pins.test_matrix_recurrence_acts_on_eigenvalues,
    pins.test_matrix_maps_for_polynomial_responses,
    pins.test_diagonal_and_rotated_inputs,
    lambda: pins.test_block_matrix_D_closed_form(10),
    pins.test_brute_force_4x3,
    pins.test_special_cases,
    pins.test_soft_response_is_max_minus_tau,
]


def _any_pin_fails():
    for f in PIN_FUNCS:
        try:
            f()
        except (AssertionError, ValueError, IndexError):
            return True
    return False


def _coeff_half_node_dropped(h, Lambda, K):
    th = np.array([math.pi * l / K for l in range(1, K + 1)])
    return np.array([2.0 / K * sum(math.cos(k * t) * h(Lambda / 2 * (math.cos(t) + 1)) for t in th)
                     for k in range(K)])


def _coeff_wrong_scale(h, Lambda, K):
    th = chebyshev.node_angles(K)
    return np.array([1.0 / K * sum(math.cos(k * t) * h(Lambda / 2 * (math.cos(t) + 1)) for t in th)
                     for k in range(K)])


def _coeff_no_shift(h, Lambda, K):
    th = chebyshev.node_angles(K)
    return np.array([2.0 / K * sum(math.cos(k * t) * h(Lambda * math.cos(t)) for t in th)
                     for k in range(K)])


def _sum_no_half(Phi, c, Lambda):
    c2 = np.array(c, dtype=float).copy()
    return cpa_orig_sum(Phi, c2, Lambda) + 0.5 * c2[0] * np.eye(Phi.shape[0])


def _sum_wrong_sign(Phi, c, Lambda):
    d = Phi.shape[0]
    Bh = (2.0 / Lambda) * Phi - np.eye(d)
    pp, p = np.eye(d), Bh
    H = 0.5 * c[0] * pp + (c[1] * p if len(c) > 1 else 0)
    for k in range(2, len(c)):
        pn = 2.0 * (Bh @ p) + pp
        H = H + c[k] * pn
        pp, p = p, pn
    return H


def _sum_wrong_shift(Phi, c, Lambda):
    return cpa_orig_sum(Phi * 0.5, c, Lambda)


def _sum_index_slip(Phi, c, Lambda):
    d = Phi.shape[0]
    Bh = (2.0 / Lambda) * Phi - np.eye(d)
    pp, p = np.eye(d), Bh
    H = 0.5 * c[0] * pp + (c[1] * p if len(c) > 1 else 0)
    for k in range(2, len(c)):
        pn = 2.0 * (Bh @ p) - pp
        H = H + c[k - 1] * pn
        pp, p = p, pn
    return H


def _shrink_transposed(B, shrink, Lambda, K):
    B = np.asarray(B, dtype=np.float64)
    if Lambda <= 0:
        return np.zeros(B.shape)
    Phi, side = cpa.gram(B)
    c = chebyshev.coefficients_shifted(shrink, Lambda, K)
    H = cpa.chebyshev_matrix_sum(Phi, c, Lambda)
    return (B @ H.T[::-1, ::-1]) if side == "right" else (H[::-1, ::-1] @ B)


def _h_no_threshold(self, x):
    x = float(x)
    if x <= 0:
        return 0.0
    s = math.sqrt(x)
    return (s - self.tau) / s


cpa_orig_sum = cpa.chebyshev_matrix_sum

MUTATIONS = [
    ("node angle without the half shift", chebyshev, "coefficients_shifted", _coeff_half_node_dropped),
    ("coefficient scale 1/K instead of 2/K", chebyshev, "coefficients_shifted", _coeff_wrong_scale),
    ("nodes not mapped to [0, Lambda]", chebyshev, "coefficients_shifted", _coeff_no_shift),
    ("c_0 not halved", cpa, "chebyshev_matrix_sum", _sum_no_half),
    ("recurrence sign flipped", cpa, "chebyshev_matrix_sum", _sum_wrong_sign),
    ("shift scale wrong", cpa, "chebyshev_matrix_sum", _sum_wrong_shift),
    ("coefficient index off by one", cpa, "chebyshev_matrix_sum", _sum_index_slip),
    ("operand transposed/permuted", cpa, "cpa_shrink", _shrink_transposed),
    ("soft threshold test dropped", shrinkage_mod.Shrinkage, "h", _h_no_threshold),
]


@pytest.mark.parametrize("name,mod,attr,fn", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(monkeypatch, name, mod, attr, fn):
    assert not _any_pin_fails(), "pins must pass on the unmodified oracle"
    monkeypatch.setattr(mod, attr, fn)
    if mod is chebyshev:
        # cpa imported the module, so patching the module attribute is enough
        pass
    assert _any_pin_fails(), f"planted mistake not detected: {name}"


# ---- predictor network: slips in the backward pass or the loss derivative

import tests.test_oracle_mlp as mlp_pins
from oracle import mlp as mlp_mod

MLP_PINS = [mlp_pins.test_gradient_matches_central_differences, mlp_pins.test_linear_closed_form]


def _mlp_pin_fails():
    for f in MLP_PINS:
        try:
            f()
        except AssertionError:
            return True
    return False


def _backward_no_tanh_derivative(p, cache, dy):
    W1, b1, W2, b2, W3, b3 = mlp_mod.unpack(p)
    F, a1, a2 = cache
    dz2 = dy @ W3                       # (1 - a2^2) dropped
    da1 = dz2 @ W2
    dz1 = da1 * (1.0 - a1 * a1)
    return mlp_mod.pack([dz1.T @ F, dz1.sum(0), dz2.T @ a1, dz2.sum(0), dy.T @ a2, dy.sum(0)])


def _backward_transposed_w2(p, cache, dy):
    W1, b1, W2, b2, W3, b3 = mlp_mod.unpack(p)
    F, a1, a2 = cache
    dz2 = (dy @ W3) * (1.0 - a2 * a2)
    da1 = dz2 @ W2.T                    # should be dz2 @ W2
    dz1 = da1 * (1.0 - a1 * a1)
    return mlp_mod.pack([dz1.T @ F, dz1.sum(0), dz2.T @ a1, dz2.sum(0), dy.T @ a2, dy.sum(0)])


def _pinball_sign_flipped(y, t, q):
    loss, dy = mlp_orig_pinball(y, t, q)
    return loss, -dy


mlp_orig_pinball = mlp_mod.pinball


@pytest.mark.parametrize("name,fn", [
    ("backward", _backward_no_tanh_derivative),
    ("backward", _backward_transposed_w2),
    ("pinball", _pinball_sign_flipped),
])
def test_mlp_planted_mistake_is_caught(name, fn, monkeypatch):
    monkeypatch.setattr(mlp_mod, name, fn)
    assert _mlp_pin_fails()
