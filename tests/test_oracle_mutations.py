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


# ---- drivers (Appendix B ADMM, SVT): slips in the iteration's algebra --------

import tests.test_oracle_drivers as drv_pins
from oracle import drivers as drv_mod
from oracle import bound as bound_mod
from oracle.shrinkage import soft as _soft

_rpca_step_orig = drv_mod.rpca_step
_svt_orig = drv_mod.svt_complete


def _rpca_pins_fail(monkeypatch):
    for f in (drv_pins.test_rpca_exact_prox_meets_pcp_optimality, drv_pins.test_rpca_cpa_recovers_planted_parts):
        try:
            with monkeypatch.context() as mp:
                f(mp) if f is drv_pins.test_rpca_exact_prox_meets_pcp_optimality else f()
        except (AssertionError, FloatingPointError, np.linalg.LinAlgError, ValueError):
            return True
    return False


def _rpca_step_variant(z1_from_l=False, u3_keeps_I=False, swap_ls=False, z2_tau_from_rho=False):
    def step(state, I, inv_rho, eta_over_rho, K, v=None, seed=0, power_iters=100, tol_power=1e-7, delta=0.01):
        I = np.asarray(I, dtype=np.float64)
        l_new, s_new = drv_mod.admm_lsolve(state["z1"], state["z2"], I, state["u1"], state["u2"], state["u3"])
        if swap_ls:
            l_new, s_new = s_new, l_new
        x = l_new if z1_from_l else l_new + state["u1"]
        Phi, _ = cpa.gram(x)
        Lam, _, _, _, v = bound_mod.power_bound(Phi, seed=seed, max_iter=power_iters, tol=tol_power,
                                                delta=delta, v0=v)
        z1 = cpa.cpa_shrink(x, _soft(inv_rho), Lam, K)
        z2 = drv_mod.soft_elementwise(s_new + state["u2"], inv_rho if z2_tau_from_rho else eta_over_rho)
        new = {"l": l_new, "s": s_new, "z1": z1, "z2": z2,
               "u1": state["u1"] + l_new - z1, "u2": state["u2"] + s_new - z2,
               "u3": state["u3"] + l_new + s_new - (0.0 if u3_keeps_I else I)}
        num = math.sqrt(float(np.sum((l_new - state["l"]) ** 2)))
        den = math.sqrt(float(np.sum(l_new ** 2)))
        return new, {"x": x, "Lambda": Lam, "v": v, "E": (num / den if den > 0 else 0.0)}
    return step


RPCA_MUTATIONS = [
    ("z1 shrinks l instead of l + u1", dict(z1_from_l=True)),
    ("u3 update without -I", dict(u3_keeps_I=True)),
    ("l and s swapped in the least-squares step", dict(swap_ls=True)),
    ("l1 prox threshold 1/rho instead of eta/rho", dict(z2_tau_from_rho=True)),
]


@pytest.mark.parametrize("name,kw", RPCA_MUTATIONS, ids=[m[0] for m in RPCA_MUTATIONS])
def test_rpca_planted_mistake_is_caught(monkeypatch, name, kw):
    assert not _rpca_pins_fail(monkeypatch), "pins must pass on the unmodified oracle"
    with np.errstate(all="ignore"):
        monkeypatch.setattr(drv_mod, "rpca_step", _rpca_step_variant(**kw))
        assert _rpca_pins_fail(monkeypatch), f"planted mistake not detected: {name}"


def _svt_variant(k0_floor=False, step_sign=1.0):
    def svt(m, n, rows, cols, vals, tau, step, iters, K, seed=0, power_iters=100, tol_power=1e-7,
            delta_bound=0.01):
        vals = np.asarray(vals, dtype=np.float64)
        P = np.zeros((m, n))
        P[rows, cols] = vals
        G0 = P.T @ P if m >= n else P @ P.T
        _, mu0, _, _, v = bound_mod.power_bound(G0, seed=seed, max_iter=200, tol=1e-9, delta=delta_bound,
                                                cap=float(np.trace(G0)))
        nrm2 = math.sqrt(max(mu0, 0.0))
        q = tau / (step * nrm2) if nrm2 > 0 else 1.0
        k0 = max(math.floor(q), 1) if k0_floor else math.ceil(q)
        Y = np.zeros((m, n))
        Y[rows, cols] = k0 * step * vals
        X = np.zeros((m, n))
        res = []
        nrm = math.sqrt(float(vals @ vals))
        for _ in range(iters):
            Phi, _ = cpa.gram(Y)
            Lam, _, _, _, v = bound_mod.power_bound(Phi, seed=seed, max_iter=power_iters, tol=tol_power,
                                                    delta=delta_bound, v0=v, cap=float(np.trace(Phi)))
            X = cpa.cpa_shrink(Y, _soft(tau), Lam, K)
            r = vals - X[rows, cols]
            Y[rows, cols] += step_sign * step * r
            res.append(math.sqrt(float(r @ r)) / nrm)
        return X, res, k0
    return svt


def _svt_pins_fail(monkeypatch):
    for f in (drv_pins.test_svt_k0_closed_form, drv_pins.test_svt_k0_defining_inequality,
              drv_pins.test_svt_exact_prox_recovers, drv_pins.test_svt_cpa_recovers):
        try:
            with monkeypatch.context() as mp:
                f(mp) if f is drv_pins.test_svt_exact_prox_recovers else f()
        except (AssertionError, FloatingPointError, np.linalg.LinAlgError, ValueError, OverflowError):
            return True
    return False


SVT_MUTATIONS = [
    ("k0 rounded down", dict(k0_floor=True)),
    ("step sign flipped", dict(step_sign=-1.0)),
]


@pytest.mark.parametrize("name,kw", SVT_MUTATIONS, ids=[m[0] for m in SVT_MUTATIONS])
def test_svt_planted_mistake_is_caught(monkeypatch, name, kw):
    # the unmodified SVT oracle passes its pins (one run here; the pins file runs them too)
    monkeypatch.setattr(drv_mod, "svt_complete", _svt_variant())
    assert not _svt_pins_fail(monkeypatch), "the restated SVT must pass the pins"
    with np.errstate(all="ignore"):
        monkeypatch.setattr(drv_mod, "svt_complete", _svt_variant(**kw))
        assert _svt_pins_fail(monkeypatch), f"planted mistake not detected: {name}"


def test_restated_drivers_equal_the_oracle():
    """The unmutated restatements above compute exactly what the oracle does, so a
    caught mutation is a mistake the pins would catch in the oracle itself."""
    I, _, _ = drv_pins._rpca_instance()
    st = drv_mod.rpca_start(I)
    a, ia = _rpca_step_orig(st, I, 1.0, 0.125, 20)
    b, ib = _rpca_step_variant()(st, I, 1.0, 0.125, 20)
    assert all(np.array_equal(a[k], b[k]) for k in a) and ia["E"] == ib["E"]
    m, n, M, rows, cols, tau, step = drv_pins._svt_instance()
    Xa, ra, ka = _svt_orig(m, n, rows, cols, M[rows, cols], tau, step, 5, 25)
    Xb, rb, kb = _svt_variant()(m, n, rows, cols, M[rows, cols], tau, step, 5, 25)
    assert np.array_equal(Xa, Xb) and ra == rb and ka == kb
