"""Pins for the oracle's k-step Lanczos bound (the maximum-eigenvalue step of
Algorithm 1, read as a Lanczos run), against closed forms and facts of the
symmetric eigenproblem, not against the oracle's own algebra."""
import math

import numpy as np
import pytest

from oracle import bound


def _toeplitz(d):
    return 2.0 * np.eye(d) - np.eye(d, k=1) - np.eye(d, k=-1)


@pytest.mark.parametrize("k", [1, 2, 5, 9])
def test_toeplitz_from_e1_has_closed_forms(k):
    """From e_1 the Krylov vectors of the [-1, 2, -1] matrix are e_1, e_2, ...: the
    recurrence returns alpha = 2, beta = 1 and T_k is the matrix's leading block,
    whose largest eigenvalue is 2 + 2 cos(pi / (k + 1)); the top eigenvector's last
    component is sqrt(2 / (k + 1)) sin(pi / (k + 1)), and beta_k = 1 (d > k)."""
    d = 20
    e1 = np.zeros(d)
    e1[0] = 1.0
    Lam, theta, r, m, y, a, b = bound.lanczos_bound(_toeplitz(d), steps=k, v0=e1, delta=0.0)
    assert m == k
    assert np.max(np.abs(a - 2.0)) < 1e-14
    assert np.max(np.abs(b - 1.0)) < 1e-14
    assert abs(theta - (2.0 + 2.0 * math.cos(math.pi / (k + 1)))) < 1e-13
    assert abs(r - math.sqrt(2.0 / (k + 1)) * math.sin(math.pi / (k + 1))) < 1e-13
    # the Ritz vector lives on the first k coordinates: sin(i j pi / (k + 1)) up to sign
    j = np.arange(1, k + 1)
    ref = np.sin(j * k * math.pi / (k + 1)) * math.sqrt(2.0 / (k + 1))
    assert min(np.max(np.abs(y[:k] - ref)), np.max(np.abs(y[:k] + ref))) < 1e-12
    assert np.max(np.abs(y[k:])) == 0.0


def test_one_step_is_one_power_product():
    """theta_1 = q.Phi q = mu_1 and beta_1 = ||Phi q - mu q|| = the power residual,
    so one Lanczos step gives the power iteration's one-product bound."""
    g = np.random.default_rng(5)
    A = g.standard_normal((40, 25))
    G = A.T @ A
    for seed in (0, 3):
        Ll, th, r, m, *_ = bound.lanczos_bound(G, seed=seed, steps=1)
        Lp, mu, rp, it, _ = bound.power_bound(G, seed=seed, max_iter=1)
        assert m == 1 and it == 1
        assert abs(th - mu) <= 1e-13 * mu and abs(r - rp) <= 1e-9 * mu and abs(Ll - Lp) <= 1e-12 * Lp


def test_as_many_steps_as_distinct_eigenvalues():
    """The Krylov space of a matrix with three distinct eigenvalues has dimension
    three: three steps find the largest exactly, and beta_3 vanishes (up to
    rounding)."""
    g = np.random.default_rng(8)
    Qm, _ = np.linalg.qr(g.standard_normal((30, 30)))
    lam = np.repeat([0.5, 2.0, 7.25], 10)
    Phi = (Qm * lam) @ Qm.T
    Lam, theta, r, m, y, a, b = bound.lanczos_bound(Phi, seed=2, steps=3, delta=0.0)
    assert abs(theta - 7.25) < 1e-12
    assert r < 1e-10
    assert abs(b[2]) < 1e-10


@pytest.mark.parametrize("seed", [0, 1, 4])
def test_ritz_value_and_residual_on_seeded_grams(seed):
    """theta <= lambda_max (Cauchy interlacing: T_k is a compression of Phi); the
    Ritz pair's residual ||Phi y - theta y|| equals beta_k |s_k|, and some
    eigenvalue lies within it of theta (Krylov-Weinstein) -- after a few steps
    not necessarily the largest, after enough steps the largest, and then the
    bound covers lambda_max."""
    g = np.random.default_rng(100 + seed)
    A = g.standard_normal((90, 60)) @ np.diag(np.linspace(3.0, 0.1, 60))
    G = A.T @ A
    ev = np.linalg.eigvalsh(G)
    lmax = float(ev[-1])
    for k in (3, 6, 12, 30):
        Lam, theta, r, m, y, a, b = bound.lanczos_bound(G, seed=seed, steps=k)
        assert theta <= lmax * (1 + 1e-14)
        assert abs(np.linalg.norm(y) - 1.0) < 1e-10
        assert abs(np.linalg.norm(G @ y - theta * y) - r) <= 1e-9 * lmax
        assert float(np.min(np.abs(ev - theta))) <= r * (1 + 1e-9) + 1e-12 * lmax
        if k >= 12:
            assert lmax - theta <= r * (1 + 1e-9)
            assert Lam >= lmax
    # converged: theta matches eigh far past the power iteration's reach in as many products
    Lam, theta, r, m, *_ = bound.lanczos_bound(G, seed=seed, steps=30, delta=0.0)
    assert abs(theta - lmax) <= 1e-12 * lmax


def test_degenerate_inputs():
    Z = np.zeros((6, 6))
    assert bound.lanczos_bound(Z)[0] == 0.0
    # a first product that vanishes while ||Phi||_F > 0: the Frobenius norm
    P = np.zeros((4, 4))
    P[3, 3] = 5.0
    e1 = np.array([1.0, 0.0, 0.0, 0.0])
    Lam, theta, r, m, *_ = bound.lanczos_bound(P, v0=e1)
    assert Lam == 5.0 and m == 1
    # the 1 x 1 matrix: theta is its entry after one step, the residual zero
    Lam, theta, r, m, *_ = bound.lanczos_bound(np.array([[3.0]]), steps=5, delta=0.0)
    assert m == 1 and theta == 3.0 and r == 0.0


def test_early_stop_matches_a_fixed_run():
    """With tol > 0 the run stops at the first step j >= 2 whose Ritz value moved
    by at most tol theta_j: a fixed run of that many steps gives the same bound,
    the Ritz values of the fixed runs of j - 1 and j steps meet the test, and
    those of every earlier pair of consecutive steps do not."""
    g = np.random.default_rng(21)
    A = g.standard_normal((80, 50)) @ np.diag(np.linspace(2.0, 0.2, 50))
    G = A.T @ A
    tol = 1e-7
    L, th, r, m, *_ = bound.lanczos_bound(G, seed=1, steps=32, tol=tol)
    assert 2 <= m < 32
    Lf, thf, rf, mf, *_ = bound.lanczos_bound(G, seed=1, steps=m)
    assert mf == m and Lf == L and thf == th and rf == r
    ths = [bound.lanczos_bound(G, seed=1, steps=j)[1] for j in range(1, m + 1)]
    assert abs(ths[-1] - ths[-2]) <= tol * ths[-1]
    for j in range(1, m - 1):
        assert abs(ths[j] - ths[j - 1]) > tol * ths[j]
