"""Pins for the FP64 oracle: each check compares the oracle with something the
paper or the mathematics fixes independently of the oracle's own code
(closed forms, special cases, brute force, published generator outputs)."""
import math

import numpy as np
import pytest

import synth
from oracle import bound, chebyshev, cpa, drivers, exact, metrics
from oracle.shrinkage import Shrinkage, hard, soft, weighted_const, weighted_fn


class Poly:
    """A response h given as a plain Python function (for polynomial pins)."""

    def __init__(self, f):
        self.f = f

    def h(self, x):
        return self.f(x)

    def __call__(self, x):
        return self.f(x)


# ---- Chebyshev scalar machinery (Sec. II-B) ---------------------------------

def test_cos_form_matches_recurrence():
    th = np.linspace(0.0, math.pi, 97)
    x = np.cos(th)
    for k in range(0, 65):
        # T_k(cos t) = cos(k t): the closed form, not the oracle's own routine
        ref = np.cos(k * th)
        assert np.max(np.abs(chebyshev.cheb_recurrence(k, x) - ref)) < 5e-13
        assert np.max(np.abs(chebyshev.cheb_cos(k, x) - ref)) < 5e-13


def test_node_angles_closed_form():
    K = 7
    th = chebyshev.node_angles(K)
    # nodes are the zeros of T_K
    assert np.max(np.abs(np.cos(K * th))) < 1e-14
    assert th[0] == pytest.approx(math.pi / (2 * K))
    assert th[-1] == pytest.approx(math.pi - math.pi / (2 * K))


def test_coefficients_exact_for_polynomials():
    Lam, K = 7.3, 12
    c = chebyshev.coefficients_shifted(Poly(lambda x: 1.0), Lam, K)
    assert c[0] == pytest.approx(2.0, abs=1e-14) and np.max(np.abs(c[1:])) < 1e-14
    c = chebyshev.coefficients_shifted(Poly(lambda x: x), Lam, K)
    # x = Lam/2 (t + 1) = Lam/2 T_0 + Lam/2 T_1  =>  c_0/2 = Lam/2, c_1 = Lam/2
    assert c[0] == pytest.approx(Lam, abs=1e-13)
    assert c[1] == pytest.approx(Lam / 2, abs=1e-13)
    assert np.max(np.abs(c[2:])) < 1e-13
    c = chebyshev.coefficients_shifted(Poly(lambda x: x * x), Lam, K)
    # t = 2x/Lam - 1, x^2 = Lam^2/4 (t+1)^2 = Lam^2/4 (3/2 + 2 T_1 + T_2/2)
    q = Lam * Lam / 4
    assert c[0] == pytest.approx(3 * q, rel=1e-13)
    assert c[1] == pytest.approx(2 * q, rel=1e-13)
    assert c[2] == pytest.approx(q / 2, rel=1e-13)
    assert np.max(np.abs(c[3:])) < 1e-12
    for j in range(1, K):
        c = chebyshev.coefficients_shifted(
            Poly(lambda x, j=j: math.cos(j * math.acos(max(-1.0, min(1.0, 2 * x / Lam - 1))))), Lam, K)
        e = np.zeros(K)
        e[j] = 1.0
        assert np.max(np.abs(c - e)) < 1e-13
    # T_K vanishes at every node: aliasing to the zero series
    c = chebyshev.coefficients_shifted(
        Poly(lambda x: math.cos(K * math.acos(max(-1.0, min(1.0, 2 * x / Lam - 1))))), Lam, K)
    assert np.max(np.abs(c)) < 1e-13


def test_interpolation_at_nodes():
    for sh in (soft(1.3), hard(0.9), weighted_const(2.0), weighted_fn(1.5, 0.4, 1e-3)):
        for K in (5, 16, 31):
            Lam = 9.0
            c = chebyshev.coefficients_shifted(sh, Lam, K)
            xl = Lam / 2 * (np.cos(chebyshev.node_angles(K)) + 1)
            got = chebyshev.series_shifted(c, Lam, xl)
            ref = np.array([sh.h(x) for x in xl])
            assert np.max(np.abs(got - ref)) < 1e-13


def test_discrete_orthogonality():
    K = 9
    th = chebyshev.node_angles(K)
    for j in range(K):
        for k in range(K):
            s = sum(math.cos(j * t) * math.cos(k * t) for t in th)
            ref = K if j == k == 0 else (K / 2 if j == k else 0.0)
            assert s == pytest.approx(ref, abs=1e-12)


# ---- shrinkage responses (Sec. IV-A) ----------------------------------------

def test_soft_response_is_max_minus_tau():
    sh = soft(2.5)
    for s in [0.0, 0.5, 2.4999, 2.5, 2.5001, 3.0, 100.0]:
        assert sh.g(s) == pytest.approx(max(s - 2.5, 0.0), abs=1e-14)
    assert sh.h(2.5 ** 2) == 0.0  # strict threshold


def test_hard_and_weighted_responses():
    hh = hard(2.0)
    assert hh.g(1.999) == 0.0 and hh.g(2.0) == 0.0 and hh.g(2.001) == pytest.approx(2.001)
    wc = weighted_const(1.5)
    for s in [0.3, 1.5, 1.7, 9.0]:
        assert wc.g(s) == pytest.approx(max(s - 1.5, 0.0), abs=1e-14)
    wf = weighted_fn(w_c=2.0, w_sigma=1.0, w_eps=1e-3)
    s = 3.0
    w = 2.0 / (math.sqrt(s * s - 1.0) + 1e-3)
    assert wf.g(s) == pytest.approx(s - w, rel=1e-14)


# ---- matrix CPA (Sec. III, Algorithm 1) ------------------------------------

def _rotated(m, n, s, seed):
    q1 = synth.random_orthogonal(m, seed)
    q2 = synth.random_orthogonal(n, seed + 1)
    d = np.zeros((m, n))
    d[np.arange(len(s)), np.arange(len(s))] = s
    return q1 @ d @ q2.T, q1, q2


def test_matrix_recurrence_acts_on_eigenvalues():
    d = 12
    q = synth.random_orthogonal(d, 11)
    th = np.linspace(0.1, 3.0, d)
    Lam = 5.0
    # Phi with eigenvalues Lam/2 (cos th + 1): hat B = Q diag(cos th) Q^T
    Phi = (q * (Lam / 2 * (np.cos(th) + 1))) @ q.T
    for j in range(1, 20):
        c = np.zeros(j + 1)
        c[j] = 1.0
        psi = cpa.chebyshev_matrix_sum(Phi, c, Lam)
        ref = (q * np.cos(j * th)) @ q.T
        assert np.max(np.abs(psi - ref)) < 1e-12


def test_matrix_maps_for_polynomial_responses():
    X = synth.dense_lowrank(9, 6, rank=3, noise=0.3, seed=5)
    Lam = 1.05 * np.linalg.eigvalsh(X.T @ X)[-1]
    Y = cpa.cpa_shrink(X, Poly(lambda x: 1.0), Lam, 7)
    assert np.max(np.abs(Y - X)) < 1e-12
    Y = cpa.cpa_shrink(X, Poly(lambda x: x), Lam, 7)
    ref = X @ (X.T @ X)
    assert metrics.rel_fro(Y, ref) < 1e-12
    # left side (m < n)
    Xt = X.T.copy()
    Y = cpa.cpa_shrink(Xt, Poly(lambda x: x), Lam, 4)
    assert metrics.rel_fro(Y, (Xt @ Xt.T) @ Xt) < 1e-12


@pytest.mark.parametrize("shape", [(17, 9), (9, 17), (12, 12), (64, 48)])
@pytest.mark.parametrize("K", [1, 2, 3, 16, 30])
def test_forms_agree(shape, K):
    m, n = shape
    X = synth.dense_lowrank(m, n, rank=4, noise=0.2, seed=m * 100 + n)
    G = X.T @ X if m >= n else X @ X.T
    lmax = np.linalg.eigvalsh(G)[-1]
    Lam = 1.02 * lmax
    for sh in (soft(0.4 * math.sqrt(lmax)), hard(0.3 * math.sqrt(lmax)), weighted_fn(2.0, 0.5, 1e-3)):
        a = cpa.cpa_shrink(X, sh, Lam, K)
        b = cpa.cpa_shrink_yform(X, sh, Lam, K)
        c = cpa.cpa_shrink_spectral(X, sh, Lam, K)
        d = cpa.cpa_shrink_operator(X, sh, Lam, K)
        scale = max(metrics.fro(a), metrics.fro(X) * 1e-3)
        for other in (b, c, d):
            assert metrics.fro(a - other) / scale < 1e-10


def test_diagonal_and_rotated_inputs():
    s = np.array([9.0, 5.5, 3.0, 1.2, 0.4])
    sh = soft(2.0)
    Lam, K = 1.01 * 81.0, 20
    c = chebyshev.coefficients_shifted(sh, Lam, K)
    # closed form of the CPA on one singular value: s * hat h(s^2)
    scal = s * chebyshev.series_shifted(c, Lam, s * s)
    D = np.zeros((7, 5))
    D[np.arange(5), np.arange(5)] = s
    Y = cpa.cpa_shrink(D, sh, Lam, K)
    ref = np.zeros((7, 5))
    ref[np.arange(5), np.arange(5)] = scal
    assert np.max(np.abs(Y - ref)) < 1e-12
    Ye = exact.svt_svd(D, sh)
    ref_e = np.zeros((7, 5))
    ref_e[np.arange(5), np.arange(5)] = np.maximum(s - 2.0, 0.0)
    assert np.max(np.abs(Ye - ref_e)) < 1e-13
    X, q1, q2 = _rotated(7, 5, s, 21)
    assert metrics.rel_fro(cpa.cpa_shrink(X, sh, Lam, K), q1 @ ref @ q2.T) < 1e-12
    assert metrics.rel_fro(exact.svt_svd(X, sh), q1 @ ref_e @ q2.T) < 1e-12
    assert metrics.rel_fro(exact.svt_evd(X, sh), q1 @ ref_e @ q2.T) < 1e-10


@pytest.mark.parametrize("nblocks", [10, 100, 200, 500])
def test_block_matrix_D_closed_form(nblocks):
    """D of Sec. V-F: J - blkdiag(0.5 J_b). With u = 1/sqrt(N) and P the block
    averaging projector, D = (N - b/2) u u^T - (b/2)(P - u u^T): singular values
    N - b/2 (once) and b/2 (nblocks - 1 times), the rest zero."""
    N = 1000
    b = N // nblocks
    D = synth.block_matrix_D(N, nblocks)
    s1, s2 = N - b / 2.0, b / 2.0
    sv = np.linalg.svd(D, compute_uv=False)
    assert sv[0] == pytest.approx(s1, rel=1e-12)
    assert np.max(np.abs(sv[1:nblocks] - s2)) < 1e-9
    assert np.max(np.abs(sv[nblocks:])) < 1e-9
    tau = 0.3 * s2
    sh = soft(tau)
    u = np.full((N, 1), 1.0 / math.sqrt(N))
    P = np.zeros((N, N))
    for i in range(nblocks):
        P[i * b:(i + 1) * b, i * b:(i + 1) * b] = 1.0 / b
    uu = u @ u.T
    ref = max(s1 - tau, 0) * uu - max(s2 - tau, 0) * (P - uu)
    assert metrics.rel_fro(exact.svt_svd(D, sh), ref) < 1e-10
    if nblocks == 10:
        Lam, K = 1.01 * s1 * s1, 20
        Y = cpa.cpa_shrink(D, sh, Lam, K)
        c = chebyshev.coefficients_shifted(sh, Lam, K)
        a1 = s1 * chebyshev.series_shifted(c, Lam, s1 * s1)
        a2 = s2 * chebyshev.series_shifted(c, Lam, s2 * s2)
        ref_cpa = a1 * uu - a2 * (P - uu)
        assert metrics.rel_fro(Y, ref_cpa) < 1e-10


def test_brute_force_4x3():
    g = synth.rng(77)
    for trial in range(10):
        X = g.standard_normal((4, 3))
        G = X.T @ X
        lam = exact.eig3_sym(G)
        assert np.max(np.abs(lam - np.linalg.eigvalsh(G))) < 1e-10 * lam[-1]
        V = np.stack([exact.null_vector3(G - l * np.eye(3)) for l in lam], axis=1)
        sh = soft(0.8 * math.sqrt(lam[1]))
        hh = np.array([sh.h(l) for l in lam])
        ref = X @ (V * hh) @ V.T
        assert metrics.rel_fro(exact.svt_svd(X, sh), ref) < 1e-9
        assert metrics.rel_fro(exact.svt_evd(X, sh), ref) < 1e-9
        # CPA: the same eigenpairs with the interpolant in place of h
        Lam, K = 1.01 * lam[-1], 12
        c = chebyshev.coefficients_shifted(sh, Lam, K)
        hc = chebyshev.series_shifted(c, Lam, lam)
        assert metrics.rel_fro(cpa.cpa_shrink(X, sh, Lam, K), X @ (V * hc) @ V.T) < 1e-9


def test_invariances():
    X = synth.dense_lowrank(20, 13, rank=4, noise=0.2, seed=3)
    lmax = np.linalg.eigvalsh(X.T @ X)[-1]
    Lam, K = 1.03 * lmax, 18
    tau = 0.35 * math.sqrt(lmax)
    Y = cpa.cpa_shrink(X, soft(tau), Lam, K)
    # homogeneity: shrink_{c tau}(c X) with Lambda c^2 = c shrink_tau(X)
    cc = 3.7
    Y2 = cpa.cpa_shrink(cc * X, soft(cc * tau), Lam * cc * cc, K)
    assert metrics.rel_fro(Y2, cc * Y) < 1e-12
    # transpose
    Yt = cpa.cpa_shrink(X.T.copy(), soft(tau), Lam, K)
    assert metrics.rel_fro(Yt, Y.T) < 1e-12
    # orthogonal equivariance
    q1 = synth.random_orthogonal(20, 8)
    q2 = synth.random_orthogonal(13, 9)
    Yr = cpa.cpa_shrink(q1 @ X @ q2, soft(tau), Lam, K)
    assert metrics.rel_fro(Yr, q1 @ Y @ q2) < 1e-11
    # contraction: ||Y_k||_F <= ||X||_F for Lambda >= lambda_max
    Phi = X.T @ X
    for j in range(1, K):
        c = np.zeros(j + 1)
        c[j] = 1.0
        Yj = X @ cpa.chebyshev_matrix_sum(Phi, c, Lam)
        assert metrics.fro(Yj) <= metrics.fro(X) * (1 + 1e-12)


def test_error_vs_order_envelope_and_scalar_formula():
    X = synth.dense_lowrank()  # 64 x 48, rank 5 + noise 0.1
    s = np.linalg.svd(X, compute_uv=False)
    sh = soft(0.5 * s[0])
    Lam = 1.01 * s[0] ** 2
    Ye = exact.svt_svd(X, sh)
    errs = {}
    for K in (5, 10, 20, 40, 80):
        Y = cpa.cpa_shrink(X, sh, Lam, K)
        e = metrics.rel_fro(Y, Ye)
        _, e2 = exact.cpa_error_from_spectrum(s, sh, Lam, K)
        assert e == pytest.approx(e2, rel=1e-8)
        errs[K] = e
    Ks = sorted(errs)
    env = [max(errs[k] for k in Ks if k >= K) for K in Ks]
    assert all(env[i] >= env[i + 1] for i in range(len(env) - 1))
    assert errs[80] < errs[5] / 10


def test_special_cases():
    X = synth.dense_lowrank(10, 7, rank=3, noise=0.1, seed=4)
    lmax = np.linalg.eigvalsh(X.T @ X)[-1]
    Lam = 1.01 * lmax
    assert np.max(np.abs(cpa.cpa_shrink(X, soft(0.0), Lam, 9) - X)) < 1e-12
    assert np.all(cpa.cpa_shrink(X, soft(math.sqrt(Lam)), Lam, 9) == 0.0)
    assert np.all(cpa.cpa_shrink(np.zeros((5, 4)), soft(1.0), 0.0, 9) == 0.0)
    c = chebyshev.coefficients_shifted(soft(0.3 * math.sqrt(lmax)), Lam, 1)
    Y1 = cpa.cpa_shrink(X, soft(0.3 * math.sqrt(lmax)), Lam, 1)
    assert np.max(np.abs(Y1 - 0.5 * c[0] * X)) < 1e-14
    assert cpa.cpa_shrink(np.zeros((0, 4)), soft(1.0), 1.0, 3).shape == (0, 4)
    with pytest.raises(ValueError):
        cpa.cpa_shrink(X, soft(1.0), Lam, 0)


# ---- spectral bound ----------------------------------------------------------

def test_splitmix64_published_outputs():
    # first outputs of the reference SplitMix64 generator seeded with 0
    assert bound.splitmix64(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF
    assert bound.splitmix64((2 * 0x9E3779B97F4A7C15) & ((1 << 64) - 1)) == 0x6E789E6AA1B965F4
    assert bound.splitmix64((3 * 0x9E3779B97F4A7C15) & ((1 << 64) - 1)) == 0x06C45D188009454F


def test_power_bound_is_an_upper_bound():
    for seed in range(6):
        X = synth.dense_lowrank(40, 25, rank=5, noise=0.3, seed=100 + seed)
        G = X.T @ X
        lam = np.linalg.eigvalsh(G)
        Lam, mu, r, it, v = bound.power_bound(G, seed=seed)
        assert Lam >= lam[-1] * (1 - 1e-12)
        assert mu <= lam[-1] * (1 + 1e-12)
        assert Lam <= 1.01 * math.sqrt(float(np.sum(G * G))) * (1 + 1e-15)
        assert abs(mu - lam[-1]) < 1e-6 * lam[-1]
    Dg = np.diag([4.0, 1.0, 0.5, 0.25])
    Lam, mu, r, it, v = bound.power_bound(Dg, seed=1)
    assert mu == pytest.approx(4.0, rel=1e-7)
    assert Lam == pytest.approx(4.04, rel=1e-6)
    # rank one: ||G||_F == lambda_max, the cap keeps the margin
    u = np.array([[1.0], [2.0], [2.0]])
    Lam1 = bound.power_bound(u @ u.T, seed=3)[0]
    assert Lam1 == pytest.approx(9.0 * 1.01, rel=1e-9)
    assert bound.power_bound(np.zeros((3, 3)))[0] == 0.0


# ---- drivers (Appendix B) ----------------------------------------------------

def test_admm_lsolve_closed_form():
    g = synth.rng(5)
    z1, z2, z3, u1, u2, u3 = (g.standard_normal((4, 3)) for _ in range(6))
    l, s = drivers.admm_lsolve(z1, z2, z3, u1, u2, u3)
    # l' minimises ||K l' - (z - u)||^2: normal equations K^T K l' = K^T (z - u)
    r1, r2, r3 = z1 - u1, z2 - u2, z3 - u3
    assert np.max(np.abs((2 * l + s) - (r1 + r3))) < 1e-13
    assert np.max(np.abs((l + 2 * s) - (r2 + r3))) < 1e-13


def test_l1_prox_closed_form():
    x = np.array([-3.0, -0.5, 0.0, 0.2, 0.7, 5.0])
    t = 0.6
    ref = np.array([-2.4, 0.0, 0.0, 0.0, 0.1, 4.4])
    assert np.max(np.abs(drivers.soft_elementwise(x, t) - ref)) < 1e-15
    # the prox minimises t|y| + (y-x)^2/2: brute force on a fine grid
    ys = np.linspace(-6, 6, 120001)
    for xi in x:
        obj = t * np.abs(ys) + 0.5 * (ys - xi) ** 2
        assert ys[np.argmin(obj)] == pytest.approx(drivers.soft_elementwise(xi, t), abs=2e-4)


def test_rpca_admm_converges_on_small_input():
    I, L0, S0 = synth.rpca_frames(64, 64, rank=3, outlier_frac=0.05, seed=9)
    l, s, E, lams = drivers.rpca_admm(I.astype(np.float64), inv_rho=1.0, eta_over_rho=1.0 / 8,
                                      iters=40, K=30)
    assert E[-1] < E[2]
    assert E[-1] < 2e-2
    assert all(x > 0 for x in lams)


def test_rows_yform_matches_full():
    X = synth.dense_lowrank(40, 12, rank=3, noise=0.2, seed=31)
    Phi = X.T @ X
    Lam = 1.02 * np.linalg.eigvalsh(Phi)[-1]
    sh = soft(0.3 * math.sqrt(Lam))
    full = cpa.cpa_shrink(X, sh, Lam, 17)
    rows = [0, 5, 39]
    assert np.max(np.abs(cpa.cpa_rows_yform(Phi, X[rows], sh, Lam, 17) - full[rows])) < 1e-11


def test_power_bound_trace_cap():
    X = synth.dense_lowrank(30, 10, rank=1, noise=0.0, seed=32)
    Phi = X.T @ X
    lam, mu, _, _, _ = bound.power_bound(Phi, cap=float(np.trace(Phi)))
    # rank one: trace == lambda_max, so the trace cap still keeps the margin
    assert lam == pytest.approx(1.01 * np.trace(Phi), rel=1e-9)


def test_svt_reduces_residual():
    g = synth.rng(40)
    m, n, r = 60, 30, 2
    M = g.standard_normal((m, r)) @ g.standard_normal((r, n))
    idx = np.sort(g.choice(m * n, size=900, replace=False))
    rows, cols = idx // n, idx % n
    tau, step = 5 * math.sqrt(m * n), 1.2 * m * n / len(idx)
    X, res, k0 = drivers.svt_complete(m, n, rows, cols, M[rows, cols], tau, step, 30, 25)
    assert k0 >= 1 and res[-1] < res[0]
