"""Pins for the oracle's sparsified Algorithm 1 (transform T, truncation eps):
each check compares it with something fixed independently of its own code --
scipy's DCT, the T = Id shrinkage (an orthogonal similarity leaves the result
unchanged), an eigendecomposition of the truncated matrix, a full sort."""
import math

import numpy as np
import pytest
import scipy.fft

import synth
from oracle import chebyshev, cpa, sparsify
from oracle.shrinkage import Shrinkage


@pytest.mark.parametrize("n", [1, 2, 8, 16, 40])
def test_dct_matrix_is_scipys_orthonormal_dct2(n):
    D = sparsify.dct_matrix(n)
    ref = scipy.fft.dct(np.eye(n), type=2, norm="ortho", axis=0)
    assert np.allclose(D, ref, atol=1e-14)
    assert np.allclose(D @ D.T, np.eye(n), atol=1e-13)


def test_block_dct_transforms_each_block():
    n = 48
    T = sparsify.block_dct(n, 8)
    x = np.random.default_rng(3).standard_normal(n)
    ref = np.concatenate([scipy.fft.dct(x[i:i + 8], type=2, norm="ortho") for i in range(0, n, 8)])
    assert np.allclose(T @ x, ref, atol=1e-13)
    assert np.allclose(T @ T.T, np.eye(n), atol=1e-13)
    with pytest.raises(ValueError):
        sparsify.block_dct(20, 8)


def test_kth_largest_matches_a_full_sort():
    A = np.random.default_rng(4).standard_normal((13, 11))
    s = np.sort(np.abs(A).ravel())[::-1]
    for k in (1, 2, 7, 50, A.size):
        assert sparsify.kth_largest_abs(A, k) == s[k - 1]
    assert sparsify.keep_count(1000, 0.5e-4) == 50
    assert sparsify.keep_count(10, 1e-9) == 1


@pytest.mark.parametrize("shape", [(40, 24), (24, 40)])
@pytest.mark.parametrize("which", ["dct", "block"])
def test_without_truncation_any_orthogonal_transform_gives_the_plain_shrinkage(shape, which):
    m, n = shape
    B = synth.dense_lowrank(m, n, rank=4, noise=0.1, seed=5 + m)
    d = min(m, n)
    T = sparsify.dct_matrix(d) if which == "dct" else sparsify.block_dct(d, 8)
    G = B.T @ B if m >= n else B @ B.T
    lam = 1.01 * float(np.linalg.eigvalsh(G)[-1])
    sh = Shrinkage(0, 0.3 * math.sqrt(lam))
    Y, eps, nnz = sparsify.cpa_shrink_sparsified(B, sh, lam, 12, T, d * d)
    ref = cpa.cpa_shrink(B, sh, lam, 12)
    assert nnz == d * d
    assert np.abs(Y - ref).max() <= 1e-10 * np.abs(ref).max()


def _spectral_reference(B, T, k, sh, K):
    """The same result from an eigendecomposition of the truncated matrix:
    B T^T V diag(hat h(lambda)) V^T T (right side), hat h evaluated by the scalar
    recurrence at 2 lambda / Lambda - 1."""
    m, n = B.shape
    G = B.T @ B if m >= n else B @ B.T
    Phi = T @ G @ T.T
    Phi = 0.5 * (Phi + Phi.T)
    a = np.sort(np.abs(Phi).ravel())[::-1]
    eps = a[k - 1]
    Phil = np.where(np.abs(Phi) >= eps, Phi, 0.0)
    lam, V = np.linalg.eigh(Phil)
    Lam = 1.01 * float(lam[-1])
    c = chebyshev.coefficients_shifted(sh, Lam, K)
    x = 2.0 * lam / Lam - 1.0
    hh = 0.5 * c[0] + sum(c[j] * chebyshev.cheb_recurrence(j, x) for j in range(1, K))
    M = T.T @ (V * hh) @ V.T @ T
    return (B @ M if m >= n else M @ B), Lam, eps, int(np.count_nonzero(np.abs(Phi) >= eps))


@pytest.mark.parametrize("shape", [(64, 32), (32, 64)])
@pytest.mark.parametrize("frac", [0.02, 0.1, 0.4])
def test_truncated_shrinkage_matches_spectral_form(shape, frac):
    m, n = shape
    B = synth.block_smooth(m, n, rank=3, noise=1e-3, seed=17 + m)
    d = min(m, n)
    T = sparsify.block_dct(d, 8)
    k = sparsify.keep_count(d, frac)
    sh = Shrinkage(3, 0.0, 2.0, 0.5, 1e-3)
    ref, Lam, eps_ref, nnz_ref = _spectral_reference(B, T, k, sh, 16)
    Y, eps, nnz = sparsify.cpa_shrink_sparsified(B, sh, Lam, 16, T, k)
    # Phi is symmetric: the k-th value's mirror entry ties with it and is kept too
    assert eps == eps_ref and nnz == nnz_ref and k <= nnz <= k + 1
    # the truncated spectrum stays (up to the dropped noise) inside [0, Lambda]
    G = B.T @ B if m >= n else B @ B.T
    Phil = sparsify.truncate(0.5 * (T @ G @ T.T + (T @ G @ T.T).T), eps)
    assert np.array_equal(Phil, Phil.T)
    lam = np.linalg.eigvalsh(Phil)
    assert lam[0] >= -1e-3 * lam[-1]
    assert np.abs(Y - ref).max() <= 1e-9 * np.abs(ref).max()


def test_transform_order_matters_under_truncation():
    """With truncation the result depends on applying T (not T^T) to the Gram:
    swapping them changes it, so the pins above see that order."""
    B = synth.dense_lowrank(64, 32, rank=3, noise=0.05, seed=99)
    T = sparsify.dct_matrix(32)
    k = sparsify.keep_count(32, 0.05)
    G = B.T @ B
    Lam = 1.01 * float(np.linalg.eigvalsh(G)[-1])
    sh = Shrinkage(0, 0.2 * math.sqrt(Lam))
    Y1, _, _ = sparsify.cpa_shrink_sparsified(B, sh, Lam, 10, T, k)
    Y2, _, _ = sparsify.cpa_shrink_sparsified(B, sh, Lam, 10, T.T.copy(), k)
    assert np.abs(Y1 - Y2).max() > 1e-3 * np.abs(Y1).max()


def test_haar_matrix_sums_and_differences():
    r = math.sqrt(0.5)
    H = sparsify.haar_matrix(4)
    assert np.allclose(H @ np.array([1.0, 2.0, 3.0, 5.0]), [3 * r, 8 * r, -1 * r, -2 * r], atol=1e-15)
    for n in (2, 8, 40):
        Hn = sparsify.haar_matrix(n)
        assert np.allclose(Hn @ Hn.T, np.eye(n), atol=1e-15)
    with pytest.raises(ValueError):
        sparsify.haar_matrix(7)


def _cheb_scalar(sh, Lam, K, lam):
    c = chebyshev.coefficients_shifted(sh, Lam, K)
    x = 2.0 * np.asarray(lam, dtype=np.float64) / Lam - 1.0
    return 0.5 * c[0] + sum(c[j] * chebyshev.cheb_recurrence(j, x) for j in range(1, K))


@pytest.mark.parametrize("shape", [(64, 32), (32, 64)])
@pytest.mark.parametrize("frac", [0.05, 0.25])
def test_lowpass_haar_equals_the_low_block_spectral_form(shape, frac):
    """High frequencies set to zero: the truncated matrix lives on the low-pass
    block, so hat G = B T_L^T V hat h(lambda) V^T T_L + hat h(0) B T_H^T T_H with
    V, lambda from an eigendecomposition of the truncated low-pass block."""
    m, n = shape
    B = synth.block_smooth(m, n, rank=3, noise=1e-3, seed=41 + m)
    d = min(m, n)
    T = sparsify.haar_matrix(d)
    TL, TH = T[: d // 2], T[d // 2:]
    G = B.T @ B if m >= n else B @ B.T
    PL = TL @ G @ TL.T
    PL = 0.5 * (PL + PL.T)
    k = sparsify.keep_count(d // 2, frac)
    eps = np.sort(np.abs(PL).ravel())[::-1][k - 1]
    lam, V = np.linalg.eigh(np.where(np.abs(PL) >= eps, PL, 0.0))
    Lam = 1.01 * float(lam[-1])
    sh = Shrinkage(0, 0.2 * math.sqrt(Lam))
    K = 14
    M = TL.T @ (V * _cheb_scalar(sh, Lam, K, lam)) @ V.T @ TL + _cheb_scalar(sh, Lam, K, [0.0])[0] * (TH.T @ TH)
    ref = B @ M if m >= n else M @ B
    zero = np.arange(d) >= d // 2
    Y, eps_o, nnz = sparsify.cpa_shrink_sparsified(B, sh, Lam, K, T, k, zero=zero)
    assert eps_o == eps
    assert np.abs(Y - ref).max() <= 1e-9 * np.abs(ref).max()


def test_block_ordered_haar_gives_the_same_result():
    """kron(I, haar_matrix(8)) is a row permutation of haar_matrix(n) (the low-pass
    rows of each 8-block first); the result, eps and the kept count do not change,
    with or without the high frequencies zeroed."""
    B = synth.block_smooth(96, 48, rank=3, noise=1e-3, seed=55)
    d = 48
    Tg = sparsify.haar_matrix(d)
    Tb = np.kron(np.eye(d // 8), sparsify.haar_matrix(8))
    # the two have the same rows
    assert sorted(map(tuple, np.round(Tg, 12))) == sorted(map(tuple, np.round(Tb, 12)))
    G = B.T @ B
    Lam = 1.01 * float(np.linalg.eigvalsh(G)[-1])
    sh = Shrinkage(0, 0.2 * math.sqrt(Lam))
    k = sparsify.keep_count(d, 0.05)
    for zg, zb in ((None, None), (np.arange(d) >= d // 2, np.arange(d) % 8 >= 4)):
        Y1, e1, n1 = sparsify.cpa_shrink_sparsified(B, sh, Lam, 12, Tg, k, zero=zg)
        Y2, e2, n2 = sparsify.cpa_shrink_sparsified(B, sh, Lam, 12, Tb, k, zero=zb)
        assert n1 == n2 and abs(e1 - e2) <= 1e-12 * e1
        assert np.abs(Y1 - Y2).max() <= 1e-10 * np.abs(Y1).max()


def _schedule_fixture():
    """The fractions and switch points printed in eq. (recommendation_epsilon) and
    Table IV's caption (tests/golden/keep_schedule.txt), as exact decimals."""
    from decimal import Decimal
    from fractions import Fraction
    from pathlib import Path
    vals = {}
    for line in (Path(__file__).parent / "golden" / "keep_schedule.txt").read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            parts = line.split()
            vals[parts[0]] = Fraction(Decimal(parts[1]))
    return vals


def test_keep_schedule_matches_the_printed_fractions():
    """k = ceil(f n^2) with the printed fraction f of each case, for sizes where the
    product is and is not an integer; the paper's own n = 1000 comparison gives
    k_1, k_2, k_3 = 50, 150, 500."""
    g = _schedule_fixture()
    E_l, E_m = float(g["E_l"]), float(g["E_m"])
    assert (E_l, E_m) == (0.03, 6e-4)
    for n in (8, 96, 141, 256, 1000, 1024, 1920, 4000):
        for E, key in ((math.inf, "k_1"), (1.0, "k_1"), (0.01, "k_2"), (1e-4, "k_3"), (0.0, "k_3")):
            want = max(1, math.ceil(g[key] * n * n))
            assert sparsify.keep_schedule(E, n) == want, (n, E)
    assert [sparsify.keep_schedule(E, 1000) for E in (1.0, 0.01, 1e-4)] == [50, 150, 500]
    assert math.ceil(g["k_4"] * 1000 ** 2) == 1000 ** 2


def test_keep_schedule_case_edges():
    """E_t = E_l falls in the second case and E_t = E_m in the third (the equation's
    inequalities); the count never leaves [1, n^2]."""
    assert sparsify.keep_schedule(0.03, 1000) == 150
    assert sparsify.keep_schedule(math.nextafter(0.03, 1.0), 1000) == 50
    assert sparsify.keep_schedule(6e-4, 1000) == 500
    assert sparsify.keep_schedule(math.nextafter(6e-4, 1.0), 1000) == 150
    assert sparsify.keep_schedule(1.0, 1) == 1 and sparsify.keep_schedule(0.0, 1) == 1
    assert sparsify.keep_schedule(0.0, 44) == 1          # 1936 / 2000 rounds up to 1
    assert sparsify.keep_schedule(0.0, 45) == 2          # 2025 / 2000 rounds up to 2
    with pytest.raises(ValueError):
        sparsify.keep_schedule(math.nan, 8)


def test_inpaint_step_without_truncation_is_the_plain_step():
    """With every component kept (k = n^2, Table IV's k_4) the sparsified z1 of the
    inpainting step is the plain shrink (an orthogonal similarity), for the DCT
    and the block DCT; with a keep count below n^2 it differs."""
    from oracle import drivers
    import synth
    I, om, bd, _ = synth.texture(48, 40, border=4, seed=5)
    st = drivers.inpaint_start(om)
    st, _ = drivers.inpaint_step(st, I, om, bd, 1.0, 0.01, 15)
    ref, info = drivers.inpaint_step(st, I, om, bd, 1.0, 0.01, 15, power_iters=300, tol_power=1e-12)
    for T in (sparsify.dct_matrix(40), sparsify.block_dct(40, 8)):
        sp, info_s = drivers.inpaint_step(st, I, om, bd, 1.0, 0.01, 15, power_iters=300, tol_power=1e-12,
                                          sparsify={"T": T, "keep": 40 * 40})
        for k in ("l", "z1", "u1", "z2", "z5"):
            assert np.linalg.norm(sp[k] - ref[k]) <= 1e-9 * max(np.linalg.norm(ref[k]), 1.0), k
        assert abs(info_s["E"] - info["E"]) <= 1e-12
        cut, _ = drivers.inpaint_step(st, I, om, bd, 1.0, 0.01, 15, sparsify={"T": T, "keep": 4})
        assert np.linalg.norm(cut["z1"] - ref["z1"]) > 1e-3 * np.linalg.norm(ref["z1"])


def test_scheduled_inpaint_uses_the_previous_change():
    """The scheduled ADMM takes iteration t's keep from E_{t-1} (E_prev first)."""
    from oracle import drivers
    import synth
    I, om, bd, _ = synth.texture(64, 64, border=4, seed=5)
    st, E, keeps = drivers.inpaint_admm(I, om, bd, 1.0, 0.01, 8, 15,
                                        schedule={"T": sparsify.dct_matrix(64), "E_l": 0.7, "E_m": 0.3,
                                                  "E_prev": 0.3})
    want = [sparsify.keep_schedule(e, 64, 0.7, 0.3) for e in [0.3] + E[:-1]]
    assert keeps == want
    assert len(set(keeps)) >= 2


def test_given_threshold():
    """eq. (threshold_components) with eps given: eps = K(|Phi|, k) gives the keep-k
    result; eps = 0 keeps every component (the T = Id shrinkage, an orthogonal
    similarity); an eps above every |Phi_ij| keeps nothing (zero matrix, zero bound,
    zero result)."""
    from oracle.shrinkage import Shrinkage
    rng = np.random.default_rng(4)
    B = rng.standard_normal((40, 24)) @ np.diag(np.linspace(3.0, 0.2, 24))
    T = sparsify.block_dct(24, 8)
    Phi, _ = sparsify.transformed_gram(B, T)
    sh = Shrinkage(0, 1.5)
    for k in (5, 40, 200):
        e = sparsify.kth_largest_abs(Phi, k)
        Lam = 1.01 * float(np.linalg.eigvalsh(sparsify.truncate(Phi, e))[-1])
        a = sparsify.cpa_shrink_sparsified(B, sh, Lam, 20, T, k)
        b = sparsify.cpa_shrink_sparsified(B, sh, Lam, 20, T, None, eps=e)
        assert np.array_equal(a[0], b[0]) and a[2] == b[2]
    Lam = 1.01 * float(np.linalg.eigvalsh(Phi)[-1])
    full, _, nnz = sparsify.cpa_shrink_sparsified(B, sh, Lam, 20, T, None, eps=0.0)
    plain = cpa.cpa_shrink(B, sh, Lam, 20)
    assert nnz == 24 * 24
    assert np.linalg.norm(full - plain) <= 1e-10 * np.linalg.norm(plain)
    top = float(np.abs(Phi).max())
    Phil = sparsify.truncate(Phi, 2.0 * top)
    assert not Phil.any()
    for lam in (0.0, Lam):   # zero whatever the bound: h(0) = 0
        zero, _, nnz = sparsify.cpa_shrink_sparsified(B, sh, lam, 20, T, None, eps=2.0 * top)
        assert nnz == 0 and not zero.any()
