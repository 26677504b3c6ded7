"""Pins for the oracle's texture-inpainting ADMM (Appendix A, eq.
admm_algorithm_inp), each against something fixed independently of its code:
the l-update against a least-squares solve with K written out as a matrix, the
2-D DCT against scipy, the mean projection against the geometry of its affine
set, and the recovery of a low-rank texture's missing block."""
import numpy as np
import pytest
import scipy.fft

import synth
from oracle import drivers, sparsify


def _state(m, n, seed):
    g = np.random.default_rng(seed)
    return {k: g.standard_normal((m, n)) for k in drivers.INPAINT_NAMES}


def test_dct2_is_scipys_orthonormal_2d_dct():
    L = np.random.default_rng(1).standard_normal((7, 5))
    assert np.allclose(drivers.dct2(L), scipy.fft.dctn(L, type=2, norm="ortho"), atol=1e-13)
    assert np.allclose(drivers.idct2(drivers.dct2(L)), L, atol=1e-13)


@pytest.mark.parametrize("with_mean", [True, False])
def test_l_update_is_the_least_squares_solution(with_mean):
    """l = (K^T K)^{-1} K^T (z - u) with K = [Id; Psi; Omega; Id; Omega_bar]
    (the last block only with the mean term) built as a dense matrix; Psi acts on
    row-major vec(L) as kron(D_m, D_n)."""
    m, n = 6, 5
    omega = np.ones((m, n))
    omega[1:4, 2:4] = 0.0
    border = np.zeros((m, n), dtype=bool)
    border[0, :] = True
    st = _state(m, n, 3)
    I = np.random.default_rng(4).random((m, n))
    new, _ = drivers.inpaint_step(st, I, omega, border if with_mean else None, 0.3, 0.1, 6)
    Psi = np.kron(sparsify.dct_matrix(m), sparsify.dct_matrix(n))
    Id = np.eye(m * n)
    blocks = [Id, Psi, np.diag(omega.ravel()), Id] + ([np.diag(1.0 - omega.ravel())] if with_mean else [])
    Kmat = np.vstack(blocks)
    names = ["1", "2", "3", "4"] + (["5"] if with_mean else [])
    rhs = np.concatenate([(st["z" + k] - st["u" + k]).ravel() for k in names])
    l_ls = np.linalg.lstsq(Kmat, rhs, rcond=None)[0]
    assert np.allclose(new["l"].ravel(), l_ls, atol=1e-12)


def test_projections():
    m, n = 12, 10
    I, omega, border, _ = synth.texture(m, n, hole=(3, 8, 2, 6), border=2, seed=7)
    st = _state(m, n, 8)
    new, _ = drivers.inpaint_step(st, I, omega, border, 0.3, 0.1, 6)
    # Pi_I keeps the observed pixels
    assert np.array_equal(new["z3"], omega * I)
    # Pi_D: the nearest point of the box [0, 1]
    y4 = new["l"] + st["u4"]
    assert np.all((new["z4"] >= 0.0) & (new["z4"] <= 1.0))
    assert np.array_equal(new["z4"], np.minimum(np.maximum(y4, 0.0), 1.0))
    # Pi_M: the region's mean equals the surrounding pixels' mean, and the move
    # from y is constant on the region and zero elsewhere (the normal of the set)
    reg = omega == 0.0
    y5 = (1.0 - omega) * new["l"] + st["u5"]
    assert abs(np.mean(new["z5"][reg]) - np.mean(I[border])) <= 1e-12
    d = new["z5"] - y5
    assert np.allclose(d[~reg], 0.0, atol=0.0)
    assert np.ptp(d[reg]) <= 1e-12
    # the duals move by K l - z
    assert np.allclose(new["u3"], st["u3"] + omega * new["l"] - new["z3"])
    assert np.allclose(new["u2"], st["u2"] + drivers.dct2(new["l"]) - new["z2"])


def test_inpainting_recovers_a_low_rank_texture():
    """120 iterations on a 48 x 40 texture with a 12 x 10 hole: E_t falls below
    1e-4 and the hole is recovered to 25% (it starts at 150% from the all-ones
    start)."""
    I, omega, border, L0 = synth.texture(48, 40, seed=5)
    reg = omega == 0.0
    l, E = drivers.inpaint_admm(I, omega, border, 1.0, 0.01, 120, 20)
    err = np.linalg.norm((l - L0)[reg]) / np.linalg.norm(L0[reg])
    assert E[-1] < 1e-4
    assert err < 0.25
