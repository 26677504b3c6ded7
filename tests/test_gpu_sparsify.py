"""Sparsified shrinkage (Algorithm 1 with the 8 x 8 block DCT or the identity and
component truncation) against the FP64 oracle.  The keep counts sit at a clear
gap in |Phi| (the kept and the first dropped magnitude differ by more than 2%),
so the truncation keeps the same entries in the kernel's FP32 and the oracle's
FP64; the threshold and the kept count are compared, then the result."""
import math

import numpy as np
import pytest

import synth
from tests import parity
from oracle import bound as obound
from oracle import cpa as ocpa
from oracle import metrics, sparsify
from oracle.shrinkage import Shrinkage

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def _lib():
    import paper_1705_07112_amd as cpa
    return cpa


def _gap_keep(Phi, frac):
    """A keep count near frac * d^2 at a gap of more than 2% in the sorted |Phi|."""
    a = np.sort(np.abs(Phi).ravel())[::-1]
    target = max(1, int(frac * a.size))
    ratio = a[:-1] / np.maximum(a[1:], 1e-300)
    cand = np.nonzero(ratio > 1.02)[0]
    j = cand[np.argmin(np.abs(cand + 1 - target))]
    return int(j + 1)


def _case(X, T, transform, frac, K, sh_o, sh_c, side_right=True, ev="auto", zero=None, keep=None, eps_tol=1e-6):
    import torch
    cpa = _lib()
    m, n = X.shape
    Phi, _ = sparsify.transformed_gram(X, T)
    if zero is not None:
        Phi[zero, :] = 0.0
        Phi[:, zero] = 0.0
    if keep is None:
        keep = _gap_keep(Phi, frac) if frac < 1.0 else Phi.size
    eps_o = sparsify.kth_largest_abs(Phi, keep)
    Phil = sparsify.truncate(Phi, eps_o)
    lam = 1.01 * float(np.linalg.eigvalsh(Phil)[-1])
    ref, _, nnz_o = sparsify.cpa_shrink_sparsified(X, sh_o, lam, K, T, keep, zero=zero)
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    Y, info = cpa.shrink_dense_sparsified(Xd, sh_c, cpa.Opts(K=K, Lambda=lam, eval=ev), keep=keep,
                                          transform=transform, info=True)
    torch.cuda.synchronize()
    err = metrics.rel_fro(Y.cpu().numpy().astype(np.float64), ref, X)
    print(f"sparsified {transform} {ev} {m}x{n} K={K} keep={keep} nnz={info['nnz']} (oracle {nnz_o}) "
          f"eps={info['eps']:.6e} (oracle {eps_o:.6e}) rel_fro={err:.3e}", flush=True)
    assert info["nnz"] == nnz_o
    # FP32 Gram (and FP32 transform products for the full DCT): absolute rounding
    # on the scale of the largest entry of Phi
    assert abs(info["eps"] - eps_o) <= eps_tol * float(np.abs(Phi).max())
    assert info["side"] == (0 if side_right else 1)
    parity.check(Y.cpu().numpy().astype(np.float64), ref, TOL32, X, f"sparsified {transform} {ev}")
    return Y


@pytest.mark.parametrize("ev", ["auto", "recurrence"])
@pytest.mark.parametrize("shape,frac,K,kind", [((256, 128), 0.02, 20, 0), ((128, 256), 0.02, 20, 0),
                                               ((512, 512), 0.01, 30, 3), ((320, 64), 0.1, 16, 1),
                                               ((64, 192), 0.05, 8, 0)])
def test_block_dct_truncated_matches_oracle(shape, frac, K, kind, ev):
    cpa = _lib()
    m, n = shape
    X = synth.as_f32_exact(synth.block_smooth(m, n, rank=4, noise=1e-3, seed=9100 + m + n))
    d = min(m, n)
    T = sparsify.block_dct(d, 8)
    G = X.T @ X if m >= n else X @ X.T
    s1 = math.sqrt(float(np.linalg.eigvalsh(G)[-1]))
    if kind == 0:
        sh_o, sh_c = Shrinkage(0, 0.2 * s1), cpa.soft(0.2 * s1)
    elif kind == 1:
        sh_o, sh_c = Shrinkage(1, 0.2 * s1), cpa.hard(0.2 * s1)
    else:
        wc, ws = 0.05 * s1 * s1, 0.01 * s1 * s1
        sh_o, sh_c = Shrinkage(3, 0.0, wc, ws, 1e-3), cpa.weighted_fn(wc, ws, 1e-3)
    _case(X, T, "block_dct8", frac, K, sh_o, sh_c, side_right=m >= n, ev=ev)


@pytest.mark.parametrize("ev", ["auto", "recurrence"])
@pytest.mark.parametrize("shape,frac", [((256, 128), 0.02), ((96, 200), 1e-9), ((512, 256), 0.004)])
def test_empty_rows_are_left_out_of_hat_h(shape, frac, ev):
    """hat H is computed on the rows with kept entries only (an empty row is an
    eigenvector with eigenvalue 0, where hat H is hat h(0)), by the matrix
    polynomial on that block (auto) or by the sparse recurrence; cases with many
    empty rows, a count of nonempty rows that is not a multiple of 4, and a keep
    count of a few entries."""
    cpa = _lib()
    m, n = shape
    X = synth.as_f32_exact(synth.block_smooth(m, n, rank=4, noise=1e-3, seed=9150 + m))
    d = min(m, n)
    T = sparsify.block_dct(d, 8)
    Phi, _ = sparsify.transformed_gram(X, T)
    keep = _gap_keep(Phi, frac)
    nonempty = int(np.count_nonzero(np.abs(sparsify.truncate(Phi, sparsify.kth_largest_abs(Phi, keep))).sum(1)))
    print(f"{m}x{n} keep {keep}: {nonempty} of {d} rows nonempty", flush=True)
    assert nonempty < d
    G = X.T @ X if m >= n else X @ X.T
    s1 = math.sqrt(float(np.linalg.eigvalsh(G)[-1]))
    _case(X, T, "block_dct8", frac, 18, Shrinkage(0, 0.15 * s1), cpa.soft(0.15 * s1), side_right=m >= n, ev=ev)


@pytest.mark.parametrize("ev", ["auto", "recurrence"])
@pytest.mark.parametrize("transform", ["haar1", "haar1_lowpass"])
@pytest.mark.parametrize("shape,frac", [((256, 128), 0.3), ((128, 192), 0.5), ((96, 64), 0.24)])
def test_haar_matches_oracle(shape, frac, transform, ev):
    """The one-level Haar DWT (the kernels order each 8-block's low-pass rows
    first; the oracle uses the global order, a row permutation with the same
    result), with and without every high-frequency component set to zero."""
    cpa = _lib()
    m, n = shape
    X = synth.as_f32_exact(synth.block_smooth(m, n, rank=4, noise=1e-3, seed=9700 + m + n))
    d = min(m, n)
    T = sparsify.haar_matrix(d)
    zero = (np.arange(d) >= d // 2) if transform == "haar1_lowpass" else None
    G = X.T @ X if m >= n else X @ X.T
    s1 = math.sqrt(float(np.linalg.eigvalsh(G)[-1]))
    _case(X, T, transform, frac, 20, Shrinkage(0, 0.2 * s1), cpa.soft(0.2 * s1), side_right=m >= n, ev=ev,
          zero=zero)


@pytest.mark.parametrize("ev", ["auto", "recurrence"])
@pytest.mark.parametrize("full", [False, True])
@pytest.mark.parametrize("shape", [(256, 128), (128, 192), (96, 64)])
def test_full_dct_matches_oracle(shape, full, ev):
    """The full DCT-II (FP32 transform products): smooth data whose transformed
    Gram lives on the 6 x 6 low-frequency corner; keep = 36 (that corner, a
    compact block of 6 rows, the next entry below 1e-5 of the largest) or all."""
    cpa = _lib()
    m, n = shape
    X = synth.as_f32_exact(synth.smooth_lowrank(m, n, rank=4, freqs=6, noise=1e-3, seed=9800 + m + n))
    d = min(m, n)
    G = X.T @ X if m >= n else X @ X.T
    s1 = math.sqrt(float(np.linalg.eigvalsh(G)[-1]))
    _case(X, sparsify.dct_matrix(d), "dct", 1.0, 20, Shrinkage(0, 0.2 * s1), cpa.soft(0.2 * s1), side_right=m >= n,
          ev=ev, keep=d * d if full else 36, eps_tol=1e-5)


@pytest.mark.parametrize("ev", ["auto", "recurrence"])
@pytest.mark.parametrize("transform", ["block_dct8", "identity"])
def test_no_truncation_equals_plain_shrinkage(transform, ev):
    """keep = d^2: T^T hat H(T G T^T) T = hat H(G) for orthogonal T."""
    import torch
    cpa = _lib()
    X = synth.as_f32_exact(synth.dense_lowrank(200, 96, rank=5, noise=0.2, seed=9300))
    G = X.T @ X
    lam = 1.01 * float(np.linalg.eigvalsh(G)[-1])
    tau = 0.3 * math.sqrt(lam)
    ref = ocpa.cpa_shrink(X, Shrinkage(0, tau), lam, 24)
    Y, info = cpa.shrink_dense_sparsified(torch.from_numpy(X.astype(np.float32)).cuda(), cpa.soft(tau),
                                          cpa.Opts(K=24, Lambda=lam, eval=ev), keep=96 * 96, transform=transform,
                                          info=True)
    torch.cuda.synchronize()
    err = metrics.rel_fro(Y.cpu().numpy().astype(np.float64), ref, X)
    print(f"no truncation {transform}: nnz {info['nnz']} rel_fro {err:.3e}", flush=True)
    assert info["nnz"] == 96 * 96
    assert err <= TOL32


@pytest.mark.parametrize("ev", ["auto", "recurrence"])
def test_identity_transform_truncates_a_nearly_diagonal_gram(ev):
    """Nearly orthogonal columns: the Gram is sparse in the identity basis."""
    cpa = _lib()
    m, n = 256, 64
    Q = synth.random_orthogonal(m, seed=9400)[:, :n]
    s = np.linspace(1.0, 8.0, n)
    X = synth.as_f32_exact(Q * s + 1e-3 * synth.dense_lowrank(m, n, rank=n, noise=0.0, seed=9401) / 8.0)
    T = np.eye(n)
    _case(X, T, "identity", 0.02, 16, Shrinkage(0, 3.0), cpa.soft(3.0), ev=ev)


@pytest.mark.parametrize("ev", ["auto", "recurrence"])
def test_power_bound_of_the_truncated_matrix(ev):
    """The bound from the compact block (auto) and from the whole truncated matrix
    (recurrence) both give the largest eigenvalue of the truncated matrix."""
    import torch
    cpa = _lib()
    X = synth.as_f32_exact(synth.block_smooth(256, 128, rank=4, noise=1e-3, seed=9500))
    T = sparsify.block_dct(128, 8)
    Phi, _ = sparsify.transformed_gram(X, T)
    keep = _gap_keep(Phi, 0.02)
    Phil = sparsify.truncate(Phi, sparsify.kth_largest_abs(Phi, keep))
    lam_o = obound.power_bound(Phil, seed=0, max_iter=200, tol=1e-9)[0]
    _, info = cpa.shrink_dense_sparsified(torch.from_numpy(X.astype(np.float32)).cuda(), cpa.soft(1.0),
                                          cpa.Opts(K=8, power_iters=200, power_tol=1e-9, eval=ev), keep=keep,
                                          info=True)
    print(f"truncated power bound: gpu {info['Lambda']:.8e} oracle {lam_o:.8e}", flush=True)
    assert abs(info["Lambda"] - lam_o) <= 1e-5 * lam_o


def test_sparsified_is_deterministic_and_rejects_bad_arguments():
    import torch
    cpa = _lib()
    X = torch.from_numpy(synth.block_smooth(128, 64, rank=3, noise=1e-3, seed=9600).astype(np.float32)).cuda()
    o = cpa.Opts(K=12, bound="frobenius")
    for ev in ("auto", "recurrence"):
        oe = cpa.Opts(K=12, bound="frobenius", eval=ev)
        Y1 = cpa.shrink_dense_sparsified(X, cpa.soft(1.0), oe, keep=100).clone()
        Y2 = cpa.shrink_dense_sparsified(X, cpa.soft(1.0), oe, keep=100).clone()
        torch.cuda.synchronize()
        assert torch.equal(Y1, Y2)
    with pytest.raises(cpa.CpaError):
        cpa.shrink_dense_sparsified(X, cpa.soft(1.0), o, keep=0)
    with pytest.raises(cpa.CpaError):
        cpa.shrink_dense_sparsified(X, cpa.soft(1.0), o, keep=64 * 64 + 1)
    with pytest.raises(cpa.CpaError):
        cpa.shrink_dense_sparsified(X, cpa.soft(1.0), cpa.Opts(K=12, precision="bf16x3"), keep=100)
    with pytest.raises(cpa.CpaError):
        cpa.shrink_dense_sparsified(X, cpa.soft(1.0), cpa.Opts(K=12, check=True), keep=100)
    X2 = torch.ones((40, 36), device="cuda")
    with pytest.raises(cpa.CpaError):
        cpa.shrink_dense_sparsified(X2, cpa.soft(1.0), o, keep=10)
    # Y written over X (or over part of it) is an argument error, caught before any launch
    before = X.clone()
    with pytest.raises(cpa.CpaError) as e:
        cpa.shrink_dense_sparsified(X, cpa.soft(1.0), o, keep=100, out=X)
    assert e.value.status == cpa.ERR_ARG
    big = torch.zeros((256, 64), device="cuda")
    big[:128] = X
    with pytest.raises(cpa.CpaError) as e:
        cpa.shrink_dense_sparsified(big[:128], cpa.soft(1.0), o, keep=100, out=big[64:192])
    assert e.value.status == cpa.ERR_ARG
    torch.cuda.synchronize()
    assert torch.equal(X, before)


@pytest.mark.parametrize("ev", ["auto", "recurrence"])
@pytest.mark.parametrize("transform", ["block_dct8", "dct"])
def test_given_threshold_matches_oracle(transform, ev):
    """eq. (threshold_components) with eps given (the experiments of Table III fix
    eps): the kernels take the FP32 eps as the threshold key and skip the selection.
    eps sits midway in a gap of more than 2% of the sorted |Phi|, so the kernel's
    FP32 and the oracle's FP64 keep the same entries."""
    import torch
    cpa = _lib()
    m, n = 256, 128
    if transform == "block_dct8":
        X = synth.as_f32_exact(synth.block_smooth(m, n, rank=4, noise=1e-3, seed=9900))
        T, frac = sparsify.block_dct(n, 8), 0.02
    else:
        X = synth.as_f32_exact(synth.smooth_lowrank(m, n, rank=4, freqs=6, noise=1e-3, seed=9901))
        T, frac = sparsify.dct_matrix(n), 36.0 / (n * n)
    Phi, _ = sparsify.transformed_gram(X, T)
    keep = _gap_keep(Phi, frac)
    a = np.sort(np.abs(Phi).ravel())[::-1]
    eps = 0.5 * (a[keep - 1] + a[keep])
    lam = 1.01 * float(np.linalg.eigvalsh(sparsify.truncate(Phi, eps))[-1])
    s1 = math.sqrt(float(np.linalg.eigvalsh(X.T @ X)[-1]))
    ref, _, nnz_o = sparsify.cpa_shrink_sparsified(X, Shrinkage(0, 0.2 * s1), lam, 20, T, None, eps=eps)
    Y, info = cpa.shrink_dense_sparsified(torch.from_numpy(X.astype(np.float32)).cuda(), cpa.soft(0.2 * s1),
                                          cpa.Opts(K=20, Lambda=lam, eval=ev), eps=eps, transform=transform,
                                          info=True)
    torch.cuda.synchronize()
    err = metrics.rel_fro(Y.cpu().numpy().astype(np.float64), ref, X)
    print(f"given eps {transform} {ev}: eps={eps:.6e} nnz={info['nnz']} (oracle {nnz_o}) rel_fro={err:.3e}",
          flush=True)
    assert info["nnz"] == nnz_o
    assert info["eps"] == float(np.float32(eps))
    assert err <= TOL32


@pytest.mark.parametrize("ev", ["auto", "recurrence"])
def test_given_threshold_above_every_entry_gives_zero(ev):
    """An eps above every |Phi_ij| keeps nothing: Y = 0 exactly on both routes, with
    a power bound and with a given one, and the kept count 0."""
    import torch
    cpa = _lib()
    X = synth.as_f32_exact(synth.block_smooth(200, 96, rank=4, noise=1e-3, seed=9910))
    Phi, _ = sparsify.transformed_gram(X, sparsify.block_dct(96, 8))
    eps = 2.0 * float(np.abs(Phi).max())
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    for opts in (cpa.Opts(K=16, eval=ev), cpa.Opts(K=16, Lambda=float(np.abs(Phi).max()), eval=ev)):
        Y = torch.full_like(Xd, float("nan"))
        _, info = cpa.shrink_dense_sparsified(Xd, cpa.soft(1.0), opts, eps=eps, out=Y, info=True)
        torch.cuda.synchronize()
        print(f"eps above every entry ({ev}): nnz {info['nnz']}, nonzeros in Y {int(torch.count_nonzero(Y))}",
              flush=True)
        assert info["nnz"] == 0
        assert int(torch.count_nonzero(Y)) == 0


def test_given_threshold_argument_errors():
    import torch
    cpa = _lib()
    Xd = torch.ones(64, 32, device="cuda")
    with pytest.raises(ValueError):
        cpa.shrink_dense_sparsified(Xd, cpa.soft(1.0), cpa.Opts(K=8), keep=10, eps=1.0)
    with pytest.raises(ValueError):
        cpa.shrink_dense_sparsified(Xd, cpa.soft(1.0), cpa.Opts(K=8))
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(cpa.CpaError) as e:
            cpa.shrink_dense_sparsified(Xd, cpa.soft(1.0), cpa.Opts(K=8), eps=bad)
        assert e.value.status == 1


@pytest.mark.parametrize("ev", ["auto", "recurrence"])
def test_selection_at_ties_is_exact(ev):
    """Integer entries |x| <= 3 make the FP32 Gram exact (T = Id, Phi = G), with
    long runs of equal magnitudes.  For keep counts inside such runs the threshold
    must be the k-th largest |Phi| exactly and every entry equal to it kept, so
    the kept count (above k) matches numpy's count on the same integers; then the
    result against the oracle with that keep."""
    import torch
    cpa = _lib()
    g = synth.rng(9700)
    m, n, K = 200, 64, 12
    X = g.integers(-3, 4, size=(m, n)).astype(np.float64)
    G = X.T @ X
    a = np.sort(np.abs(G).ravel())[::-1]
    inside = [k for k in range(3, a.size) if a[k - 2] == a[k - 1] == a[k]]
    picks = sorted({inside[len(inside) // 6], inside[len(inside) // 2], inside[(5 * len(inside)) // 6]})
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    T = np.eye(n)
    for k in picks:
        eps_o = sparsify.kth_largest_abs(G, k)
        nnz_o = int(np.count_nonzero(np.abs(G) >= eps_o))
        Phil = sparsify.truncate(G, eps_o)
        lam = 1.01 * float(np.linalg.eigvalsh(Phil)[-1])
        tau = 0.3 * math.sqrt(lam)
        Y, info = cpa.shrink_dense_sparsified(Xd, cpa.soft(tau), cpa.Opts(K=K, Lambda=lam, eval=ev), keep=k,
                                              transform="identity", info=True)
        torch.cuda.synchronize()
        print(f"ties {ev}: keep {k} -> eps gpu {info['eps']} oracle {eps_o}, kept gpu {info['nnz']} "
              f"oracle {nnz_o}", flush=True)
        assert nnz_o > k
        assert info["eps"] == eps_o and info["nnz"] == nnz_o
        ref, _, nnz_r = sparsify.cpa_shrink_sparsified(X, Shrinkage(0, tau), lam, K, T, k)
        assert nnz_r == nnz_o
        parity.check(Y.cpu().numpy().astype(np.float64), ref, TOL32, X, f"ties keep={k} {ev}")


@pytest.mark.parametrize("ev", ["auto", "recurrence"])
def test_block_dct_full_size(ev):
    """The bench's sparsified workload at full size: 1024 x 1024 block-smooth
    input (rank 4, 8-blocks), block DCT, K = 30, soft tau = 0.2 sigma_1, about
    1.6% of the transformed Gram kept (at a gap in |Phi|)."""
    cpa = _lib()
    X = synth.as_f32_exact(synth.block_smooth(1024, 1024, rank=4, noise=1e-3, seed=synth.BASE_SEED + 6))
    T = sparsify.block_dct(1024, 8)
    s1 = math.sqrt(float(np.linalg.eigvalsh(X.T @ X)[-1]))
    _case(X, T, "block_dct8", 0.016, 30, Shrinkage(0, 0.2 * s1), cpa.soft(0.2 * s1), ev=ev)


def test_block_dct_paper_shape():
    """The bench's paper-shape workload: one 2560 x 1920 block-smooth component
    (Gram side 1920), block DCT, K = 30, soft tau = 0.2 sigma_1, about 1.6% of the
    transformed Gram kept (at a gap in |Phi|); every output element against the
    oracle's transform-and-truncate shrink."""
    cpa = _lib()
    X = synth.as_f32_exact(synth.block_smooth(2560, 1920, rank=4, noise=1e-3, seed=synth.BASE_SEED + 8))
    T = sparsify.block_dct(1920, 8)
    s1 = math.sqrt(float(np.linalg.eigvalsh(X.T @ X)[-1]))
    _case(X, T, "block_dct8", 0.016, 30, Shrinkage(0, 0.2 * s1), cpa.soft(0.2 * s1), ev="auto")


def test_warm_start_maps_the_block_rows():
    """opts.warm_start on the polynomial route: the compact block's power vector is
    kept in the coordinates of the full transformed Gram and mapped onto the next
    call's block.  A repeated call needs fewer products and gives the same bound to
    the iteration's tolerance; a call on another input (other kept rows) still
    matches the oracle at the bound it reports."""
    import torch
    cpa = _lib()
    T = sparsify.block_dct(128, 8)
    opts = cpa.Opts(K=20, warm_start=True, power_tol=1e-9, power_iters=300)
    res = []
    for seed in (9801, 9801, 9802):
        X = synth.as_f32_exact(synth.block_smooth(256, 128, rank=4, noise=1e-3, seed=seed))
        Phi, _ = sparsify.transformed_gram(X, T)
        keep = _gap_keep(Phi, 0.02)
        s1 = math.sqrt(float(np.linalg.eigvalsh(X.T @ X)[-1]))
        Xd = torch.from_numpy(X.astype(np.float32)).cuda()
        Y, info = cpa.shrink_dense_sparsified(Xd, cpa.soft(0.2 * s1), opts, keep=keep, info=True)
        torch.cuda.synchronize()
        ref, _, _ = sparsify.cpa_shrink_sparsified(X, Shrinkage(0, 0.2 * s1), info["Lambda"], 20, T, keep)
        parity.check(Y.cpu().numpy().astype(np.float64), ref, TOL32, X, f"warm sparsified seed {seed}")
        res.append(info)
        print(f"  seed {seed}: power products {info['power_iters_done']} Lambda {info['Lambda']:.10g}", flush=True)
    assert res[1]["power_iters_done"] < res[0]["power_iters_done"]
    assert abs(res[1]["Lambda"] - res[0]["Lambda"]) <= 1e-7 * res[0]["Lambda"]
