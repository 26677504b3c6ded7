"""GPU parity of the dense FP32 path against the FP64 oracle (Algorithm 1 with
T = Id).  Lambda is passed explicitly so parity isolates the polynomial
evaluation; a separate test compares the device bound with the oracle's.
Tolerance of the FP32 path: relative Frobenius error <= 1e-5."""
import math
import sys

import numpy as np
import pytest

import synth
from tests import parity
from oracle import bound as obound
from oracle import cpa as ocpa
from oracle import metrics
from oracle.shrinkage import Shrinkage

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def _torch():
    import torch
    return torch


def _lib():
    import paper_1705_07112_amd as cpa
    return cpa


def _gram_lmax(X):
    G = X.T @ X if X.shape[0] >= X.shape[1] else X @ X.T
    return float(np.linalg.eigvalsh(G)[-1]) if G.size else 0.0


def _run(X64, sh_c, K, Lam, ld=None, offset=0, ev="auto", side="auto"):
    torch = _torch()
    cpa = _lib()
    m, n = X64.shape
    ld = ld or n
    buf = torch.zeros(offset + m * ld + 8, dtype=torch.float32)
    view = buf[offset:offset + m * ld].view(m, ld)[:, :n]
    view.copy_(torch.from_numpy(X64.astype(np.float32)))
    bufd = buf.cuda()
    Xd = bufd[offset:offset + m * ld].view(m, ld)[:, :n]
    Y, info = cpa.shrink_dense(Xd, sh_c, cpa.Opts(K=K, Lambda=Lam, eval=ev, side=side), info=True)
    torch.cuda.synchronize()
    return Y.cpu().numpy().astype(np.float64), info


def _case(m, n, K, kind, seed, ld=None, offset=0, ev="auto", side="auto"):
    print(f"case m={m} n={n} K={K} kind={kind} seed={seed} ld={ld} off={offset} eval={ev} side={side}", flush=True)
    X = synth.as_f32_exact(synth.dense_lowrank(m, n, rank=min(4, m, n), noise=0.2, seed=seed))
    lmax = _gram_lmax(X)
    Lam = 1.01 * lmax
    tau = 0.4 * math.sqrt(lmax)
    cpa = _lib()
    if kind == 0:
        sh_o, sh_c = Shrinkage(0, tau), cpa.soft(tau)
    elif kind == 1:
        sh_o, sh_c = Shrinkage(1, tau), cpa.hard(tau)
    else:
        wc, ws = 0.3 * tau * tau, 0.05 * lmax
        sh_o, sh_c = Shrinkage(3, 0.0, wc, ws, 1e-3), cpa.weighted_fn(wc, ws, 1e-3)
    ref = ocpa.cpa_shrink(X, sh_o, Lam, K)
    got, info = _run(X, sh_c, K, Lam, ld=ld, offset=offset, ev=ev, side=side)
    err, _ = parity.check(got, ref, TOL32, X, f"{m}x{n} K={K} kind={kind}")
    assert info["side"] == {"auto": 0 if m >= n else 1, "right": 0, "left": 1}[side]
    return err


def test_config1_shape_soft():
    _case(64, 48, 20, 0, synth.BASE_SEED)


EDGE = [1, 2, 3, 15, 16, 17, 63, 64, 65, 127, 128, 129]


@pytest.mark.parametrize("m", EDGE)
def test_edge_shapes_tall(m):
    for n in (1, 3, 16, 17, 65):
        if n <= m:
            _case(m, n, 16, 0, 1000 + m * 7 + n)


@pytest.mark.parametrize("n", [2, 17, 64, 129])
def test_edge_shapes_wide(n):
    for m in (1, 3, 16, 63):
        if m < n:
            _case(m, n, 16, 0, 2000 + m * 7 + n)


@pytest.mark.parametrize("K", [1, 2, 3, 16, 30])
@pytest.mark.parametrize("kind", [0, 1, 2])
def test_orders_and_kinds(K, kind):
    _case(130, 70, K, kind, 3000 + K)
    _case(70, 130, K, kind, 4000 + K)


def test_strided_and_unaligned_input():
    _case(77, 45, 12, 0, 5001, ld=53)
    _case(77, 45, 12, 0, 5002, ld=48, offset=1)
    _case(40, 90, 12, 0, 5003, ld=97, offset=3)


def test_multi_tile_ragged_sizes():
    # several 128-wide tiles plus a ragged tail on both sides
    _case(1100, 300, 10, 0, 6001)
    _case(300, 1100, 10, 0, 6002)


def test_special_cases():
    torch = _torch()
    cpa = _lib()
    X = synth.as_f32_exact(synth.dense_lowrank(50, 30, rank=3, noise=0.1, seed=7))
    lmax = _gram_lmax(X)
    Lam = 1.01 * lmax
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    # tau = 0: identity
    Y = cpa.shrink_dense(Xd, cpa.soft(0.0), cpa.Opts(K=9, Lambda=Lam)).cpu().numpy()
    assert metrics.rel_fro(Y, X) < 1e-5
    # tau^2 >= Lambda: exact zero
    Y = cpa.shrink_dense(Xd, cpa.soft(math.sqrt(Lam)), cpa.Opts(K=9, Lambda=Lam)).cpu().numpy()
    assert np.all(Y == 0.0)
    # X = 0 with the power bound: Lambda = 0 and Y = 0
    Z = torch.zeros(20, 10, device="cuda")
    Y, info = cpa.shrink_dense(Z, cpa.soft(1.0), cpa.Opts(K=5), info=True)
    assert info["Lambda"] == 0.0 and torch.count_nonzero(Y).item() == 0
    # empty input: no-op
    E = torch.zeros(0, 5, device="cuda")
    assert cpa.shrink_dense(E, cpa.soft(1.0), cpa.Opts(K=5)).shape == (0, 5)
    # Y aliasing X is rejected
    with pytest.raises(cpa.CpaError):
        cpa.shrink_dense(Xd, cpa.soft(1.0), cpa.Opts(K=5), out=Xd)
    with pytest.raises(cpa.CpaError):
        cpa.shrink_dense(Xd, cpa.soft(1.0), cpa.Opts(K=0))


def test_device_bound_matches_oracle():
    """Gram sides from 4 to 1024, aligned and not (90)."""
    torch = _torch()
    cpa = _lib()
    for seed, (m, n) in enumerate([(64, 48), (200, 120), (90, 300), (400, 256), (256, 4), (1024, 1024)]):
        X = synth.as_f32_exact(synth.dense_lowrank(m, n, rank=5, noise=0.3, seed=7000 + seed))
        G = X.T @ X if m >= n else X @ X.T
        lam_o = obound.power_bound(G, seed=seed, max_iter=200, tol=1e-9)[0]
        Xd = torch.from_numpy(X.astype(np.float32)).cuda()
        lam_g, info = cpa.spectral_bound(Xd, cpa.Opts(K=4, power_iters=200, power_tol=1e-9, seed=seed))
        print(f"bound m={m} n={n} oracle={lam_o:.10g} gpu={lam_g:.10g} iters={info['power_iters_done']}", flush=True)
        assert abs(lam_g - lam_o) <= 2e-6 * lam_o
        assert lam_g >= float(np.linalg.eigvalsh(G)[-1]) * (1 - 1e-6)


def test_growth_check_falls_back_to_frobenius_bound():
    torch = _torch()
    cpa = _lib()
    X = synth.as_f32_exact(synth.dense_lowrank(96, 64, rank=4, noise=0.1, seed=8))
    G = X.T @ X
    lmax = float(np.linalg.eigvalsh(G)[-1])
    tau = 0.3 * math.sqrt(lmax)
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    Y, info = cpa.shrink_dense(Xd, cpa.soft(tau), cpa.Opts(K=20, Lambda=0.6 * lmax, check=True), info=True)
    assert info["fallback"] == 1
    fro = math.sqrt(float(np.sum(G * G)))
    assert info["Lambda"] == pytest.approx(fro, rel=1e-5)
    ref = ocpa.cpa_shrink(X, Shrinkage(0, tau), info["Lambda"], 20)
    assert metrics.rel_fro(Y.cpu().numpy(), ref) < TOL32
    # a sound bound passes the check without fallback
    _, info = cpa.shrink_dense(Xd, cpa.soft(tau), cpa.Opts(K=20, check=True), info=True)
    assert info["fallback"] == 0 and info["max_growth"] <= 1.0 + 1e-3


def test_full_size_rpca_matrix_sampled_rows():
    """1024 x 1024, K = 30, the shrink of the ADMM workload (tau = 1/rho = 10),
    checked on sampled output rows (rows of X H depend only on those rows of X)."""
    torch = _torch()
    cpa = _lib()
    I, _, _ = synth.rpca_frames()
    X = I.astype(np.float64)
    G = X.T @ X
    lam_o = obound.power_bound(G, seed=0)[0]
    K, tau = 30, 10.0
    Xd = torch.from_numpy(I).cuda()
    Y = cpa.shrink_dense(Xd, cpa.soft(tau), cpa.Opts(K=K, Lambda=lam_o)).cpu().numpy()
    rows = np.array([0, 1, 2, 63, 64, 65, 511, 512, 777, 1000, 1022, 1023])
    ref = ocpa.cpa_rows(X, Shrinkage(0, tau), lam_o, K, rows)
    err, _ = parity.check(Y[rows].astype(np.float64), ref, TOL32, label="full-size sampled rows")
    assert err <= TOL32
    # the power bound path on the device agrees with the oracle's bound
    lam_g, _ = cpa.spectral_bound(Xd, cpa.Opts(K=K))
    assert abs(lam_g - lam_o) <= 2e-6 * lam_o


@pytest.mark.parametrize("ev", ["recurrence", "polynomial"])
@pytest.mark.parametrize("shape,K", [((64, 48), 20), ((130, 70), 30), ((70, 130), 30), ((129, 129), 7),
                                     ((300, 1100), 16), ((1, 5), 9), ((5, 1), 9), ((200, 3), 64),
                                     ((64, 64), 100), ((64, 64), 144), ((97, 33), 2), ((97, 33), 3),
                                     ((40, 30), 256), ((192, 320), 30), ((320, 192), 25), ((128, 128), 40),
                                     ((256, 320), 30), ((640, 320), 25), ((512, 512), 16)])
def test_both_evaluation_routes(ev, shape, K):
    """The recurrence over X and the matrix polynomial on the d x d side (baby
    steps / giant steps) against the same oracle."""
    m, n = shape
    for kind in (0, 1, 2):
        _case(m, n, K, kind, seed=7000 + m + n + K, ev=ev)


def test_polynomial_route_full_size_and_unaligned():
    torch = _torch()
    cpa = _lib()
    I, _, _ = synth.rpca_frames()
    X = I.astype(np.float64)
    lam_o = obound.power_bound(X.T @ X, seed=0)[0]
    Xd = torch.from_numpy(I).cuda()
    rows = np.array([0, 5, 64, 511, 777, 1023])
    for K in (16, 30, 64):
        Y = cpa.shrink_dense(Xd, cpa.soft(10.0), cpa.Opts(K=K, Lambda=lam_o, eval="polynomial")).cpu().numpy()
        ref = ocpa.cpa_rows(X, Shrinkage(0, 10.0), lam_o, K, rows)
        err, _ = parity.check(Y[rows].astype(np.float64), ref, TOL32, label=f"polynomial route 1024^2 K={K} sampled")
        assert err <= TOL32
    # odd d (no 16-byte rows) and a strided input
    _case(131, 77, 25, 0, seed=91, ev="polynomial")
    _case(77, 131, 25, 0, seed=92, ev="polynomial", ld=140, offset=3)


def test_polynomial_route_is_deterministic():
    """The polynomial route (direct global-to-LDS products at these sizes) gives
    the same bits on every call."""
    torch = _torch()
    cpa = _lib()
    for d, K in ((256, 30), (512, 25), (1024, 30)):
        X = torch.from_numpy(synth.dense_lowrank(d, d, rank=8, noise=0.1, seed=d).astype(np.float32)).cuda()
        o = cpa.Opts(K=K, eval="polynomial", bound="frobenius")
        Y1 = cpa.shrink_dense(X, cpa.soft(0.5), o).clone()
        Y2 = cpa.shrink_dense(X, cpa.soft(0.5), o).clone()
        torch.cuda.synchronize()
        assert torch.equal(Y1, Y2), d


def test_polynomial_route_limits_and_check():
    torch = _torch()
    cpa = _lib()
    Xd = torch.ones((8, 4), device="cuda")
    with pytest.raises(cpa.CpaError):
        cpa.shrink_dense(Xd, cpa.soft(0.1), cpa.Opts(K=1025, eval="polynomial"))
    # the recurrence reports its growth, the polynomial route its weighted means (<= 1)
    _, info = cpa.shrink_dense(Xd, cpa.soft(0.1), cpa.Opts(K=9, check=True, eval="recurrence"), info=True)
    assert info["max_growth"] > 0.0
    _, info = cpa.shrink_dense(Xd, cpa.soft(0.1), cpa.Opts(K=9, check=True, eval="polynomial"), info=True)
    assert 0.0 < info["max_growth"] <= 1.0 + 1e-3 and info["fallback"] == 0


@pytest.mark.parametrize("ev", ["polynomial", "recurrence"])
@pytest.mark.parametrize("shape,factor", [((300, 200), 0.9), ((1024, 1024), 0.9), ((120, 300), 0.6)])
def test_check_catches_a_bound_below_lambda_max(ev, shape, factor):
    """Lambda = 0.9 (or 0.6) lambda_max puts the top eigenvalue outside [-1, 1]: the
    check fires on both routes and the result is recomputed at Lambda = ||G||_F,
    equal to the oracle there; a sound bound passes with no fallback.  The 1024 x
    1024 case is the RPCA frames (the headline shape, where the top eigenvalue
    carries almost all the weight of tr G)."""
    torch = _torch()
    cpa = _lib()
    m, n = shape
    if shape == (1024, 1024):
        X = synth.rpca_frames()[0].astype(np.float64)
        tau = 10.0
    else:
        X = synth.as_f32_exact(synth.dense_lowrank(m, n, rank=8, noise=0.3, seed=7500 + m))
        tau = 0.2 * math.sqrt(_gram_lmax(X))
    lmax = _gram_lmax(X)
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    Y, info = cpa.shrink_dense(Xd, cpa.soft(tau), cpa.Opts(K=30, Lambda=factor * lmax, check=True, eval=ev),
                               info=True)
    print(f"check {ev} {m}x{n} Lambda={factor} lambda_max: max_growth {info['max_growth']:.4g} "
          f"fallback {info['fallback']}", flush=True)
    assert info["fallback"] == 1
    G = X.T @ X if m >= n else X @ X.T
    assert info["Lambda"] == pytest.approx(math.sqrt(float(np.sum(G * G))), rel=1e-5)
    ref = ocpa.cpa_shrink(X, Shrinkage(0, tau), info["Lambda"], 30)
    parity.check(Y.cpu().numpy(), ref, TOL32, X, f"after fallback {ev}")
    _, info = cpa.shrink_dense(Xd, cpa.soft(tau), cpa.Opts(K=30, check=True, eval=ev), info=True)
    assert info["fallback"] == 0 and info["max_growth"] <= 1.0 + 1e-3


def test_power_bound_large_d_reads_iterate_from_global():
    """d above the LDS copy of the iterate (4096): the cooperative power iteration
    reads w_{t-1} with agent-scope loads; its bound matches the oracle's."""
    torch = _torch()
    cpa = _lib()
    X = synth.dense_lowrank(4160, 4160, rank=12, noise=0.05, seed=4160).astype(np.float32)
    G = X.astype(np.float64).T @ X.astype(np.float64)
    lam_o = obound.power_bound(G, seed=0, max_iter=100, tol=1e-7)[0]
    lam_g, _ = cpa.spectral_bound(torch.from_numpy(X).cuda(), cpa.Opts(K=8))
    print(f"d=4160 power bound: gpu {lam_g:.9e} oracle {lam_o:.9e}", flush=True)
    assert abs(lam_g - lam_o) <= 2e-6 * lam_o


@pytest.mark.parametrize("ev", ["recurrence", "polynomial"])
@pytest.mark.parametrize("shape,side", [((130, 70), "left"), ((70, 130), "right"), ((130, 70), "right"),
                                        ((70, 130), "left"), ((64, 64), "left"), ((128, 192), "right")])
def test_explicit_gram_side(ev, shape, side):
    """X h(X^T X) = h(X X^T) X: forcing the larger Gram gives the same shrinkage
    (within the FP32 bar) on both evaluation routes."""
    m, n = shape
    for kind in (0, 2):
        _case(m, n, 20, kind, seed=8800 + m + 3 * n, ev=ev, side=side)


def test_side_rejections():
    torch = _torch()
    cpa = _lib()
    X = torch.ones((8, 4), device="cuda")
    bad = cpa.Opts(K=4).to_c()
    bad.side = 3
    import ctypes
    Y = torch.empty_like(X)
    st = cpa.lib().cpa_shrink_dense(ctypes.c_void_p(cpa.context(0)), cpa._stream(X), 8, 4, ctypes.c_void_p(X.data_ptr()), 4,
                                    ctypes.c_void_p(Y.data_ptr()), 4, ctypes.byref(cpa.soft(0.5)), ctypes.byref(bad), None)
    assert st == 1   # CPA_ERR_ARG


def test_workspace_bytes_query():
    """The workspace query covers the Gram, both Y buffers and the polynomial
    buffers of the route that runs, grows with the shape, and allocates nothing
    the following shrink would not reuse."""
    cpa = _lib()
    rec = cpa.workspace_bytes(1024, 1024, cpa.Opts(K=30, eval="recurrence"))
    poly = cpa.workspace_bytes(1024, 1024, cpa.Opts(K=30, eval="polynomial"))
    small = cpa.workspace_bytes(256, 128, cpa.Opts(K=30))
    d, mn = 1024, 1024 * 1024
    assert rec >= 4 * (d * d + 2 * mn) + 8 * d
    # s = 6, J = 5: T_1..T_6, R_0..R_4 and three Clenshaw buffers of d x d
    assert poly >= rec + 4 * 14 * d * d
    assert 4 * (128 * 128 + 2 * 256 * 128) <= small < rec
    assert cpa.workspace_bytes(0, 5, cpa.Opts(K=4)) == 0
    # the larger Gram (300 x 300 instead of 100 x 100) on the same route
    left = cpa.workspace_bytes(300, 100, cpa.Opts(K=8, side="left", eval="recurrence"))
    right = cpa.workspace_bytes(300, 100, cpa.Opts(K=8, eval="recurrence"))
    assert left - right >= 4 * (300 * 300 - 100 * 100)


@pytest.mark.parametrize("damping", ["jackson", "lanczos"])
@pytest.mark.parametrize("ev", ["recurrence", "polynomial"])
def test_damped_coefficients_match_oracle(damping, ev):
    """Coefficients times the Jackson or Lanczos factors (opts.damping; not in the
    paper), including the high-order hard threshold (K = 64) it is meant for."""
    torch = _torch()
    cpa = _lib()
    for (m, n), K, kind in (((130, 70), 64, 1), ((70, 130), 30, 0), ((256, 192), 64, 1)):
        X = synth.as_f32_exact(synth.dense_lowrank(m, n, rank=4, noise=0.2, seed=7700 + m + K))
        lmax = _gram_lmax(X)
        Lam, tau = 1.01 * lmax, 0.4 * math.sqrt(lmax)
        sh_o, sh_c = (Shrinkage(1, tau), cpa.hard(tau)) if kind == 1 else (Shrinkage(0, tau), cpa.soft(tau))
        ref = ocpa.cpa_shrink(X, sh_o, Lam, K, damping=damping)
        Y = cpa.shrink_dense(torch.from_numpy(X.astype(np.float32)).cuda(), sh_c,
                             cpa.Opts(K=K, Lambda=Lam, eval=ev, damping=damping))
        torch.cuda.synchronize()
        err = metrics.rel_fro(Y.cpu().numpy().astype(np.float64), ref, X)
        undamped = ocpa.cpa_shrink(X, sh_o, Lam, K)
        print(f"damping {damping} {ev} {m}x{n} K={K} kind={kind}: rel_fro={err:.3e} "
              f"(damped vs undamped oracle {metrics.rel_fro(ref, undamped, X):.2e})", flush=True)
        assert err <= TOL32
        assert metrics.rel_fro(ref, undamped, X) > 1e-4   # the damping changed the result


def test_release_and_row_stride_checks():
    """release() destroys the contexts (as at interpreter exit); the next call
    makes a fresh one and gives the same result.  Tensors whose rows overlap are
    refused by the binding."""
    import torch
    import paper_1705_07112_amd as cpa
    X = torch.from_numpy(synth.as_f32_exact(synth.dense_lowrank(100, 70, rank=4, seed=77)).astype(np.float32)).cuda()
    Y1 = cpa.shrink_dense(X, cpa.soft(1.0), cpa.Opts(K=12)).clone()
    cpa.release()
    Y2 = cpa.shrink_dense(X, cpa.soft(1.0), cpa.Opts(K=12))
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)
    row = torch.ones((1, 70), device="cuda")
    with pytest.raises(ValueError):
        cpa.shrink_dense(row.expand(100, 70), cpa.soft(1.0), cpa.Opts(K=4))
    with pytest.raises(ValueError):
        cpa.shrink_dense(torch.ones(8 * 99 + 70, device="cuda").as_strided((100, 70), (8, 1)), cpa.soft(1.0),
                         cpa.Opts(K=4))


@pytest.mark.parametrize("ev", ["recurrence", "polynomial"])
def test_frobenius_bound_without_margin_on_rpca_frames(ev):
    """Lambda = ||G||_F with no margin (the Frobenius rule, and the bound the
    growth-check and barrier-timeout fallbacks take): on the 1024 x 1024 frames
    ||G||_F / lambda_max is 1 + 1e-5, so the top eigenvalue sits at the end of
    [-1, 1], where T_k has slope k^2 and rounding is amplified the most.  The
    whole output against the oracle at the same Lambda, on both routes; then the
    device's own Frobenius rule (its FP32 Gram's norm) at the Lambda it reports."""
    torch = _torch()
    cpa = _lib()
    I, _, _ = synth.rpca_frames()
    X = I.astype(np.float64)
    G = X.T @ X
    Lam = float(np.linalg.norm(G))
    lmax = float(np.linalg.eigvalsh(G)[-1])
    print(f"frames: ||G||_F / lambda_max - 1 = {Lam / lmax - 1:.3e}, eval={ev}", flush=True)
    Xd = torch.from_numpy(I).cuda()
    Y = cpa.shrink_dense(Xd, cpa.soft(10.0), cpa.Opts(K=30, Lambda=Lam, eval=ev)).cpu().numpy()
    ref = ocpa.cpa_shrink(X, Shrinkage(0, 10.0), Lam, 30)
    parity.check(Y, ref, TOL32, X, f"Lambda = ||G||_F {ev}")
    Y2, info = cpa.shrink_dense(Xd, cpa.soft(10.0), cpa.Opts(K=30, bound="frobenius", eval=ev), info=True)
    assert abs(info["Lambda"] - Lam) <= 1e-6 * Lam
    ref2 = ocpa.cpa_shrink(X, Shrinkage(0, 10.0), info["Lambda"], 30)
    parity.check(Y2.cpu().numpy(), ref2, TOL32, X, f"device Frobenius rule {ev}")


@pytest.mark.parametrize("shape", [(1400, 1344), (1300, 1300), (1250, 1400)])
def test_polynomial_route_symmetric_products(shape):
    """Gram sides above 1024: the matrix polynomial's products cover only the
    upper-triangle tiles and write each tile mirrored (d = 1344 through the
    direct-to-LDS kernel; 1300 and the left side, d = 1250, through the
    register-staged one), against the oracle at two orders."""
    m, n = shape
    cpa = _lib()
    X = synth.as_f32_exact(synth.dense_lowrank(m, n, rank=6, noise=0.2, seed=7300 + m + n))
    lmax = _gram_lmax(X)
    Lam, tau = 1.01 * lmax, 0.4 * math.sqrt(lmax)
    for K in (9, 30):
        got, info = _run(X, cpa.soft(tau), K, Lam, ev="polynomial")
        ref = ocpa.cpa_shrink(X, Shrinkage(0, tau), Lam, K)
        parity.check(got, ref, TOL32, X, f"symmetric products {m}x{n} K={K}")


@pytest.mark.parametrize("shape,orders", [((130, 64), (9, 30)), ((300, 128), (9, 30)), ((400, 320), (5, 30)),
                                          ((128, 700), (9, 30)), ((1100, 1024), (9, 30)), ((2100, 2048), (9,))])
def test_polynomial_route_symmetric_pieces(shape, orders):
    """Gram sides that are multiples of 64 up to 2048: the products of the matrix
    polynomial run in pieces (each tile above the diagonal as two 64 x 32 halves,
    each diagonal tile's upper triangle; stored and mirrored): one diagonal piece
    only (d = 64), no XCD interleave (d = 320, 25 pieces), the left side (d = 128),
    one round on 256 CUs (d = 1024) and four rounds (d = 2048), against the oracle."""
    m, n = shape
    cpa = _lib()
    X = synth.as_f32_exact(synth.dense_lowrank(m, n, rank=6, noise=0.2, seed=7400 + m + n))
    lmax = _gram_lmax(X)
    Lam, tau = 1.01 * lmax, 0.4 * math.sqrt(lmax)
    for K in orders:
        print(f"case pieces {m}x{n} K={K}", flush=True)
        got, info = _run(X, cpa.soft(tau), K, Lam, ev="polynomial")
        ref = ocpa.cpa_shrink(X, Shrinkage(0, tau), Lam, K)
        parity.check(got, ref, TOL32, X, f"symmetric pieces {m}x{n} K={K}")


def test_non_finite_input():
    """A NaN or an infinity in X: synchronising calls (info, check) return
    CPA_ERR_NONFINITE, whatever the bound rule; an asynchronous call cannot
    report it and the NaN propagates into Y (as the header states)."""
    torch = _torch()
    cpa = _lib()
    X = synth.as_f32_exact(synth.dense_lowrank(130, 70, rank=4, seed=76)).astype(np.float32)
    for bad in (float("nan"), float("inf"), -float("inf")):
        Xb = X.copy()
        Xb[17, 33] = bad
        Xd = torch.from_numpy(Xb).cuda()
        for opts in (cpa.Opts(K=12), cpa.Opts(K=12, Lambda=100.0), cpa.Opts(K=12, bound="frobenius"),
                     cpa.Opts(K=12, eval="recurrence")):
            with pytest.raises(cpa.CpaError) as e:
                cpa.shrink_dense(Xd, cpa.soft(1.0), opts, info=True)
            assert e.value.status == cpa.ERR_NONFINITE, (bad, opts)
        with pytest.raises(cpa.CpaError) as e:
            cpa.shrink_dense(Xd, cpa.soft(1.0), cpa.Opts(K=12, check=True))
        assert e.value.status == cpa.ERR_NONFINITE
        Y = cpa.shrink_dense(Xd, cpa.soft(1.0), cpa.Opts(K=12))
        torch.cuda.synchronize()
        assert not torch.isfinite(Y).all()
    # the sparse path reports it too (through info)
    rowptr = np.array([0, 1, 2, 3], dtype=np.int32)
    vals = np.array([1.0, float("nan"), 2.0], dtype=np.float32)
    with pytest.raises(cpa.CpaError) as e:
        cpa.shrink_csr(3, 3, torch.from_numpy(rowptr).cuda(), torch.from_numpy(np.array([0, 1, 2], np.int32)).cuda(),
                       torch.from_numpy(vals).cuda(), cpa.soft(0.1), cpa.Opts(K=5), info=True)
    assert e.value.status == cpa.ERR_NONFINITE


def _model(seed, X, bias0=None):
    """A predictor model whose input normalisation centres X's features."""
    from oracle import mlp as omlp
    from paper_1705_07112_amd import predictor
    f = omlp.features(X)
    m = predictor.init_model(seed, f - np.array([0.7, -0.4, 0.9]), np.ones(3))
    g = synth.rng(seed)
    m[192:256] = g.uniform(-0.3, 0.3, 64)      # hidden biases, so every layer matters
    m[4352:4416] = g.uniform(-0.3, 0.3, 64)
    m[4544] = -0.4
    if bias0 is not None:
        m[4416:4480] = 0.0        # y0 = bias only
        m[4544] = bias0
    return m


def test_learned_bound_rule():
    """CPA_BOUND_LEARNED on the dense path: Lambda = (1 + margin) ||G||_F exp(min(y0, 0))
    from the network on (log ||X||_F, log ||G||_F^2, log mn), against the oracle
    network; the shrink at that Lambda against the oracle; a network that says
    Lambda = 0.05 ||G||_F (below lambda_max) is caught by the check and the result
    recomputed at the power bound; the allocation-free entry point agrees; the
    other paths refuse the rule."""
    torch = _torch()
    cpa = _lib()
    from oracle import mlp as omlp
    X = synth.as_f32_exact(synth.dense_lowrank(200, 150, rank=5, noise=0.2, seed=78))
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    G = X.T @ X
    fro = math.sqrt(float(np.sum(G * G)))
    tau = 0.3 * math.sqrt(float(np.linalg.eigvalsh(G)[-1]))
    for ev in ("polynomial", "recurrence"):
        m = _model(91, X)
        md = torch.from_numpy(m).cuda()
        y = omlp.forward_model(m, omlp.features(X))[0]
        lam_o = omlp.decide(y, fro, 0.01, 2, 64)[0]
        Y, info = cpa.shrink_dense(Xd, cpa.soft(tau), cpa.Opts(K=20, bound="learned", model=md, eval=ev), info=True)
        print(f"learned {ev}: Lambda gpu {info['Lambda']:.8g} oracle {lam_o:.8g} (y0 {y[0]:.4f})", flush=True)
        assert y[0] < -0.05 and info["Lambda"] == pytest.approx(lam_o, rel=2e-5)
        parity.check(Y.cpu().numpy(), ocpa.cpa_shrink(X, Shrinkage(0, tau), info["Lambda"], 20), TOL32, X,
                      f"learned bound {ev}")
        out = torch.empty_like(Xd)
        cpa.shrink_dense_noalloc(Xd, cpa.soft(tau), cpa.Opts(K=20, bound="learned", model=md, eval=ev), out)
        torch.cuda.synchronize()
        assert torch.equal(out, Y)
        # a network that underestimates: check -> recompute at the power bound
        low = torch.from_numpy(_model(92, X, bias0=-3.0)).cuda()
        Y2, info2 = cpa.shrink_dense(Xd, cpa.soft(tau), cpa.Opts(K=20, bound="learned", model=low, eval=ev,
                                                                 check=True), info=True)
        lam_p, _ = cpa.spectral_bound(Xd, cpa.Opts(K=20))
        print(f"  low network {ev}: fallback {info2['fallback']} Lambda {info2['Lambda']:.8g} power {lam_p:.8g}",
              flush=True)
        assert info2["fallback"] == 1 and info2["Lambda"] == pytest.approx(lam_p, rel=1e-12)
        parity.check(Y2.cpu().numpy(), ocpa.cpa_shrink(X, Shrinkage(0, tau), info2["Lambda"], 20), TOL32, X,
                     f"learned fallback {ev}")
    lam_l, _ = cpa.spectral_bound(Xd, cpa.Opts(K=20, bound="learned", model=md))
    assert lam_l == pytest.approx(lam_o, rel=2e-5)
    with pytest.raises(cpa.CpaError) as e:
        cpa.shrink_csr(3, 3, torch.tensor([0, 1, 2, 3], dtype=torch.int32, device="cuda"),
                       torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda"),
                       torch.ones(3, device="cuda"), cpa.soft(0.1), cpa.Opts(K=5, bound="learned", model=md))
    assert e.value.status == cpa.ERR_UNSUPPORTED
    with pytest.raises(cpa.CpaError) as e:
        cpa.shrink_dense(Xd, cpa.soft(tau), cpa.Opts(K=20, bound="learned"))
    assert e.value.status == cpa.ERR_ARG


@pytest.mark.parametrize("K,damping", [(300, "none"), (512, "lanczos"), (1024, "none")])
def test_polynomial_route_high_orders(K, damping):
    """Orders beyond 256 on the matrix-polynomial route (s = ceil(sqrt K) up to
    32 baby steps): both Gram sides against the oracle."""
    cpa = _lib()
    for m, n in ((150, 100), (90, 140)):
        X = synth.as_f32_exact(synth.dense_lowrank(m, n, rank=5, noise=0.2, seed=7700 + K + m))
        lmax = _gram_lmax(X)
        Lam, tau = 1.01 * lmax, 0.3 * math.sqrt(lmax)
        torch = _torch()
        Y = cpa.shrink_dense(torch.from_numpy(X.astype(np.float32)).cuda(), cpa.soft(tau),
                             cpa.Opts(K=K, Lambda=Lam, eval="polynomial", damping=damping)).cpu().numpy()
        ref = ocpa.cpa_shrink(X, Shrinkage(0, tau), Lam, K, damping=damping)
        parity.check(Y, ref, TOL32, X, f"polynomial K={K} {damping} {m}x{n}")


def test_high_order_on_rpca_frames():
    """K = 360 on the 1024 x 1024 frames (the order at which this workload's CPA
    meets 1e-3 against the exact shrinkage): sampled rows against the oracle."""
    torch = _torch()
    cpa = _lib()
    I, _, _ = synth.rpca_frames()
    X = I.astype(np.float64)
    lam = obound.power_bound(X.T @ X, seed=0)[0]
    Y = cpa.shrink_dense(torch.from_numpy(I).cuda(), cpa.soft(10.0), cpa.Opts(K=360, Lambda=lam)).cpu().numpy()
    rows = np.array([0, 5, 511, 1023])
    parity.check(Y[rows].astype(np.float64), ocpa.cpa_rows(X, Shrinkage(0, 10.0), lam, 360, rows), TOL32,
                 label="frames K=360 sampled rows")
