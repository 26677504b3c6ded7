"""Split-precision recurrence (bf16 hi + lo, three products, FP32 accumulation)
against the FP64 oracle.  Bar: relative Frobenius error <= 1e-3 (the
split-precision tolerance); the measured error is printed and is typically
1e-6..1e-5."""
import math

import numpy as np
import pytest

import synth
from tests import parity
from oracle import bound as obound
from oracle import cpa as ocpa
from oracle import metrics
from oracle.shrinkage import Shrinkage

pytestmark = pytest.mark.gpu

TOL_SPLIT = 1e-3


def _case(m, n, K, kind, seed, ld=None, ev="auto"):
    import torch
    import paper_1705_07112_amd as cpa
    X = synth.as_f32_exact(synth.dense_lowrank(m, n, rank=min(4, m, n), noise=0.2, seed=seed))
    G = X.T @ X if m >= n else X @ X.T
    lmax = float(np.linalg.eigvalsh(G)[-1])
    Lam, tau = 1.01 * lmax, 0.4 * math.sqrt(lmax)
    if kind == 0:
        sh_o, sh_c = Shrinkage(0, tau), cpa.soft(tau)
    elif kind == 1:
        sh_o, sh_c = Shrinkage(1, tau), cpa.hard(tau)
    else:
        wc, ws = 0.3 * tau * tau, 0.05 * lmax
        sh_o, sh_c = Shrinkage(3, 0.0, wc, ws, 1e-3), cpa.weighted_fn(wc, ws, 1e-3)
    ld = ld or n
    buf = torch.zeros(m * ld, dtype=torch.float32)
    buf.view(m, ld)[:, :n] = torch.from_numpy(X.astype(np.float32))
    Xd = buf.cuda().view(m, ld)[:, :n]
    Y = cpa.shrink_dense(Xd, sh_c, cpa.Opts(K=K, Lambda=Lam, precision="bf16x3", eval=ev)).cpu().numpy()
    err, _ = parity.check(Y, ocpa.cpa_shrink(X, sh_o, Lam, K), TOL_SPLIT, X,
                          f"bf16x3 m={m} n={n} K={K} kind={kind} eval={ev}")
    return err


@pytest.mark.parametrize("shape", [(64, 48), (130, 70), (70, 130), (1, 5), (5, 1), (129, 129), (300, 1100)])
def test_split_shapes(shape):
    _case(*shape, 16, 0, 9000 + shape[0] * 3 + shape[1])


@pytest.mark.parametrize("K", [1, 2, 30])
@pytest.mark.parametrize("kind", [0, 1, 2])
def test_split_orders_and_kinds(K, kind):
    _case(96, 80, K, kind, 9100 + K)


def test_split_strided():
    _case(77, 45, 12, 0, 9201, ld=53)


def test_split_full_size_rpca_matrix():
    import torch
    import paper_1705_07112_amd as cpa
    I, _, _ = synth.rpca_frames()
    X = I.astype(np.float64)
    lam = obound.power_bound(X.T @ X, seed=0)[0]
    Y = cpa.shrink_dense(torch.from_numpy(I).cuda(), cpa.soft(10.0),
                         cpa.Opts(K=30, Lambda=lam, precision="bf16x3")).cpu().numpy()
    rows = np.array([0, 1, 63, 64, 500, 1023])
    parity.check(Y[rows].astype(np.float64), ocpa.cpa_rows(X, Shrinkage(0, 10.0), lam, 30, rows), TOL_SPLIT,
                 label="bf16x3 full size sampled rows")


@pytest.mark.parametrize("ev", ["recurrence", "polynomial"])
@pytest.mark.parametrize("shape", [(130, 70), (70, 130), (129, 129)])
def test_split_both_evaluation_routes(ev, shape):
    _case(*shape, 30, 0, 9300 + shape[0] + shape[1], ev=ev)
