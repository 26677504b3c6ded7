"""Host-side pieces of the predictor workflow (CPU only): packed segment sums,
the exact soft shrinkage used for labels, and the model blob."""
import math

import numpy as np
import pytest

import synth
from oracle import exact
from oracle import mlp as omlp
from oracle.shrinkage import Shrinkage


def test_segment_errors_match_loop():
    import torch
    from paper_1705_07112_amd import predictor as P
    g = np.random.Generator(np.random.PCG64(1))
    ms = np.array([2, 3, 1, 4], dtype=np.int32)
    ns = np.array([4, 1, 5, 2], dtype=np.int32)
    offs = np.concatenate([[0], np.cumsum(ms * ns)[:-1]]).astype(np.int64)
    tot = int((ms * ns).sum())
    Y = torch.tensor(g.standard_normal(tot), dtype=torch.float32)
    Z = torch.tensor(g.standard_normal(tot), dtype=torch.float32)
    Z[offs[3]:offs[3] + 8] = 0.0          # zero reference: error is the plain norm
    b = P.segment_bounds(torch, ms, ns, offs, "cpu")
    e, r2 = P.rel_errors(torch, Y, Z, b)
    for j in range(4):
        a, c = offs[j], offs[j] + ms[j] * ns[j]
        y, z = Y[a:c].double().numpy(), Z[a:c].double().numpy()
        nz = np.linalg.norm(z)
        ref = np.linalg.norm(y - z) / (nz if nz > 0 else 1.0)
        assert abs(float(e[j]) - ref) <= 1e-12 * max(1.0, ref)
        assert abs(float(r2[j]) - nz * nz) <= 1e-12 * max(1.0, nz * nz)


def test_exact_soft_batch_matches_oracle_svd():
    from paper_1705_07112_amd import predictor as P
    flat, ms, ns, offs, _, noises = synth.patch_groups(batch=40, rank_range=(1, 16), noise_range=(0.05, 0.5),
                                                       seed=5)
    taus = noises * (np.sqrt(ms) + np.sqrt(ns))
    Y = P.exact_soft_batch(flat, ms, ns, offs, taus, threads=2)
    for j in range(40):
        X = flat[offs[j]:offs[j] + ms[j] * ns[j]].reshape(ms[j], ns[j]).astype(np.float64)
        ref = exact.svt_svd(X, Shrinkage(0, float(taus[j]), 0, 0, 0))
        got = Y[offs[j]:offs[j] + ms[j] * ns[j]].reshape(ms[j], ns[j])
        assert np.max(np.abs(got - ref)) <= 1e-5 * max(1.0, np.max(np.abs(ref)))


def test_model_layout_and_blob(tmp_path):
    from paper_1705_07112_amd import predictor as P
    import paper_1705_07112_amd as cpa
    assert cpa.PRED_PARAMS == omlp.N_PARAMS and cpa.PRED_MODEL_FLOATS == omlp.MODEL_FLOATS
    m = P.init_model(3, [1.0, 2.0, 3.0], [0.5, 2.0, 4.0])
    p, mean, inv = omlp.split_model(m)
    assert np.allclose(mean, [1, 2, 3]) and np.allclose(inv, [2.0, 0.5, 0.25])
    W1, b1, W2, b2, W3, b3 = omlp.unpack(p)
    assert np.all(b1 == 0) and np.all(b2 == 0) and np.all(b3 == 0)
    assert np.max(np.abs(W1)) <= 1 / math.sqrt(3) and np.max(np.abs(W2)) <= 1 / 8
    path = str(tmp_path / "model.npz")
    P.save_model(path, m)
    assert np.array_equal(P.load_model(path), m)
    np.savez(path, version=np.int32(99), model=m)
    with pytest.raises(ValueError):
        P.load_model(path)
