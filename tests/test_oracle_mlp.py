"""Pins for the FP64 predictor-network oracle: central finite differences and a
closed-form linear case."""
import numpy as np
import pytest

from oracle import mlp


def test_param_count():
    assert mlp.N_PARAMS == 4546


def test_gradient_matches_central_differences():
    g = np.random.Generator(np.random.PCG64(3))
    p = mlp.init_params(5) + 0.1 * g.standard_normal(mlp.N_PARAMS)
    F = g.standard_normal((17, 3))
    T = g.standard_normal((17, 2))
    q = np.array([0.99, 0.9])
    loss, grad = mlp.loss_and_grad(p, F, T, q)
    idx = g.choice(mlp.N_PARAMS, size=60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, F, T, q)[0] - mlp.loss_and_grad(p - e, F, T, q)[0]) / (2 * h)
        assert fd == pytest.approx(grad[i], rel=1e-6, abs=1e-9)


def test_linear_closed_form():
    # zero hidden weights: a1 = a2 = 0 except biases; make tanh layers pass a constant,
    # then y = W3 tanh(b2) + b3 and dL/db3 = sum dy, dL/dW3 = dy^T tanh(b2)
    g = np.random.Generator(np.random.PCG64(4))
    W1, b1, W2, b2, W3, b3 = mlp.unpack(np.zeros(mlp.N_PARAMS))
    b2 = g.standard_normal(64) * 0.5
    W3 = g.standard_normal((2, 64))
    b3 = g.standard_normal(2)
    p = mlp.pack([W1, b1, W2, b2, W3, b3])
    F = g.standard_normal((9, 3))
    T = g.standard_normal((9, 2))
    q = np.array([0.7, 0.3])
    y, _ = mlp.forward(p, F)
    a2 = np.tanh(b2)
    assert np.max(np.abs(y - (a2 @ W3.T + b3))) < 1e-14
    r = T - y
    dy = np.where(r >= 0, -q, 1 - q) / y.size
    _, grad = mlp.loss_and_grad(p, F, T, q)
    gp = mlp.unpack(grad)
    assert np.max(np.abs(gp[5] - dy.sum(axis=0))) < 1e-14
    assert np.max(np.abs(gp[4] - dy.T @ np.tile(a2, (9, 1)))) < 1e-13
    # W2 gradient is zero because a1 = tanh(0) = 0
    assert np.max(np.abs(gp[2])) == 0.0


def test_pinball_quantile_property():
    # minimiser of the pinball loss over a constant is the q-quantile of the targets
    t = np.linspace(0, 1, 1001).reshape(-1, 1)
    cands = np.linspace(0, 1, 2001)
    for q in (0.1, 0.5, 0.9, 0.99):
        losses = [mlp.pinball(np.full_like(t, c), t, np.array([q]))[0] for c in cands]
        assert cands[int(np.argmin(losses))] == pytest.approx(q, abs=2e-3)


def test_adam_matches_definition():
    p = np.array([1.0, -2.0])
    g = np.array([0.5, 0.25])
    p1, m1, v1 = mlp.adam_step(p, g, np.zeros(2), np.zeros(2), 1, 0.1)
    # first step with bias correction moves every coordinate by lr * sign(g)
    assert np.max(np.abs(p1 - (p - 0.1 * np.sign(g)))) < 1e-6


def test_features_closed_form():
    # X = Q1 diag(s) Q2^T with known singular values: ||X||_F^2 = sum s^2, ||G||_F^2 = sum s^4
    import synth
    s = np.array([3.0, 2.0, 0.5, 0.25])
    for (m, n) in ((4, 7), (7, 4)):
        Q1 = synth.random_orthogonal(m, seed=11)[:, :4]
        Q2 = synth.random_orthogonal(n, seed=12)[:, :4]
        X = Q1 @ np.diag(s) @ Q2.T
        f = mlp.features(X)
        assert f[0] == pytest.approx(0.5 * np.log(np.sum(s ** 2)), abs=1e-13)
        assert f[1] == pytest.approx(np.log(np.sum(s ** 4)), abs=1e-13)
        assert f[2] == pytest.approx(np.log(m * n), abs=1e-15)


def test_decide_rule():
    # y0 above zero never raises Lambda past (1 + margin)||G||_F; K clamps at both ends
    assert mlp.decide([0.7, np.log(10.2)], 2.0, 0.01, 2, 64) == (pytest.approx(2.02), 11)
    assert mlp.decide([np.log(0.5), np.log(100.0)], 2.0, 0.0, 2, 64) == (pytest.approx(1.0), 64)
    assert mlp.decide([-1.0, np.log(0.5)], 1.0, 0.0, 4, 64)[1] == 4


def test_forward_model_applies_normalisation():
    g = np.random.Generator(np.random.PCG64(9))
    p = mlp.init_params(2)
    mean = np.array([1.0, -2.0, 3.0])
    inv = np.array([0.5, 2.0, 0.25])
    model = np.concatenate([p, mean, inv, [0.0, 0.0]])
    F = g.standard_normal((5, 3))
    y = mlp.forward_model(model, F)
    assert np.max(np.abs(y - mlp.forward(p, (F - mean) * inv)[0])) == 0.0
    # the identity normalisation is a no-op
    model2 = np.concatenate([p, np.zeros(3), np.ones(3), [0.0, 0.0]])
    assert np.max(np.abs(mlp.forward_model(model2, F) - mlp.forward(p, F)[0])) == 0.0
