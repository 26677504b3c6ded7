"""FP64 reference of the spectral-bound / order predictor network (oracle; test
infrastructure only).

Not from the paper: a small multilayer perceptron 3 -> 64 -> 64 -> 2 with tanh
hidden activations that stands in for the maximum-eigenvalue step of
Algorithm 1 and picks the order per matrix.  Inputs are cheap statistics of X
(m x n) and its Gram G:
    f = (log ||X||_F, log ||G||_F^2, log(m n)),   x = (f - mean) * inv_std
and the outputs are read as y0 ~ log(lambda_max / ||G||_F), y1 ~ log K:
    Lambda = (1 + margin) ||G||_F exp(min(y0, 0)),  K = clamp(ceil(exp(y1)), K_min, K_max).
Training uses a pinball (quantile) loss per output so the predictions err on
the safe side:
    L = mean over samples and outputs of  max(q_o (t - y), (q_o - 1)(t - y)).
Model layout (float, 4554 entries), the same convention as the library's
(re-declared here; nothing is imported from it):
    W1[64][3], b1[64], W2[64][64], b2[64], W3[2][64], b3[2]   (row-major, out x in;
    4546 trainable parameters), mean[3], inv_std[3], 2 unused

Pins: central finite differences of the loss (FP64, <= 1e-6 relative);
a network whose hidden layers are switched off reduces to a linear model whose
gradient has a closed form; the pinball minimiser over constants is the
quantile; features of a matrix built with known singular values match their
closed forms (sum s^2, sum s^4).  Parity: pinned.
"""
from __future__ import annotations

import numpy as np

H = 64
N_IN = 3
N_OUT = 2
SIZES = [(H, N_IN), (H,), (H, H), (H,), (N_OUT, H), (N_OUT,)]
N_PARAMS = sum(int(np.prod(s)) for s in SIZES)
MODEL_FLOATS = N_PARAMS + 8


def split_model(model):
    """(parameters, mean[3], inv_std[3]) of a model buffer."""
    model = np.asarray(model, dtype=np.float64)
    return model[:N_PARAMS], model[N_PARAMS:N_PARAMS + 3], model[N_PARAMS + 3:N_PARAMS + 6]


def features(X):
    """(log ||X||_F, log ||G||_F^2, log(m n)) with G the Gram of the short side."""
    X = np.asarray(X, dtype=np.float64)
    m, n = X.shape
    G = X @ X.T if m <= n else X.T @ X
    return np.array([0.5 * np.log(np.sum(X * X)), np.log(np.sum(G * G)), np.log(float(m) * float(n))])


def forward_model(model, Fraw):
    """Network outputs for raw feature rows: the normalisation stored in the model first."""
    p, mean, inv_std = split_model(model)
    Fraw = np.atleast_2d(np.asarray(Fraw, dtype=np.float64))
    return forward(p, (Fraw - mean) * inv_std)[0]


def decide(y, fro_gram, margin, K_min, K_max):
    """(Lambda, K) from the outputs (y0, y1) of one matrix."""
    Lam = (1.0 + margin) * fro_gram * np.exp(min(float(y[0]), 0.0))
    K = int(np.ceil(np.exp(float(y[1]))))
    return Lam, max(K_min, min(K_max, K))


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = [], 0
    for s in SIZES:
        k = int(np.prod(s))
        out.append(p[o:o + k].reshape(s))
        o += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in parts])


def forward(p, F):
    """F (batch x 3) -> (Y (batch x 2), cache)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    F = np.asarray(F, dtype=np.float64)
    z1 = F @ W1.T + b1
    a1 = np.tanh(z1)
    z2 = a1 @ W2.T + b2
    a2 = np.tanh(z2)
    y = a2 @ W3.T + b3
    return y, (F, a1, a2)


def pinball(y, t, q):
    """Mean pinball loss and its derivative with respect to y (same shape as y)."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64).reshape(1, -1)
    r = t - y
    loss = np.where(r >= 0, q * r, (q - 1.0) * r)
    n = y.size
    dy = np.where(r >= 0, -q, 1.0 - q) / n
    return float(loss.sum() / n), dy


def backward(p, cache, dy):
    """Gradient of the loss with respect to the packed parameters, given dL/dy."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    F, a1, a2 = cache
    gW3 = dy.T @ a2
    gb3 = dy.sum(axis=0)
    da2 = dy @ W3
    dz2 = da2 * (1.0 - a2 * a2)
    gW2 = dz2.T @ a1
    gb2 = dz2.sum(axis=0)
    da1 = dz2 @ W2
    dz1 = da1 * (1.0 - a1 * a1)
    gW1 = dz1.T @ F
    gb1 = dz1.sum(axis=0)
    return pack([gW1, gb1, gW2, gb2, gW3, gb3])


def loss_and_grad(p, F, T, q):
    y, cache = forward(p, F)
    loss, dy = pinball(y, T, q)
    return loss, backward(p, cache, dy)


def init_params(seed: int):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for s in SIZES:
        if len(s) == 2:
            b = 1.0 / np.sqrt(s[1])
            parts.append(g.uniform(-b, b, size=s))
        else:
            parts.append(np.zeros(s))
    return pack(parts)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) with bias correction; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
