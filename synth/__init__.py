"""Seeded synthetic workloads shared by the oracle side and the GPU side.

This module only draws inputs: it holds none of the shrinkage arithmetic
(no Gram, no bound, no coefficients, no recurrence).  Every generator takes an
explicit integer seed and uses numpy's PCG64, so the same call returns
bit-identical arrays on any machine running the same numpy.

Workload shapes follow the paper's applications with synthetic content
(the paper's images and video are not available):

* ``dense_lowrank``  - a rank-r product of N(0,1) factors plus N(0, s^2)
  noise, the single-matrix case (64 x 48, rank 5, s = 0.1).
* ``rpca_frames``    - a background/foreground split as in the paper's video
  experiment (Sec. V-D, frames stacked as columns): a rank-40 product of
  U(0,1) factors min-max normalised to [0,1], plus additive outliers
  U(-1,1) at an exact count of distinct positions.
* ``completion``     - rank-r N(0,1) ground truth with an exact number of
  uniformly sampled observed entries, stored CSR with sorted columns.
* ``patch_groups``   - many small low-rank-plus-noise matrices with uneven
  column counts, packed back to back (row-major), with int64 offsets.
* ``block_matrix_D`` - the structured synthetic matrix of Sec. V-F
  (all-ones minus a block diagonal of 0.5-blocks).
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 1705071120


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def dense_lowrank(m: int = 64, n: int = 48, rank: int = 5, noise: float = 0.1,
                  seed: int = BASE_SEED) -> np.ndarray:
    """X = A @ B + E with A (m x r), B (r x n) ~ N(0,1), E ~ N(0, noise^2); FP64."""
    g = rng(seed)
    a = g.standard_normal((m, rank))
    b = g.standard_normal((rank, n))
    e = noise * g.standard_normal((m, n))
    return a @ b + e


def rpca_frames(m: int = 1024, n: int = 1024, rank: int = 40, outlier_frac: float = 0.05,
                seed: int = BASE_SEED + 1):
    """Returns (I, L0, S0) as float32 arrays, I = L0 + S0.

    L0 = minmax(U V^T), U (m x rank), V (n x rank) ~ U(0,1).  S0 has exactly
    round(outlier_frac * m * n) nonzeros at distinct uniformly drawn positions,
    each ~ U(-1, 1).  Outliers are additive.
    """
    g = rng(seed)
    u = g.random((m, rank))
    v = g.random((n, rank))
    low = u @ v.T
    low = (low - low.min()) / (low.max() - low.min())
    count = int(round(outlier_frac * m * n))
    pos = g.choice(m * n, size=count, replace=False)
    s0 = np.zeros(m * n)
    s0[pos] = g.uniform(-1.0, 1.0, size=count)
    s0 = s0.reshape(m, n)
    l0 = low.astype(np.float32)
    s0 = s0.astype(np.float32)
    return (l0 + s0).astype(np.float32), l0, s0


def completion(m: int = 20000, n: int = 4000, rank: int = 10, frac: float = 0.02,
               seed: int = BASE_SEED + 2):
    """Returns (U, V, rowptr, colidx, vals): ground truth M = U V^T (float32
    factors, N(0,1)), observed set of exactly round(frac*m*n) distinct entries in
    CSR (int32 rowptr/colidx, sorted columns, float32 values of M)."""
    g = rng(seed)
    u = g.standard_normal((m, rank)).astype(np.float32)
    v = g.standard_normal((n, rank)).astype(np.float32)
    count = int(round(frac * m * n))
    flat = np.sort(g.choice(m * n, size=count, replace=False))
    rows = (flat // n).astype(np.int64)
    cols = (flat % n).astype(np.int64)
    vals = np.einsum('ij,ij->i', u[rows].astype(np.float64), v[cols].astype(np.float64)).astype(np.float32)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    return u, v, rowptr, cols.astype(np.int32), vals


def patch_groups(batch: int = 8192, rows: int = 64, ncol_lo: int = 40, ncol_hi: int = 120,
                 rank: int = 4, noise: float = 0.2, seed: int = BASE_SEED + 3,
                 rank_range=None, noise_range=None):
    """Packed batch of row-major float32 matrices X_j = A_j B_j + noise*N(0,1).

    n_j ~ U{ncol_lo..ncol_hi} inclusive.  With ``rank_range=(lo, hi)`` the rank
    of each matrix is drawn U{lo..hi}; with ``noise_range=(lo, hi)`` its noise
    level is drawn U[lo, hi].  Returns (X_packed, m[int32], n[int32],
    offsets[int64], ranks, noises).
    """
    g = rng(seed)
    ncols = g.integers(ncol_lo, ncol_hi + 1, size=batch).astype(np.int32)
    ms = np.full(batch, rows, dtype=np.int32)
    sizes = ms.astype(np.int64) * ncols.astype(np.int64)
    offsets = np.zeros(batch + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    out = np.empty(int(offsets[-1]), dtype=np.float32)
    ranks = np.empty(batch, dtype=np.int32)
    noises = np.empty(batch, dtype=np.float64)
    for j in range(batch):
        r = rank if rank_range is None else int(g.integers(rank_range[0], rank_range[1] + 1))
        s = noise if noise_range is None else float(g.uniform(noise_range[0], noise_range[1]))
        a = g.standard_normal((rows, r))
        b = g.standard_normal((r, int(ncols[j])))
        x = a @ b + s * g.standard_normal((rows, int(ncols[j])))
        out[offsets[j]:offsets[j + 1]] = x.astype(np.float32).ravel()
        ranks[j] = r
        noises[j] = s
    return out, ms, ncols, offsets[:-1].copy(), ranks, noises


def block_smooth(m: int, n: int, rank: int = 3, noise: float = 1e-3, seed: int = BASE_SEED) -> np.ndarray:
    """m x n data that varies only between 8-blocks along its shorter side (the
    side of its Gram), plus N(0, noise^2): a rank-`rank` product whose factor on
    that side is piecewise constant over 8 entries.  Its 8 x 8 block-DCT
    transformed Gram is concentrated on the blocks' DC entries -- the kind of
    input the transform-and-truncate form of the shrinkage is meant for.  FP64."""
    g = rng(seed)
    d = min(m, n)
    smooth = np.repeat(g.standard_normal((max(d // 8, 1), rank)), 8, axis=0)[:d]   # d x rank
    other = g.standard_normal((rank, max(m, n)))
    B = (smooth @ other).T if m >= n else smooth @ other
    return B + noise * g.standard_normal((m, n))


def smooth_lowrank(m: int, n: int, rank: int = 3, freqs: int = 4, noise: float = 1e-3,
                   seed: int = BASE_SEED) -> np.ndarray:
    """m x n data whose factor along its shorter side (the side of its Gram) is a
    sum of the `freqs` lowest cosines cos(pi f (i + 1/2) / d) with N(0, 1)
    weights, times a N(0, 1) factor, plus N(0, noise^2): its DCT-transformed Gram
    is concentrated on the freqs x freqs low-frequency corner.  FP64."""
    g = rng(seed)
    d = min(m, n)
    i = np.arange(d)[:, None] + 0.5
    basis = np.cos(np.pi * np.arange(freqs)[None, :] * i / d)          # d x freqs
    smooth = basis @ g.standard_normal((freqs, rank))                  # d x rank
    other = g.standard_normal((rank, max(m, n)))
    B = (smooth @ other).T if m >= n else smooth @ other
    return B + noise * g.standard_normal((m, n))


def texture(m: int, n: int, terms: int = 3, noise: float = 0.01, hole=None, border: int = 4,
            seed: int = BASE_SEED):
    """A periodic texture stand-in for the inpainting experiment (the paper's
    images are not available): L0 = minmax(sum of `terms` separable products
    cos(2 pi f r / m + a) cos(2 pi g c / n + b), integer f, g in 1..8) + N(0,
    noise^2), clipped to [0, 1] (rank <= 2 terms).  hole = (r0, r1, c0, c1) is the
    missing rectangle (default: the central quarter of each side); border is the
    width of the surrounding frame of observed pixels (m_del).  Returns
    (I, omega, border_mask, L0): I = L0 with the hole set to 0, omega = 1 on the
    observed pixels, FP64 arrays."""
    g = rng(seed)
    r = np.arange(m)[:, None]
    c = np.arange(n)[None, :]
    L = np.zeros((m, n))
    for _ in range(terms):
        f, h = g.integers(1, 9, size=2)
        a, b = g.uniform(0, 2 * np.pi, size=2)
        L += g.uniform(0.5, 1.0) * np.cos(2 * np.pi * f * r / m + a) * np.cos(2 * np.pi * h * c / n + b)
    L = (L - L.min()) / (L.max() - L.min())
    L = np.clip(L + noise * g.standard_normal((m, n)), 0.0, 1.0)
    if hole is None:
        hole = (3 * m // 8, 5 * m // 8, 3 * n // 8, 5 * n // 8)
    r0, r1, c0, c1 = hole
    omega = np.ones((m, n))
    omega[r0:r1, c0:c1] = 0.0
    frame = np.zeros((m, n), dtype=bool)
    frame[max(r0 - border, 0):min(r1 + border, m), max(c0 - border, 0):min(c1 + border, n)] = True
    frame &= omega > 0
    I = L * omega
    return I, omega, frame, L


def block_matrix_D(size: int = 1000, nblocks: int = 10) -> np.ndarray:
    """D = J - blkdiag(0.5 * 1_b 1_b^T, repeated nblocks times), b = size / nblocks."""
    b = size // nblocks
    assert b * nblocks == size
    d = np.ones((size, size))
    for i in range(nblocks):
        d[i * b:(i + 1) * b, i * b:(i + 1) * b] -= 0.5
    return d


def random_orthogonal(n: int, seed: int, reflectors: int | None = None) -> np.ndarray:
    """Product of seeded Householder reflectors (I - 2 v v^T / v^T v); exactly orthogonal
    up to rounding.  Used to rotate test matrices with a known spectrum."""
    g = rng(seed)
    q = np.eye(n)
    for _ in range(n if reflectors is None else reflectors):
        v = g.standard_normal(n)
        q = q - 2.0 * np.outer(q @ v, v) / (v @ v)
    return q


def as_f32_exact(x: np.ndarray) -> np.ndarray:
    """Round once to float32 and widen back: the values both sides consume."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)
