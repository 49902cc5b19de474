"""CPU oracle for the learned ordering -- TEST INFRASTRUCTURE ONLY.

Plain numpy, float64: the 8 vertex features, the MLP forward pass and the
analytic gradient of the mean squared error.  Shares no code with the GPU
library; only tests, the smoke check and the benchmark's CPU leg use it.

Features of vertex v (d = degree, N(v) its neighbours):
  0 d        1 log2(1 + d)
  2, 3, 4    min, mean, max of deg(w) over N(v) (0 when d = 0)
  5          sum over N(v) of (deg(w) - 1): paths of length two leaving v
  6          triangle estimate: of 8 sampled wedges (pairs of distinct
             neighbours), the closed fraction times d (d - 1) / 2; sample i
             of v draws h = mix(seed * G + mix(8 v + i + 1)) with splitmix64's
             output mix `mix` and G = 0x9E3779B97F4A7C15, and takes row
             positions a = (h mod 2^32) mod d, b = (h div 2^32) mod (d - 1),
             b + 1 if b >= a
  7          core estimate: the H operator (Lu, Zhou, Zhang and Stanley,
             "The H-index of a network node and its relation to degree and
             coreness", Nature Communications 2016) applied CORE_STEPS
             times to the degrees, where H maps values x to the h-index of
             the neighbours' values (largest h such that at least h
             neighbours w have x(w) >= h); one step is the h-index of the
             neighbour degrees, and the iteration falls to the coreness
MLP: x = (log1p(f) - mean) / std, y = W3 relu(W2 relu(W1 x + b1) + b2) + b3.
Normalisation: mean and population standard deviation of log1p(f) per
feature over the training vertices (variance floored at 1e-12).
Training target of smallest-last position r among n vertices:
log(1 + r) / log(max(n, 2)).
Optimiser: one Adam step (Kingma and Ba, "Adam: a method for stochastic
optimization", 2015, Algorithm 1) with bias-corrected first and second
moment estimates.
"""
from __future__ import annotations

import numpy as np

NF, NH, NPARAM = 8, 64, 4801
CORE_STEPS = 4
W1, B1, W2, B2, W3, B3 = 0, 512, 576, 4672, 4736, 4800
GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def mix(z):
    """splitmix64 output function on uint64 arrays (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def mix_int(z: int) -> int:
    """Same function on Python ints (reference for the array version)."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def wedge_positions(v, d, i, seed):
    """Row positions (a, b) of sample i of vertex v with degree d >= 2."""
    with np.errstate(over="ignore"):
        inner = mix(np.asarray(v, dtype=np.uint64) * np.uint64(8) + np.asarray(i, dtype=np.uint64) + np.uint64(1))
        h = mix(np.uint64(seed) * np.uint64(GAMMA) + inner)
    d = np.asarray(d, dtype=np.uint64)
    a = (h & np.uint64(0xFFFFFFFF)) % d
    b = (h >> np.uint64(32)) % (d - np.uint64(1))
    b = b + (b >= a).astype(np.uint64)
    return a.astype(np.int64), b.astype(np.int64)


def h_operator(row_ptr, col_idx, x) -> np.ndarray:
    """One application of H: for every vertex v, the largest h such that at
    least h neighbours w have x[w] >= h (0 without neighbours).  Sorting each
    row's neighbour values in descending order, h counts the 1-based
    positions p whose value is >= p."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col_idx, dtype=np.int64)
    n = row_ptr.shape[0] - 1
    if col.size == 0:
        return np.zeros(n, dtype=np.int64)
    deg = np.diff(row_ptr)
    src = np.repeat(np.arange(n), deg)
    nv = np.asarray(x, dtype=np.int64)[col]
    order = np.lexsort((-nv, src))
    pos = np.arange(col.size) - row_ptr[src[order]] + 1
    return np.bincount(src[order], weights=(nv[order] >= pos).astype(np.float64), minlength=n).astype(np.int64)


def core_estimate(row_ptr, col_idx, steps: int = CORE_STEPS) -> np.ndarray:
    """H applied `steps` times to the degrees (steps = 0: the degrees)."""
    h = np.diff(np.asarray(row_ptr, dtype=np.int64))
    for _ in range(steps):
        h = h_operator(row_ptr, col_idx, h)
    return h


def features(row_ptr, col_idx, seed: int = 0x5EED, core_steps: int = CORE_STEPS) -> np.ndarray:
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col_idx, dtype=np.int64)
    n = row_ptr.shape[0] - 1
    deg = np.diff(row_ptr)
    src = np.repeat(np.arange(n), deg)
    nd = deg[col].astype(np.float64)
    F = np.zeros((n, NF), dtype=np.float64)
    F[:, 0] = deg
    F[:, 1] = np.log2(1.0 + deg)
    has = deg > 0
    if col.size:
        starts = row_ptr[:-1][has]
        F[has, 2] = np.minimum.reduceat(nd, starts)
        F[has, 4] = np.maximum.reduceat(nd, starts)
        s = np.add.reduceat(nd, starts)
        F[has, 3] = s / deg[has]
        F[has, 5] = s - deg[has]
    F[:, 7] = core_estimate(row_ptr, col, core_steps)
    # wedges
    cand = np.flatnonzero(deg >= 2)
    if cand.size:
        keys = np.sort(src * n + col)
        vv = np.repeat(cand, 8)
        ii = np.tile(np.arange(8), cand.size)
        a, b = wedge_positions(vv, deg[vv], ii, seed)
        wa = col[row_ptr[vv] + a]
        wb = col[row_ptr[vv] + b]
        q = wa * n + wb
        pos = np.searchsorted(keys, q)
        closed = (pos < keys.size) & (keys[np.minimum(pos, keys.size - 1)] == q)
        frac = closed.reshape(-1, 8).sum(axis=1) / 8.0
        d = deg[cand].astype(np.float64)
        F[cand, 6] = frac * 0.5 * d * (d - 1)
    return F


def bf16_round(x: np.ndarray) -> np.ndarray:
    """float32 values rounded to bfloat16 (nearest even), returned as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    u = (np.asarray(bits).astype(np.uint16).astype(np.uint32) << np.uint32(16))
    return u.view(np.float32).astype(np.float64)


def unpack(master, wbf=None):
    """Weights as the forward pass sees them: W from the BF16 copy (or the
    master rounded to BF16), biases from the FP32 master."""
    master = np.asarray(master, dtype=np.float64)
    w = bf16_bits_to_f64(wbf) if wbf is not None else bf16_round(master)
    return (w[W1:B1].reshape(NH, NF), master[B1:W2], w[W2:B2].reshape(NH, NH), master[B2:W3],
            w[W3:B3], master[B3])


def normalise(F, norm):
    norm = np.asarray(norm, dtype=np.float64)
    return (np.log1p(F) - norm[:NF]) / norm[NF:]


def forward(X, params):
    """X: normalised inputs (m, 8).  Returns y and the intermediate values."""
    w1, b1, w2, b2, w3, b3 = params
    z1 = X @ w1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ w2.T + b2
    a2 = np.maximum(z2, 0.0)
    y = a2 @ w3 + b3
    return y, (z1, a1, z2, a2)


def loss(X, t, params):
    y, _ = forward(X, params)
    return float(np.mean((y - t) ** 2))


def grad(X, t, params):
    """Analytic gradient of mean((y - t)^2) w.r.t. (w1, b1, w2, b2, w3, b3),
    packed in the parameter layout; also returns the loss."""
    w1, b1, w2, b2, w3, b3 = params
    y, (z1, a1, z2, a2) = forward(X, params)
    m = X.shape[0]
    dy = 2.0 * (y - t) / m
    g = np.zeros(NPARAM, dtype=np.float64)
    g[W3:B3] = a2.T @ dy
    g[B3] = dy.sum()
    dz2 = np.outer(dy, w3) * (z2 > 0)
    g[W2:B2] = (dz2.T @ a1).ravel()
    g[B2:W3] = dz2.sum(axis=0)
    dz1 = (dz2 @ w2) * (z1 > 0)
    g[W1:B1] = (dz1.T @ X).ravel()
    g[B1:W2] = dz1.sum(axis=0)
    return g, float(np.mean((y - t) ** 2))


def params_from_vector(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[W1:B1].reshape(NH, NF), p[B1:W2], p[W2:B2].reshape(NH, NH), p[B2:W3], p[W3:B3], p[B3])


def keys_from_scores(s):
    """Order-preserving float32 -> uint32 map (negative: all bits flipped;
    non-negative: sign bit set)."""
    u = np.asarray(s, dtype=np.float32).view(np.uint32)
    return np.where(u & np.uint32(0x80000000), ~u, u | np.uint32(0x80000000)).astype(np.uint32)


def feature_sums(F):
    """Per feature: sum of log1p(f) and sum of log1p(f)^2 over the rows of F
    (the statistics the normalisation is fitted from)."""
    L = np.log1p(np.asarray(F, dtype=np.float64))
    return np.concatenate([L.sum(axis=0), (L * L).sum(axis=0)])


def norm_from_sums(sums, count):
    """Mean and population standard deviation per feature from the sums of
    feature_sums over `count` vertices; the variance is floored at 1e-12."""
    sums = np.asarray(sums, dtype=np.float64)
    mean = sums[:NF] / count
    var = np.maximum(sums[NF:] / count - mean * mean, 1e-12)
    return np.concatenate([mean, np.sqrt(var)])


def rank_target(rank):
    """Target of smallest-last position r (0 = coloured first) among n
    vertices: log(1 + r) / log(max(n, 2))."""
    rank = np.asarray(rank, dtype=np.float64)
    n = rank.shape[0]
    return np.log1p(rank) / np.log(max(n, 2))


def adam_step(w, m, v, g, step, lr, beta1, beta2, eps):
    """One Adam step on parameters w with first / second moment estimates m, v
    and gradient g (all float64; step >= 1 counts this step).  Returns the
    new (w, m, v)."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return w - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
