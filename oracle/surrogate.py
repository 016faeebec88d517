"""CPU oracle of the learned pre-screen (test infrastructure only).

What it computes:
  - bf16 / bf16_to_f32: round-to-nearest-even FP32 -> BF16 and back.
  - features: the 256 inputs of the pre-screen for one candidate offspring --
    per-stage processing load of the jobs in each of B = floor(240/S)
    position buckets, normalised by the stage's total load (240 values at
    most), and 16 scalars (parent makespans over the lower bound, cut and swap
    positions over n, operator flags, instance shape).  Integer sums exactly,
    each ratio as one correctly rounded FP32 division, then BF16.
  - target: (C - LB) / LB of an exact decode, FP32.
  - mlp_forward / mlp_backward: the 256-512-512-1 ReLU network in FP64 from
    BF16 operands, MSE loss; mlp_layers exposes each layer separately so a
    GPU layer can be checked from the GPU's own BF16 inputs.
  - adam: the Adam update (Kingma & Ba, ICLR 2015) in FP64.
  - spearman: rank correlation on average ranks (ties share their mean rank).

The pre-screen itself is not in the paper: it ranks candidate children of a
cellular cell (Section 4.2's one-child-per-cell step) so that only the best
candidate is decoded exactly; the exact decode decides every makespan.
"""
from __future__ import annotations

import numpy as np

N_FEATURES = 256
HIDDEN = 512


def bf16(x) -> np.ndarray:
    """FP32 -> BF16 bit pattern (uint16), round to nearest even (finite values)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_to_f32(h) -> np.ndarray:
    h = np.ascontiguousarray(np.asarray(h, dtype=np.uint16))
    return (h.astype(np.uint32) << 16).view(np.float32)


def lower_bound(m, p) -> int:
    m = np.asarray(m, dtype=np.int64)
    p = np.asarray(p, dtype=np.int64)
    stage = max(int(-(-p[:, k].sum() // m[k])) for k in range(p.shape[1]))
    return max(stage, int(p.sum(axis=1).max()))


def features(m, p, child, mk1: int, mk2: int, meta) -> np.ndarray:
    """uint16[256] BF16 features of one candidate.  meta = (p1, p2, crossover,
    a, b, mutation, i, j) as produced by the candidate's draws."""
    m = np.asarray(m, dtype=np.int64)
    p = np.asarray(p, dtype=np.int64)
    n, S = p.shape
    B = 240 // S
    f32 = np.float32
    out = np.zeros(N_FEATURES, dtype=np.float32)
    Pk = p.sum(axis=0)
    load = np.zeros((B, S), dtype=np.int64)
    for t in range(n):
        b = (t * B) // n
        load[b] += p[child[t]]
    for b in range(B):
        for k in range(S):
            out[b * S + k] = f32(load[b, k] * B) / f32(Pk[k])
    LB = lower_bound(m, p)
    E = int(p.sum())
    _, _, cx, a, bb, mx, i, j = [int(v) for v in meta]
    sc = [f32(mk1) / f32(LB), f32(mk2) / f32(LB), f32(a) / f32(n), f32(bb) / f32(n), f32(cx), f32(mx),
          f32(i) / f32(n), f32(j) / f32(n), f32(LB) / f32(E), f32(n) / f32(1000), f32(S) / f32(20),
          f32(int(m.sum())) / f32(6 * S)]
    out[240:240 + len(sc)] = np.array(sc, dtype=np.float32)
    return bf16(out)


def target(makespan: int, LB: int) -> np.float32:
    return np.float32(makespan - LB) / np.float32(LB)


def _relu(x):
    return np.maximum(x, 0.0)


def mlp_layers(x, W1, b1, W2, b2, w3, b3):
    """FP64 forward from given operands (all arrays of values; the caller
    passes BF16-rounded values where the network uses BF16).  Returns
    (z1, z2, y) where layer 2 uses relu(z1) exactly as given."""
    z1 = x.astype(np.float64) @ W1.astype(np.float64) + b1.astype(np.float64)
    h1 = _relu(z1)
    z2 = h1 @ W2.astype(np.float64) + b2.astype(np.float64)
    h2 = _relu(z2)
    y = h2 @ w3.astype(np.float64) + float(b3)
    return z1, z2, y


def mlp_forward(x, W1, b1, W2, b2, w3, b3, bf16_activations: bool = True):
    """FP64 forward; with bf16_activations the hidden activations are rounded
    to BF16 as the network stores them between layers."""
    z1 = x.astype(np.float64) @ W1.astype(np.float64) + b1.astype(np.float64)
    h1 = _relu(z1)
    if bf16_activations:
        h1 = bf16_to_f32(bf16(h1.astype(np.float32))).astype(np.float64)
    z2 = h1 @ W2.astype(np.float64) + b2.astype(np.float64)
    h2 = _relu(z2)
    if bf16_activations:
        h2 = bf16_to_f32(bf16(h2.astype(np.float32))).astype(np.float64)
    y = h2 @ w3.astype(np.float64) + float(b3)
    return dict(z1=z1, h1=h1, z2=z2, h2=h2, y=y)


def mlp_backward(x, t, W1, b1, W2, b2, w3, b3):
    """Gradients of L = mean((y - t)^2) with respect to every parameter, FP64,
    no rounding anywhere (the analytic reference of the training kernels)."""
    x = x.astype(np.float64)
    M = x.shape[0]
    z1 = x @ W1 + b1
    h1 = _relu(z1)
    z2 = h1 @ W2 + b2
    h2 = _relu(z2)
    y = h2 @ w3 + b3
    dy = 2.0 * (y - t) / M
    dw3 = h2.T @ dy
    db3 = dy.sum()
    dz2 = np.outer(dy, w3) * (z2 > 0)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * (z1 > 0)
    dW1 = x.T @ dz1
    db1 = dz1.sum(axis=0)
    loss = float(np.mean((y - t) ** 2))
    return dict(W1=dW1, b1=db1, W2=dW2, b2=db2, w3=dw3, b3=db3, loss=loss)


def mlp_loss(x, t, W1, b1, W2, b2, w3, b3) -> float:
    y = _relu(_relu(x @ W1 + b1) @ W2 + b2) @ w3 + b3
    return float(np.mean((y - t) ** 2))


def adam(param, grad, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), FP64; returns (param, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return param - lr * mh / (np.sqrt(vh) + eps), m, v


def average_ranks(x) -> np.ndarray:
    """Ranks 1..N of x, tied values sharing the mean of the ranks they span."""
    x = np.asarray(x)
    order = np.argsort(x, kind="stable")
    xs = x[order]
    ranks = np.empty(len(x), dtype=np.float64)
    i = 0
    while i < len(xs):
        j = i
        while j + 1 < len(xs) and xs[j + 1] == xs[i]:
            j += 1
        ranks[order[i:j + 1]] = 0.5 * (i + j) + 1.0
        i = j + 1
    return ranks


def spearman(a, b) -> float:
    """Spearman's rho: Pearson correlation of the average ranks (ties share
    their mean rank); NaN when either side is constant."""
    ra = average_ranks(a)
    rb = average_ranks(b)
    ra -= ra.mean()
    rb -= rb.mean()
    den = np.sqrt((ra * ra).sum() * (rb * rb).sum())
    return float((ra * rb).sum() / den) if den > 0 else float("nan")
