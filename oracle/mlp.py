"""FP64 reference of the learned-k network (test infrastructure only).

The network picks a neighbour-list size per cell: 12 features -> 64 -> 64 ->
7 logits (ReLU), one logit per list-size bucket {8, 12, 16, 24, 32, 48, 64}.
Training minimises the mean softmax cross-entropy against the bucket each
cell actually needed (the least bucket >= the list size at which the
security-radius test certified the cell).

The GPU kernels run the products in BF16 with FP32 accumulation.  This
reference evaluates the same formulas in float64 and, when ``bf16=True``,
rounds to bfloat16 (round to nearest even) at exactly the points where the
kernels do: the standardised inputs, the weights, the hidden activations
after ReLU, and the backward signals entering each product.  With
``bf16=False`` it is the plain FP64 network, whose gradient is pinned by
central finite differences.

Parameter layout (flat, 5447 values): W1[64][12] b1[64] W2[64][64] b2[64]
W3[7][64] b3[7].
"""
from __future__ import annotations

import numpy as np

NF, NH, NO = 12, 64, 7
SHAPES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NO, NH)), ("b3", (NO,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16(x: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even), as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + size], dtype=np.float64).reshape(shape)
        o += size
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(theta, x, mean, std, bf16_points=True):
    """Logits [B,7] and the intermediates the backward pass needs."""
    p = unpack(theta)
    r = bf16 if bf16_points else (lambda v: np.asarray(v, dtype=np.float64))
    xs = r((np.asarray(x, np.float64) - mean) / std)
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    z1 = xs @ W1.T + p["b1"]
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ W2.T + p["b2"]
    h2 = r(np.maximum(z2, 0.0))
    z3 = h2 @ W3.T + p["b3"]
    return z3, dict(xs=xs, W1=W1, W2=W2, W3=W3, z1=z1, h1=h1, z2=z2, h2=h2)


def loss_and_grad(theta, x, labels, mean, std, bf16_points=True):
    """Mean softmax cross-entropy over the batch and its gradient (flat)."""
    r = bf16 if bf16_points else (lambda v: np.asarray(v, dtype=np.float64))
    z3, c = forward(theta, x, mean, std, bf16_points)
    B = z3.shape[0]
    z = z3 - z3.max(axis=1, keepdims=True)
    e = np.exp(z)
    prob = e / e.sum(axis=1, keepdims=True)
    y = np.asarray(labels, dtype=np.int64)
    loss = float(np.mean(-np.log(prob[np.arange(B), y])))
    g3 = prob.copy()
    g3[np.arange(B), y] -= 1.0
    g3 /= B
    g3r = r(g3)
    dW3 = g3r.T @ c["h2"]
    db3 = g3.sum(axis=0)
    g2 = (g3r @ c["W3"]) * (c["z2"] > 0)
    g2r = r(g2)
    dW2 = g2r.T @ c["h1"]
    db2 = g2.sum(axis=0)
    g1 = (g2r @ c["W2"]) * (c["z1"] > 0)
    g1r = r(g1)
    dW1 = g1r.T @ c["xs"]
    db1 = g1.sum(axis=0)
    return loss, pack(dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3))


def choose(theta, x, mean, std, tau, bf16_points=True):
    """Least bucket b with P(label <= b) >= tau."""
    z3, _ = forward(theta, x, mean, std, bf16_points)
    z = z3 - z3.max(axis=1, keepdims=True)
    prob = np.exp(z)
    prob /= prob.sum(axis=1, keepdims=True)
    cdf = np.cumsum(prob, axis=1)
    ok = cdf >= tau
    ok[:, -1] = True
    return np.argmax(ok, axis=1)


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns the new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (the GPU model is given these explicitly)."""
    rng = np.random.default_rng(seed)
    parts = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shape[1])
            parts[name] = rng.uniform(-lim, lim, shape)
        else:
            parts[name] = np.zeros(shape)
    return pack(parts)
