"""Reference MLP of the learned refinement indicator -- TEST INFRASTRUCTURE ONLY.

A 16 -> 64 -> 64 -> 1 perceptron with ReLU hidden layers and a linear
output, written in plain numpy float64.  With emulate_bf16 the layer inputs,
the weights and the hidden activations are rounded to bfloat16 (round to
nearest even, from their float32 value) at the points the GPU kernels round
them; everything else is exact float64 here (the kernels accumulate in
float32).  Loss: mean squared error.  Optimiser: Adam (Kingma & Ba 2015).

Packed parameter order (float32 on the GPU): W1[64,16], b1[64], W2[64,64],
b2[64], W3[1,64], b3[1].
"""
from __future__ import annotations

import numpy as np

SIZES = [("W1", (64, 16)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (1, 64)),
         ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) via the float32 value."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def unpack(flat):
    out, o = {}, 0
    for name, shp in SIZES:
        k = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def init(seed: int = 0) -> np.ndarray:
    """Seeded initial weights (the shared input generator's)."""
    import z4c_inputs
    return z4c_inputs.mlp_init(seed)


def forward(flat, X, emulate_bf16: bool = True):
    """X: (B, 16).  Returns y (B,) and the cache the backward pass needs."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(flat)
    x = r(X)
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    a1 = x @ W1.T + p["b1"]
    h1 = r(np.maximum(a1, 0.0))
    a2 = h1 @ W2.T + p["b2"]
    h2 = r(np.maximum(a2, 0.0))
    y = (h2 @ W3.T)[:, 0] + p["b3"][0]
    return y, dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2, W1=W1, W2=W2, W3=W3)


def loss_and_grad(flat, X, t, emulate_bf16: bool = True):
    """MSE loss and its gradient with respect to the packed parameters
    (through the rounded weights, as if rounding were the identity)."""
    y, c = forward(flat, X, emulate_bf16)
    B = X.shape[0]
    d = y - t
    loss = float(np.mean(d * d))
    dy = 2.0 * d / B
    g = {}
    g["W3"] = dy[None, :] @ c["h2"]
    g["b3"] = np.array([dy.sum()])
    da2 = (dy[:, None] @ c["W3"]) * (c["a2"] > 0)
    g["W2"] = da2.T @ c["h1"]
    g["b2"] = da2.sum(0)
    da1 = (da2 @ c["W2"]) * (c["a1"] > 0)
    g["W1"] = da1.T @ c["x"]
    g["b1"] = da1.sum(0)
    return loss, pack(g)


def adam(flat, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v
