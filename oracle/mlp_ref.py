"""CPU reference of the surrogate MLP (numpy).

TEST INFRASTRUCTURE ONLY: used by the test-suite to check the HIP kernels of the
surrogate; the product path never imports it.

The network scores candidate partitionings from per-task split depths and
platform rate features: 32 -> 256 -> 256 -> 256 -> 1, ReLU, mean squared error.
Rounding follows the GPU exactly where the GPU rounds: inputs, weight copies
and hidden activations are bfloat16 (round to nearest even); products are
summed in float64 here (float32 on the GPU); biases and the output are float32.
With ``bf16=False`` every rounding is skipped (used for finite differences).
"""
from __future__ import annotations

import numpy as np

HIDDEN = 256
IN_DIM = 32


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    nan = np.isnan(x)
    if nan.any():
        out = out.copy()
        out[nan] = np.nan
    return out


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """uint16 bit patterns of bf16_round(x)."""
    return (bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)


def param_shapes(in_dim: int = IN_DIM, hidden: int = HIDDEN):
    return [("W1", (in_dim, hidden)), ("b1", (hidden,)), ("W2", (hidden, hidden)), ("b2", (hidden,)),
            ("W3", (hidden, hidden)), ("b3", (hidden,)), ("w4", (hidden,)), ("b4", (1,))]


def unflatten(flat: np.ndarray, in_dim: int = IN_DIM, hidden: int = HIDDEN):
    out, o = {}, 0
    for name, shp in param_shapes(in_dim, hidden):
        n = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    assert o == len(flat)
    return out


def flatten(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k, _ in param_shapes(
        p["W1"].shape[0], p["W1"].shape[1])])


def _r(x, bf16):
    return bf16_round(np.asarray(x, np.float32)).astype(np.float64) if bf16 else np.asarray(x, np.float64)


def forward(p, X: np.ndarray, bf16: bool = True):
    """Returns (y, cache).  X: [n, in_dim]."""
    W1, W2, W3, w4 = (_r(p[k], bf16) for k in ("W1", "W2", "W3", "w4"))
    b1, b2, b3, b4 = (np.asarray(p[k], np.float64) for k in ("b1", "b2", "b3", "b4"))
    x = _r(X, bf16)
    h1 = _r(np.maximum(x @ W1 + b1, 0.0), bf16)
    h2 = _r(np.maximum(h1 @ W2 + b2, 0.0), bf16)
    h3 = _r(np.maximum(h2 @ W3 + b3, 0.0), bf16)
    y = h3 @ w4 + b4[0]
    if bf16:
        y = y.astype(np.float32).astype(np.float64)
    return y, (x, h1, h2, h3, W1, W2, W3, w4)


def loss_and_grad(p, X: np.ndarray, t: np.ndarray, bf16: bool = True):
    """Mean squared error and the gradient of every parameter (same rounding points as the GPU)."""
    y, (x, h1, h2, h3, W1, W2, W3, w4) = forward(p, X, bf16)
    n = X.shape[0]
    t = np.asarray(t, np.float64)
    loss = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / n
    if bf16:
        dy = dy.astype(np.float32).astype(np.float64)
    g = {}
    g["w4"] = h3.T @ dy
    g["b4"] = np.array([dy.sum()])
    dz3 = _r(np.outer(dy, w4) * (h3 > 0), bf16)
    g["W3"] = h2.T @ dz3
    g["b3"] = dz3.sum(axis=0)
    dz2 = _r((dz3 @ W3.T) * (h2 > 0), bf16)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = _r((dz2 @ W2.T) * (h1 > 0), bf16)
    g["W1"] = x.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return loss, g


def adam(p, g, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (Kingma and Ba, 2015) in float64 on float32 master weights."""
    out = {}
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        out[k] = (p[k] - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32).astype(np.float64)
    return out


def init_params(seed: int, in_dim: int = IN_DIM, hidden: int = HIDDEN):
    """He-uniform weights, zero biases (float32 values)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in param_shapes(in_dim, hidden):
        if name.startswith("b"):
            p[name] = np.zeros(shp)
        else:
            fan_in = shp[0]
            lim = np.sqrt(6.0 / fan_in)
            p[name] = rng.uniform(-lim, lim, shp).astype(np.float32).astype(np.float64)
    return p
