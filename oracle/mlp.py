"""float64 reference of the ladder-predicting MLP (test oracle).

Network: 6 features -> 128 -> 128 -> 128 -> 32, GELU (exact erf form) after
the three hidden layers.  Outputs z[0..30] are logits of the 31 increments
of log Gamma along the ladder, z[31] predicts the log of the total exchange
barrier.  With `bf16=True` every GEMM operand is rounded to bfloat16
(round to nearest even) where the GPU rounds it; accumulation, bias, GELU,
loss and the optimiser stay in full precision.

Parameter layout (flat): W1[6][128], b1[128], W2[128][128], b2[128],
W3[128][128], b3[128], W4[128][32], b4[32]; W[k][n] multiplies input k into
output n.  38 048 numbers.

Decode: log Gamma_i = log Gmin + (log Gmax - log Gmin) * sum_{l<i} softmax(z)_l
for i = 0..31, a monotone ladder with the given end points (zero logits give
the geometric ladder).  Predicted acceptance per gap: 1 - exp(z[31]) / 31.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

SIZES = [(6, 128), (128, 128), (128, 128), (128, 32)]
N_PARAMS = sum(k * n + n for k, n in SIZES)
N_INC = 31


def split(params: np.ndarray) -> List[Tuple[np.ndarray, np.ndarray]]:
    out, off = [], 0
    for k, n in SIZES:
        W = params[off:off + k * n].reshape(k, n)
        off += k * n
        b = params[off:off + n]
        off += n
        out.append((W, b))
    assert off == params.size == N_PARAMS
    return out


def to_bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def gelu(x):
    from scipy.special import erf
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)


def forward(params: np.ndarray, X: np.ndarray, bf16: bool = False) -> Dict:
    rnd = to_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    h = np.asarray(X, dtype=np.float64)
    cache = {"inputs": [], "pre": []}
    layers = split(np.asarray(params, dtype=np.float64))
    for li, (W, b) in enumerate(layers):
        hin = rnd(h)
        cache["inputs"].append(hin)
        pre = hin @ rnd(W) + b
        cache["pre"].append(pre)
        h = gelu(pre) if li < len(layers) - 1 else pre
    cache["out"] = h
    return cache


def softmax(z):
    m = z.max(axis=-1, keepdims=True)
    e = np.exp(z - m)
    return e / e.sum(axis=-1, keepdims=True)


def loss_and_grad(z: np.ndarray, target_inc: np.ndarray, target_logL: np.ndarray):
    """Mean over the batch of KL(target || softmax(z[:31])) + (z[31]-logL)^2,
    and its gradient with respect to z."""
    B = z.shape[0]
    s = softmax(z[:, :N_INC])
    t = target_inc
    with np.errstate(divide="ignore", invalid="ignore"):
        tl = np.where(t > 0, t * (np.log(np.where(t > 0, t, 1.0)) - np.log(s)), 0.0)
    d = z[:, N_INC] - target_logL
    loss = (tl.sum(axis=1) + d * d).mean()
    g = np.zeros_like(z)
    g[:, :N_INC] = (s * t.sum(axis=1, keepdims=True) - t) / B
    g[:, N_INC] = 2.0 * d / B
    return float(loss), g


def backward(params: np.ndarray, cache: Dict, dout: np.ndarray, bf16: bool = False) -> np.ndarray:
    rnd = to_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    layers = split(np.asarray(params, dtype=np.float64))
    grads = []
    g = np.asarray(dout, dtype=np.float64)
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        if li < len(layers) - 1:
            g = g * gelu_grad(cache["pre"][li])
        gW = cache["inputs"][li].T @ rnd(g)
        gb = g.sum(axis=0)
        grads.append((gW, gb))
        if li > 0:
            g = rnd(g) @ rnd(W).T
    flat = []
    for gW, gb in reversed(grads):
        flat += [gW.reshape(-1), gb]
    return np.concatenate(flat)


def adam(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def decode(z: np.ndarray, gmin, gmax) -> np.ndarray:
    """[B][32] ladder from outputs z [B][32] and end points [B]."""
    s = softmax(np.asarray(z, dtype=np.float64)[:, :N_INC])
    c = np.concatenate([np.zeros((s.shape[0], 1)), np.cumsum(s, axis=1)], axis=1)
    lo = np.log(np.asarray(gmin, dtype=np.float64))[:, None]
    hi = np.log(np.asarray(gmax, dtype=np.float64))[:, None]
    return np.exp(lo + (hi - lo) * c)


def predicted_acceptance(z: np.ndarray) -> np.ndarray:
    return 1.0 - np.exp(np.asarray(z, dtype=np.float64)[:, N_INC]) / N_INC


def init_params(seed: int = 0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for k, n in SIZES:
        parts.append(rng.normal(0.0, math.sqrt(2.0 / k), size=k * n))
        parts.append(np.zeros(n))
    return np.concatenate(parts)
