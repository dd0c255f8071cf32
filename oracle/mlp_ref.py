"""FP64 reference of the size-predictor network (CPU, numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Shares no code with the
GPU kernels.

Network: 32 -> 128 -> 128 -> 65, ReLU after the two hidden layers, loss =
mean over the batch and the 65 outputs of the squared error, Adam with
beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias correction (Kingma & Ba).

`quantized=True` mirrors the points where the GPU path rounds operands to
bfloat16 (round to nearest even) before a matrix product: the normalized
inputs, the weights, the hidden activations and the back-propagated
gradients; products and sums are then taken in float64, so the only
difference left to the GPU is its float32 accumulation order.
`quantized=False` is the plain float64 network (used for finite differences).

Parameter packing: W1 [32][128], b1 [128], W2 [128][128], b2 [128],
W3 [128][65], b3 [65].
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

IN, HID, OUT = 32, 128, 65
SHAPES = [("W1", (IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, OUT)), ("b3", (OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def unpack(p: np.ndarray) -> Dict[str, np.ndarray]:
    out, q = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = np.asarray(p[q:q + k], dtype=np.float64).reshape(shape)
        q += k
    return out


def pack(d: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in SHAPES])


def _q(x, quantized):
    return bf16(x) if quantized else np.asarray(x, np.float64)


def normalize(x, mean, std):
    """As the GPU does it, in float32."""
    x = np.asarray(x, np.float32)
    return (x - np.asarray(mean, np.float32)) / np.asarray(std, np.float32)


def forward(p, mean, std, x, quantized=True):
    P = unpack(p)
    xn = normalize(x, mean, std)
    xb = _q(xn, quantized)
    if quantized:
        W1, W2, W3 = (bf16(np.asarray(P[k], np.float32)) for k in ("W1", "W2", "W3"))
    else:
        W1, W2, W3 = P["W1"], P["W2"], P["W3"]
    z1 = xb @ W1 + P["b1"]
    h1 = np.maximum(z1, 0.0)
    h1b = _q(h1, quantized)
    z2 = h1b @ W2 + P["b2"]
    h2 = np.maximum(z2, 0.0)
    h2b = _q(h2, quantized)
    y = h2b @ W3 + P["b3"]
    return {"xb": xb, "W1": W1, "W2": W2, "W3": W3, "h1": h1, "h1b": h1b, "h2": h2,
            "h2b": h2b, "y": y}


def loss_and_grads(p, mean, std, x, t, quantized=True) -> Tuple[float, np.ndarray]:
    f = forward(p, mean, std, x, quantized)
    n = x.shape[0]
    e = f["y"] - np.asarray(t, np.float64)
    loss = float((e * e).sum() / (n * OUT))
    dy = 2.0 * e / (n * OUT)
    dyq = _q(dy, quantized)
    g = {"W3": f["h2b"].T @ dyq, "b3": dy.sum(0)}
    dh2 = (dyq @ f["W3"].T) * (f["h2"] > 0)
    dh2q = _q(dh2, quantized)
    g["W2"] = f["h1b"].T @ dh2q
    g["b2"] = dh2.sum(0)
    dh1 = (dh2q @ f["W2"].T) * (f["h1"] > 0)
    dh1q = _q(dh1, quantized)
    g["W1"] = f["xb"].T @ dh1q
    g["b1"] = dh1.sum(0)
    return loss, pack(g)


def adam(p, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def abs_terms_forward(p, mean, std, x):
    """Per output: the sum of |term| of the last product plus |bias|, and the
    same for the first two layers propagated - the scale that bounds the
    rounding differences of a bf16-operand / fp32-accumulate evaluation."""
    P = unpack(p)
    f = forward(p, mean, std, x, True)
    s1 = np.abs(f["xb"]) @ np.abs(f["W1"]) + np.abs(P["b1"])
    s2 = np.abs(f["h1b"]) @ np.abs(f["W2"]) + np.abs(P["b2"]) + s1 @ np.abs(f["W2"])
    s3 = np.abs(f["h2b"]) @ np.abs(f["W3"]) + np.abs(P["b3"]) + s2 @ np.abs(f["W3"])
    return s3
