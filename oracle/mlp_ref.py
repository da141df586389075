"""Reference (fp64, numpy) of the learned batch-order proposal -- TEST
INFRASTRUCTURE ONLY (imported by the tests and nowhere in the product path).

The proposal is not part of the paper; it is the plain definition of a small
network written out:

* features: the block's reliabilities |LLR_i| sorted ascending (the ordered
  reliability curve the paper studies in Sec. III-A), scaled by 1/8 and rounded
  to BF16;
* network: logits = W3 h2 + b3, h2 = bf16(relu(W2 h1 + b2)),
  h1 = bf16(relu(W1 x + b1)), x in R^128, h1, h2 in R^256, logits in R^64; the
  weights are used rounded to BF16, the biases in full precision;
* loss: mean softmax cross-entropy against the label = index of the batch of 64
  patterns that holds the plain decoder's first hit;
* gradients: the analytic backward of that network, the BF16 rounding of the
  activations taken as identity (straight-through);
* update: Adam (Kingma and Ba, 2015) with bias correction;
* order: batches sorted by decreasing logit, ties to the lower index.

Parameter layout (flat): W1 [256 x 128], b1 [256], W2 [256 x 256], b2 [256],
W3 [64 x 256], b3 [64]  (row-major, output x input), 115,264 values.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 128, 256, 64
SHAPES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (OUT, HID)), ("b3", (OUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)
FEATURE_SCALE = 0.125


def unflatten(flat: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = flat[o:o + size].reshape(shape)
        o += size
    return out


def flatten(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16_round(x) -> np.ndarray:
    """Round float32 values to the nearest BF16 (ties to even); returns float32."""
    x = np.asarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    nan = np.isnan(x)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    return np.where(nan, np.float32(np.nan), out).astype(np.float32)


def bf16_bits(x) -> np.ndarray:
    """BF16 bit patterns (uint16) of bf16_round(x)."""
    return (bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32)


def features(llr: np.ndarray) -> np.ndarray:
    """Sorted |LLR| (ascending) / 8, BF16-rounded: [N, n] -> [N, n] float32."""
    a = np.sort(np.abs(np.asarray(llr, dtype=np.float32)), axis=1)
    return bf16_round(a * np.float32(FEATURE_SCALE))


def forward(params: np.ndarray, x: np.ndarray, round_activations: bool = True, round_weights: bool = True):
    """Returns (logits [N,64] fp64, cache).  x: [N,128] (BF16 values).
    round_weights / round_activations = False give the same network in exact
    (fp64) arithmetic, the form in which finite differences of the loss apply."""
    p = unflatten(np.asarray(params, dtype=np.float64))
    if round_weights:
        W = {k: bf16_round(p[k]).astype(np.float64) for k in ("W1", "W2", "W3")}
    else:
        W = {k: p[k] for k in ("W1", "W2", "W3")}
    q = (lambda a: bf16_round(a).astype(np.float64)) if round_activations else (lambda a: a)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W["W1"].T + p["b1"]
    h1 = q(np.maximum(z1, 0.0))
    z2 = h1 @ W["W2"].T + p["b2"]
    h2 = q(np.maximum(z2, 0.0))
    logits = h2 @ W["W3"].T + p["b3"]
    return logits, dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2, W=W)


def loss_and_dlogits(logits: np.ndarray, labels: np.ndarray):
    """Mean softmax cross-entropy and its gradient w.r.t. the logits."""
    z = logits - logits.max(axis=1, keepdims=True)
    e = np.exp(z)
    s = e / e.sum(axis=1, keepdims=True)
    N = logits.shape[0]
    lse = np.log(e.sum(axis=1)) + logits.max(axis=1)
    loss = float(np.mean(lse - logits[np.arange(N), labels]))
    d = s.copy()
    d[np.arange(N), labels] -= 1.0
    return loss, d / N


def backward(params: np.ndarray, x: np.ndarray, labels: np.ndarray, round_activations: bool = True,
             round_weights: bool = True):
    """Returns (loss, flat gradient fp64)."""
    logits, c = forward(params, x, round_activations, round_weights)
    loss, dl = loss_and_dlogits(logits, labels)
    W = c["W"]
    g = {}
    g["b3"] = dl.sum(axis=0)
    g["W3"] = dl.T @ c["h2"]
    dz2 = (dl @ W["W3"]) * (c["z2"] > 0)
    g["b2"] = dz2.sum(axis=0)
    g["W2"] = dz2.T @ c["h1"]
    dz1 = (dz2 @ W["W2"]) * (c["z1"] > 0)
    g["b1"] = dz1.sum(axis=0)
    g["W1"] = dz1.T @ c["x"]
    return loss, flatten(g)


def adam(w, m, v, g, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (w, m, v)."""
    w, m, v, g = (np.asarray(a, dtype=np.float64) for a in (w, m, v, g))
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def order(logits: np.ndarray) -> np.ndarray:
    """Batches by decreasing logit, ties to the lower index: [N,64] -> uint8 [N,64]."""
    return np.argsort(-np.asarray(logits, dtype=np.float64), axis=1, kind="stable").astype(np.uint8)


def init(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (fp32 masters)."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shape[1])
            d[name] = rng.uniform(-lim, lim, shape)
        else:
            d[name] = np.zeros(shape)
    return flatten(d).astype(np.float32)
