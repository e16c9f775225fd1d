"""The band network in float64 -- TEST INFRASTRUCTURE ONLY.

A 32 -> 64 -> 64 -> 1 multilayer perceptron with ReLU (the learned-band
extension; not in the paper) that predicts y = log2(w + 1) for a pair's band
half-width w.  Arithmetic as specified for the GPU kernels: operands of
every matrix product (inputs, weights, activations, back-propagated
gradients) are rounded to bfloat16 (round to nearest even, from float32);
products are accumulated in float32 on the GPU and in float64 here; biases,
ReLU and the loss are float32 / float64.  With round=False the same network
is evaluated without any rounding, which is what the finite-difference pin
checks.

Loss: pinball (quantile) loss with tau, r = target - y,
    l(r) = tau * r  (r >= 0),   (tau - 1) * r  (r < 0),
averaged over the minibatch; dl/dy = -tau if y < target, 1 - tau if
y > target, 0 if equal.  Optimiser: Adam with bias correction on float32
master weights.
"""
from __future__ import annotations

import numpy as np

SIZES = (32, 64, 64, 1)
PARAM_NAMES = ("w1", "b1", "w2", "b2", "w3", "b3")


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest even) via float32; returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    bits = f.view(np.uint32).astype(np.uint64)
    rounded = ((bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return rounded.view(np.float32).astype(np.float64)


def init_params(rng: np.random.Generator) -> dict:
    """He-style initial weights (float32), zero biases."""
    p = {
        "w1": rng.normal(0, np.sqrt(2 / 32), (32, 64)),
        "b1": np.zeros(64),
        "w2": rng.normal(0, np.sqrt(2 / 64), (64, 64)),
        "b2": np.zeros(64),
        "w3": rng.normal(0, np.sqrt(1 / 64), 64),
        "b3": np.zeros(1),
    }
    return {k: v.astype(np.float32) for k, v in p.items()}


def _r(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def forward(params, x, round_=True):
    """Returns y [S] and the intermediates needed by backward."""
    P = {k: np.asarray(v, dtype=np.float64) for k, v in params.items()}
    xb = _r(x, round_)
    z1 = xb @ _r(P["w1"], round_) + P["b1"]
    h1 = np.maximum(z1, 0.0)
    h1b = _r(h1, round_)
    z2 = h1b @ _r(P["w2"], round_) + P["b2"]
    h2 = np.maximum(z2, 0.0)
    h2b = _r(h2, round_)
    y = h2b @ _r(P["w3"], round_) + P["b3"][0]
    cache = dict(xb=xb, z1=z1, h1b=h1b, z2=z2, h2b=h2b, P=P)
    return y, cache


def pinball(y, target, tau):
    r = np.asarray(target, np.float64) - y
    return float(np.mean(np.where(r >= 0, tau * r, (tau - 1) * r)))


def dloss_dy(y, target, tau):
    t = np.asarray(target, np.float64)
    g = np.where(y < t, -tau, np.where(y > t, 1.0 - tau, 0.0))
    return g / len(y)


def backward(cache, gy, round_=True):
    """Gradients of sum_s gy[s] * y[s] with respect to every parameter."""
    P = cache["P"]
    grads = {}
    grads["w3"] = cache["h2b"].T @ gy
    grads["b3"] = np.array([gy.sum()])
    dz2 = gy[:, None] * _r(P["w3"], round_)[None, :] * (cache["z2"] > 0)
    dz2b = _r(dz2, round_)
    grads["w2"] = cache["h1b"].T @ dz2b
    grads["b2"] = dz2.sum(axis=0)
    dh1 = dz2b @ _r(P["w2"], round_).T
    dz1 = dh1 * (cache["z1"] > 0)
    dz1b = _r(dz1, round_)
    grads["w1"] = cache["xb"].T @ dz1b
    grads["b1"] = dz1.sum(axis=0)
    return grads


def adam_step(params, grads, state, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t >= 1); returns new params and state (float64)."""
    newp, news = {}, {}
    for k in PARAM_NAMES:
        g = np.asarray(grads[k], np.float64)
        m, v = state.get(k, (np.zeros_like(g), np.zeros_like(g)))
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        newp[k] = np.asarray(params[k], np.float64) - lr * mh / (np.sqrt(vh) + eps)
        news[k] = (m, v)
    return newp, news


def predict_width(y) -> np.ndarray:
    """Band half-width from the network output y = log2(w + 1)."""
    w = np.ceil(np.exp2(np.asarray(y, np.float64)) - 1.0)
    return np.clip(w, 0, 1 << 20).astype(np.int64)
