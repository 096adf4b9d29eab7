"""Reference multilayer perceptron for the learned bin-width allocation (oracle).

The paper motivates faster, higher-ratio compression for AI workloads
(Sec. 1) but defines no learned component; this network is a project
addition.  It maps per-level coefficient statistics to a log-scale factor of
the level's bin width.  Layers: Linear(F, H) -> ReLU -> Linear(H, H) -> ReLU ->
Linear(H, 1); weights W[out, in] row-major, y = x W^T + b.  Loss: mean squared
error.  Optimiser: Adam with bias correction.

Everything here is float64 and written out step by step so that the GPU
kernels' gradients can be checked against it.
"""
from __future__ import annotations

import numpy as np


def init(seed: int, sizes=(4, 64, 64, 1)):
    """He-normal weights, zero biases; the random draws are the only inputs."""
    rng = np.random.default_rng(seed)
    params = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        W = rng.standard_normal((fo, fi)) * np.sqrt(2.0 / fi)
        b = np.zeros(fo)
        params.append([W, b])
    return params


def forward(params, X):
    """Returns (output (B,1), cache of pre-activations and activations)."""
    acts = [np.asarray(X, dtype=np.float64)]
    pre = []
    h = acts[0]
    for k, (W, b) in enumerate(params):
        z = h @ W.T + b
        pre.append(z)
        h = np.maximum(z, 0.0) if k < len(params) - 1 else z
        acts.append(h)
    return h, (acts, pre)


def mse(pred, target):
    """Loss 1/B sum (pred - target)^2 and its gradient with respect to pred."""
    pred = np.asarray(pred, dtype=np.float64).reshape(-1)
    target = np.asarray(target, dtype=np.float64).reshape(-1)
    r = pred - target
    B = len(r)
    return float(np.dot(r, r) / B), (2.0 / B * r).reshape(-1, 1)


def backward(params, cache, dout):
    """Gradients [[dW, db], ...] for dout = dLoss/doutput (B, 1)."""
    acts, pre = cache
    grads = [None] * len(params)
    g = np.asarray(dout, dtype=np.float64)
    for k in range(len(params) - 1, -1, -1):
        W, _ = params[k]
        if k < len(params) - 1:
            g = g * (pre[k] > 0.0)
        grads[k] = [g.T @ acts[k], g.sum(axis=0)]
        g = g @ W
    return grads


def adam_init(params):
    return [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]


def adam_step(params, grads, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; t counts steps from 1."""
    for k in range(len(params)):
        for j in range(2):
            g = grads[k][j]
            m[k][j] = beta1 * m[k][j] + (1.0 - beta1) * g
            v[k][j] = beta2 * v[k][j] + (1.0 - beta2) * g * g
            mh = m[k][j] / (1.0 - beta1 ** t)
            vh = v[k][j] / (1.0 - beta2 ** t)
            params[k][j] = params[k][j] - lr * mh / (np.sqrt(vh) + eps)
    return params, m, v


# Features of a level (float64): log(rms/tau), log(max|c|/tau), log(count / stream length), l/L.
def level_features(stats, tau):
    """stats: (L+1, 3) rows of (count, sum of squares, max |c|)."""
    stats = np.asarray(stats, dtype=np.float64)
    nlev = stats.shape[0]
    tau = tau if tau > 0 else 1.0
    total = float(np.sum(stats[:, 0])) if nlev else 0.0
    total = total if total > 0 else 1.0
    out = np.zeros((nlev, 4))
    for l in range(nlev):
        cnt, ss, mx = stats[l]
        rms = np.sqrt(ss / (cnt if cnt > 0 else 1.0))
        # the level's share of the stream (not its raw count), so that a network trained on one
        # field size applies to another
        out[l] = [np.log(rms / tau + 1e-30), np.log(mx / tau + 1e-30), np.log((cnt if cnt > 0 else 1.0) / total),
                  l / (nlev - 1) if nlev > 1 else 0.0]
    return out


def level_stats(stream, offsets):
    """(count, sum of squares, max |c|) per level of a coefficient stream (float64)."""
    rows = []
    for l in range(len(offsets) - 1):
        c = np.asarray(stream[offsets[l]:offsets[l + 1]], dtype=np.float64)
        rows.append([len(c), float(np.sum(c * c)), float(np.max(np.abs(c))) if len(c) else 0.0])
    return np.asarray(rows)


def pack(params, mean, std):
    """Flat parameter vector: mean[4], std[4], W1, b1, W2, b2, W3, b3 (row-major)."""
    parts = [np.asarray(mean, dtype=np.float64).ravel(), np.asarray(std, dtype=np.float64).ravel()]
    for W, b in params:
        parts += [np.asarray(W).ravel(), np.asarray(b).ravel()]
    return np.concatenate(parts)


def unpack(flat, sizes=(4, 64, 64, 1)):
    flat = np.asarray(flat, dtype=np.float64)
    F = sizes[0]
    mean, std = flat[:F], flat[F:2 * F]
    pos = 2 * F
    params = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        W = flat[pos:pos + fo * fi].reshape(fo, fi)
        pos += fo * fi
        b = flat[pos:pos + fo]
        pos += fo
        params.append([W, b])
    return params, mean, std


def learned_bins(plain_bins, theta, scale=1.0):
    """b_l = b_plain * exp(scale * clamp(theta_l, -3, 5)); the bound check tries scale 1, then 1/2."""
    t = np.clip(np.asarray(theta, dtype=np.float64).ravel(), -3.0, 5.0)
    return [float(b) * float(np.exp(x * scale)) for b, x in zip(plain_bins, t)]
