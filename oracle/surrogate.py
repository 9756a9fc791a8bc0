"""Learned surrogate of the synthesis: MLP, Adam, PCA and the ensemble gate
(oracle, test infrastructure only).

The paper motivates data-driven activity models that learn from simulated
spectra (section 1: PCA of line-profile series, neural networks trained on
CCFs; section 5: simulations as a testbed for such methods).  The surrogate
stands in for one synthesised spectrum: an ensemble of MLPs maps the
parameters of a configuration to the normalised PCA coefficients of its
difference from the quiet spectrum.  Nothing here comes from an equation of
the paper; every function is the textbook definition written out in FP64:

  forward    h1 = silu(x W1 + b1), h2 = silu(h1 W2 + b2), y = h2 W3 + b3,
             silu(z) = z / (1 + exp(-z))
  loss       L = mean over batch and outputs of (y - t)^2
  backward   reverse-mode chain rule of the forward definition
  adam       Kingma & Ba (2015), Algorithm 1: m, v moving averages of g and
             g^2, bias corrections 1 - beta^t, step lr m^ / (sqrt(v^) + eps)
  pca        principal axes of centred data = right singular vectors of the
             centred matrix (SVD); projection coef = (d - mean) V
  gate       RV of the ensemble-mean prediction; predicted error = calib x
             sample standard deviation of the members' RVs; fallback when the
             prediction is not below the threshold or a fit failed

``bf16=True`` rounds, as the matrix-core path does, the layer inputs and the
weights of every product to bfloat16 (round to nearest, ties to even) and the
output gradient to bfloat16 before the backward products, and computes the
rest in FP64: the difference to the GPU is then only FP32 accumulation.

Parameters travel as one flat vector per member in the natural layout
W1 [n_in][H], b1 [H], W2 [H][H], b2 [H], W3 [H][O], b3 [O].
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    """Rounds float64 values to the nearest bfloat16 (ties to even), via the
    float32 bit pattern: bfloat16 keeps the top 16 bits of a float32."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def layout(n_in, hidden, n_out):
    """Slices of the flat parameter vector."""
    H, O = hidden, n_out
    sizes = [("W1", (n_in, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, O)), ("b3", (O,))]
    out, o = {}, 0
    for name, shp in sizes:
        n = int(np.prod(shp))
        out[name] = (slice(o, o + n), shp)
        o += n
    return out, o


def unpack(p, n_in, hidden, n_out):
    lay, n = layout(n_in, hidden, n_out)
    p = np.asarray(p, dtype=np.float64)
    assert p.size == n
    return {k: p[s].reshape(shp) for k, (s, shp) in lay.items()}


def pack(d, n_in, hidden, n_out):
    lay, n = layout(n_in, hidden, n_out)
    p = np.zeros(n)
    for k, (s, shp) in lay.items():
        p[s] = np.asarray(d[k], dtype=np.float64).reshape(-1)
    return p


def forward(p, x, n_in, hidden, n_out, bf16=False):
    """Returns y [B][n_out] and the cache for backward."""
    w = unpack(p, n_in, hidden, n_out)
    q = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    a0 = q(x)
    z1 = a0 @ q(w["W1"]) + w["b1"]
    a1 = q(silu(z1))
    z2 = a1 @ q(w["W2"]) + w["b2"]
    a2 = q(silu(z2))
    y = a2 @ q(w["W3"]) + w["b3"]
    return y, dict(a0=a0, z1=z1, a1=a1, z2=z2, a2=a2, w=w)


def loss(y, t):
    d = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    return float(np.mean(d * d))


def backward(p, x, t, n_in, hidden, n_out, bf16=False):
    """Loss and its gradient (flat, natural layout) by the chain rule."""
    y, c = forward(p, x, n_in, hidden, n_out, bf16)
    q = bf16_round if bf16 else (lambda a: a)
    w = c["w"]
    B = y.shape[0]
    dy = 2.0 * (y - np.asarray(t, np.float64)) / (B * n_out)
    dyq = q(dy)
    g = {}
    g["W3"] = c["a2"].T @ dyq
    g["b3"] = dyq.sum(axis=0)
    dz2 = (dyq @ q(w["W3"]).T) * silu_grad(c["z2"])
    dz2q = q(dz2)
    g["W2"] = c["a1"].T @ dz2q
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2q @ q(w["W2"]).T) * silu_grad(c["z1"])
    dz1q = q(dz1)
    g["W1"] = c["a0"].T @ dz1q
    g["b1"] = dz1.sum(axis=0)
    return loss(y, t), pack(g, n_in, hidden, n_out)


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1**t)
    vh = v / (1.0 - beta2**t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def glorot_limit(fan_in, fan_out):
    return np.sqrt(6.0 / (fan_in + fan_out))


def pca_fit(D, k):
    """mean [P], basis V [P][k] (orthonormal columns, decreasing variance)
    and the singular values of the centred data."""
    D = np.asarray(D, dtype=np.float64)
    mean = D.mean(axis=0)
    _, s, vt = np.linalg.svd(D - mean, full_matrices=False)
    return mean, vt[:k].T.copy(), s


def pca_project(D, mean, V):
    return (np.asarray(D, np.float64) - mean) @ np.asarray(V, np.float64)


def pca_reconstruct(coef, mean, V):
    return mean + np.asarray(coef, np.float64) @ np.asarray(V, np.float64).T


def gate(rv_mean, rv_members, status_ok, calib, threshold_kms):
    """rv_members [E][n]; returns (rv, predicted error, fallback flags)."""
    r = np.asarray(rv_members, dtype=np.float64)
    err = calib * r.std(axis=0, ddof=1)
    fb = (~np.asarray(status_ok, bool)) | ~(err < threshold_kms)
    return np.asarray(rv_mean, np.float64), err, fb.astype(np.int32)
