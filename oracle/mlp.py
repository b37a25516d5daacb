"""FP64 oracle of the learned warm start -- TEST INFRASTRUCTURE ONLY.

A per-contact MLP predicts the iteration-0 multiplier of each row of A_0
(the paper is silent on warm starts; the projected-gradient LCP of Eq. cqpp
accepts any start).  Network, following the written definition:

    z = w3 . GELU(W2 GELU(W1 x + b1) + b2) + b3,   gamma0 = softplus(z) * lam_scale
    GELU(t) = t Phi(t) = 0.5 t (1 + erf(t / sqrt 2))        (exact form)

x = standardised features (8), hidden width 128.  Loss: mean over the batch
of (softplus(z) - y)^2 with y = target multiplier / lam_scale.  Adam.

`emulate=True` rounds to bfloat16 exactly the operands that the GPU kernels
feed to the matrix cores (inputs, W1, the first hidden layer, W2 in the
forward pass; the back-propagated pre-activation gradients in the backward
pass); everything else stays FP64.  Parameters are a flat vector in the
order W1 (128x8, row = output unit), b1, W2 (128x128), b2, w3, b3.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

H = 128
F = 8
SIZES = [("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", ())]
NPARAM = sum(int(np.prod(s)) if s else 1 for _, s in SIZES)  # 17793


def unpack(flat):
    P, o = {}, 0
    for name, shp in SIZES:
        k = int(np.prod(shp)) if shp else 1
        P[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(shp) if shp else float(flat[o])
        o += k
    return P


def pack(P):
    return np.concatenate([np.atleast_1d(np.asarray(P[name], dtype=np.float64)).ravel() for name, _ in SIZES])


def bf16(a):
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(t):
    return 0.5 * t * (1.0 + erf(t / math.sqrt(2.0)))


def gelu_prime(t):
    return 0.5 * (1.0 + erf(t / math.sqrt(2.0))) + t * np.exp(-0.5 * t * t) / math.sqrt(2.0 * math.pi)


def softplus(z):
    return np.logaddexp(0.0, z)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def init_params(seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    P = {"W1": rng.normal(0.0, math.sqrt(2.0 / F), (H, F)), "b1": np.zeros(H),
         "W2": rng.normal(0.0, math.sqrt(2.0 / H), (H, H)), "b2": np.zeros(H),
         "w3": rng.normal(0.0, math.sqrt(1.0 / H), H), "b3": 0.0}
    return pack(P)


def standardise(X, norm):
    """norm = [mean (8), std (8), lam_scale]."""
    norm = np.asarray(norm, dtype=np.float64)
    return (np.asarray(X, dtype=np.float64) - norm[:F]) / norm[F:2 * F]


def forward(flat, Xs, emulate=False):
    P = unpack(flat)
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    X = r(Xs)
    Z1 = X @ r(P["W1"]).T + P["b1"]
    H1 = gelu(Z1)
    Z2 = r(H1) @ r(P["W2"]).T + P["b2"]
    H2 = gelu(Z2)
    z = H2 @ P["w3"] + P["b3"]
    return dict(X=X, Z1=Z1, H1=H1, Z2=Z2, H2=H2, z=z)


def loss(flat, Xs, y, emulate=False):
    f = forward(flat, Xs, emulate)
    return float(np.mean((softplus(f["z"]) - y) ** 2))


def grad(flat, Xs, y, emulate=False):
    """Analytic gradient of `loss` (back-propagation through the layers)."""
    P = unpack(flat)
    f = forward(flat, Xs, emulate)
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    B = Xs.shape[0]
    dz = (2.0 / B) * (softplus(f["z"]) - y) * sigmoid(f["z"])
    g = {}
    g["w3"] = f["H2"].T @ dz
    g["b3"] = float(dz.sum())
    dZ2 = np.outer(dz, P["w3"]) * gelu_prime(f["Z2"])
    g["b2"] = dZ2.sum(0)
    g["W2"] = r(dZ2).T @ r(f["H1"])
    dH1 = r(dZ2) @ r(P["W2"])
    dZ1 = dH1 * gelu_prime(f["Z1"])
    g["b1"] = dZ1.sum(0)
    g["W1"] = r(dZ1).T @ f["X"]
    return pack(g)


def adam(flat, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t = 1-based step count); returns new (flat, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


def predict(flat, X, norm, emulate=False):
    """Warm-start multipliers from raw features."""
    f = forward(flat, standardise(X, norm), emulate)
    return softplus(f["z"]) * float(np.asarray(norm)[2 * F])
