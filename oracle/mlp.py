"""FP64 oracle of the learned warm start -- TEST INFRASTRUCTURE ONLY.

A per-contact MLP corrects the previous-step multiplier of each row of A_0
(the paper is silent on warm starts; the projected-gradient LCP of Eq. cqpp
accepts any start).  Network and start, following the written definition:

    z = w3 . GELU(W2 GELU(W1 x + b1) + b2) + b3
    GELU(t) = t Phi(t) = 0.5 t (1 + erf(t / sqrt 2))        (exact form)
    y0 = max(0, f_2 + scale z),   gamma0 = y0 * rowscale

x = standardised features (8), hidden width 128; f_2 = the previous-step
multiplier in length units (raw feature 2), rowscale = abar / A_aa.  With
z = 0 the start is the previous-step one.  Loss: mean over the batch of
(z - t)^2 with t = (y - f_2) / scale, y the converged multiplier in length
units.  Adam.

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


def init_params(seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    P = {"W1": rng.normal(0.0, math.sqrt(2.0 / F), (H, F)), "b1": np.zeros(H),
         "W2": rng.normal(0.0, math.sqrt(2.0 / H), (H, H)), "b2": np.zeros(H),
         "w3": rng.normal(0.0, math.sqrt(1.0 / H), H), "b3": 0.0}
    return pack(P)


def standardise(X, norm):
    """norm = [mean (8), std (8), scale]."""
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


def loss(flat, Xs, t, emulate=False):
    """Mean squared error of z against the scaled correction t."""
    f = forward(flat, Xs, emulate)
    return float(np.mean((f["z"] - t) ** 2))


def grad(flat, Xs, t, emulate=False):
    """Analytic gradient of `loss` (back-propagation through the layers)."""
    P = unpack(flat)
    f = forward(flat, Xs, emulate)
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    B = Xs.shape[0]
    dz = (2.0 / B) * (f["z"] - t)
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


def correction_target(X, y, norm):
    """t = (y - f_2) / scale for raw features X and targets y (length units)."""
    return (np.asarray(y, dtype=np.float64) - np.asarray(X, dtype=np.float64)[:, 2]) / float(np.asarray(norm)[2 * F])


def adam(flat, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t = 1-based step count); returns new (flat, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


def predict(flat, X, norm, emulate=False):
    """Warm start in length units, y0 = max(0, f_2 + scale z), from raw
    features (multiply by rowscale for the multiplier)."""
    X = np.asarray(X, dtype=np.float64)
    f = forward(flat, standardise(X, norm), emulate)
    return np.maximum(0.0, X[:, 2] + float(np.asarray(norm)[2 * F]) * f["z"])


# ---------------------------------------------------------------------------
# features of the iteration-0 rows
# ---------------------------------------------------------------------------
def _semi_extents(kind, p):
    """Semi-extents along the body axes: ellipsoid semiaxes (a, b, c);
    spherocylinder with cap radius r and cylinder length l: (l/2 + r, r, r)."""
    if kind == 0:
        return np.array(p[:3], dtype=np.float64)
    r, l = float(p[0]), float(p[1])
    return np.array([0.5 * l + r, r, r])


def features(q, kind, shape, rho_xi, u_prev, prev, step, dt, dynamics=0, planar=0):
    """Features of the rows of A_0 of an oracle step result `step` (rows
    generated at recursion 0), in that result's row order, oriented so that
    body a has the smaller index.  Multipliers are taken in length units,
    A_aa gamma / abar, with A_aa the diagonal entry of A = dt D^T K D (Eq.
    relcp; K of Eq. ellipsoid_mobility or the inertial K) and abar the mean
    of the two bodies' mean semi-extents:
      0 Phi_0 / abar,
      1 dt (D^T U_prev) / abar, the previous velocity along the row
        (D^T U = -(n.u_a + (r_a x n).w_a) + n.u_b + (r_b x n).w_b),
      2 A_aa lambda_prev / abar, lambda_prev the previous multiplier sum of
        the pair (0 if it had none),
      3, 4 rows of A_0 at a, at b,
      5, 6 min / max semi-extent of a, of b,
      7 sum over the other rows of A_0 at a or at b of max(0, -Phi_0),
        over abar (the overlap load of the neighbourhood).
    u_prev: (n, 6) velocities of the previous step or None; prev = (a, b,
    lam) pair sums of the previous step or None.  Returns (ia, ib, X,
    rowscale) with rowscale = abar / A_aa (model output -> multiplier)."""
    from . import body_K
    rows = np.flatnonzero(step["rec"] == 0)
    ia, ib = step["ia"][rows].copy(), step["ib"][rows].copy()
    nb = len(kind)
    kt, Kr = body_K(dynamics, planar, dt, kind, shape, q, rho_xi)
    coord = np.bincount(np.concatenate([ia, ib]), minlength=nb)
    phi0 = step["phi"][rows]
    overlap_at = np.zeros(nb)            # sum of max(0, -Phi_0) over the rows at each body
    np.add.at(overlap_at, ia, np.maximum(0.0, -phi0))
    np.add.at(overlap_at, ib, np.maximum(0.0, -phi0))
    lam_of = {}
    if prev is not None:
        for a, b, lam in zip(*prev):
            lam_of[(int(min(a, b)), int(max(a, b)))] = float(lam)
    X = np.zeros((rows.size, F))
    rowscale = np.zeros(rows.size)
    for k, r in enumerate(rows):
        a, b = int(ia[k]), int(ib[k])
        nrm, ta, tb = step["n"][r], step["ta"][r], step["tb"][r]
        Aaa = dt * (nrm @ (kt[a] * nrm) + ta @ Kr[a] @ ta + nrm @ (kt[b] * nrm) + tb @ Kr[b] @ tb)
        ea, eb = _semi_extents(kind[a], shape[a]), _semi_extents(kind[b], shape[b])
        abar = 0.5 * (ea.mean() + eb.mean())
        rowscale[k] = abar / Aaa
        rate = 0.0
        if u_prev is not None:
            ua, ub = np.asarray(u_prev[a]), np.asarray(u_prev[b])
            rate = -(nrm @ ua[:3] + ta @ ua[3:]) + nrm @ ub[:3] + tb @ ub[3:]
        load = overlap_at[a] + overlap_at[b] - 2.0 * max(0.0, -phi0[k])
        fa = (coord[a], ea.min() / ea.max())
        fb = (coord[b], eb.min() / eb.max())
        if a > b:
            fa, fb = fb, fa
            a, b = b, a
            ia[k], ib[k] = a, b
        X[k] = [phi0[k] / abar, dt * rate / abar, lam_of.get((a, b), 0.0) / rowscale[k],
                fa[0], fb[0], fa[1], fb[1], load / abar]
    return ia, ib, X, rowscale


def targets(step, rowscale):
    """Training targets of the rows of A_0: final multiplier after the
    step's last recursion, in the features' length units (gamma / rowscale)."""
    rows = np.flatnonzero(step["rec"] == 0)
    return step["gamma"][rows] / rowscale
