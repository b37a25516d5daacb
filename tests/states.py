"""Test states: seeded generator output, optionally compressed by oracle steps.

Dense states with real contacts are made the way a compaction run makes them:
bounding-sphere random sequential addition (no overlaps), then repeated
affine compression of the periodic box, each followed by one oracle time-step.
Every such state comes from the generator module and the CPU oracle only.
"""
from __future__ import annotations

import functools

import numpy as np

import oracle as O
from paper_2506_14097_amd import inputs as I


@functools.lru_cache(maxsize=None)
def compressed_packing(seed: int, n: int, steps: int, s: float = 0.99, sphere_phi: float = 0.3, dt: float = 5e-3,
                       eps: float = 1e-5, tol: float = 1e-9, skin: float = 0.2):
    P = I.ellipsoid_packing(seed, n, sphere_phi=sphere_phi)
    x, q, box = P["x"].copy(), P["q"].copy(), P["box"].copy()
    prev = None
    for _ in range(steps):
        x *= s
        box *= s
        r = O.relcp_step(x, q, P["kind"], P["shape"], P["rho_xi"], box, dt=dt, eps=eps, tol=tol, skin=skin,
                         prev=prev)
        if r["status"] != 0:
            raise RuntimeError("compression step failed with status %d" % r["status"])
        x, q = r["x"].copy(), r["q"].copy()
        prev = O.pair_lambda(r)
    out = dict(P)
    out.update(x=x, q=q, box=box, prev=prev)
    return out


@functools.lru_cache(maxsize=None)
def compressed_monolayer(seed: int, n: int, steps: int, s: float = 0.99, dt: float = 1e-2, eps: float = 1e-5,
                         tol: float = 1e-9, skin: float = 0.2):
    P = I.spherocylinder_monolayer(seed, n, disk_fraction=0.4)
    x, q, box = P["x"].copy(), P["q"].copy(), P["box"].copy()
    prev = None
    for _ in range(steps):
        x[:, :2] *= s
        box[:2] *= s
        r = O.relcp_step(x, q, P["kind"], P["shape"], P["rho_xi"], box, dt=dt, eps=eps, tol=tol, skin=skin,
                         prev=prev, planar=1)
        if r["status"] != 0:
            raise RuntimeError("compression step failed with status %d" % r["status"])
        x, q = r["x"].copy(), r["q"].copy()
        prev = O.pair_lambda(r)
    out = dict(P)
    out.update(x=x, q=q, box=box, prev=prev)
    return out
