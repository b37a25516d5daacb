"""Compacting suspension driver (Sec. 5.2 workload): a periodic packing of
ellipsoids compressed isotropically, one affine rescale of box and centres
followed by one overdamped ReLCP step per step.  Host orchestration only:
every step runs in librelcp.
"""
from __future__ import annotations

import time

import numpy as np

from . import inputs as I
from . import relcp as R


def volume_fraction(shape, box) -> float:
    return float(np.sum(4.0 / 3.0 * np.pi * shape[:, 0] * shape[:, 1] * shape[:, 2]) / np.prod(box))


class Compaction:
    """n ellipsoids (semiaxes i.i.d. uniform [0.5, 1]) placed by random
    sequential addition of their bounding spheres at sphere fraction 0.3,
    then compressed to `phi0` at up to 1.5% per step (halved on a failed
    step, which is undone)."""

    def __init__(self, seed, n, phi0, *, dt=5e-3, eps=1e-3, tol=1e-6, precision=32, skin=0.05,
                 warm_start=R.WS_PREV, log=None, sim=None, state=None):
        self.dt, self.eps, self.tol = dt, eps, tol
        self.log = log or (lambda *a: None)
        if state is None:
            P = I.ellipsoid_packing(seed, n, sphere_phi=0.3)
            self.kind, self.shape, self.rho_xi = P["kind"], P["shape"], P["rho_xi"]
            self.box = P["box"].copy()
            x, q, u = P["x"], P["q"], None
        else:
            self.kind, self.shape, self.rho_xi = state["kind"], state["shape"], state["rho_xi"]
            self.box = state["box"].copy()
            x, q, u = state["x"], state["q"], state["U"]
        self.sim = sim or R.Simulation(x, q, self.kind, self.shape, self.rho_xi, self.box,
                                       u=None if u is None else u[:, :3], w=None if u is None else u[:, 3:],
                                       precision=precision, skin=skin, warm_start=warm_start)
        self.phi = volume_fraction(self.shape, self.box)
        if phi0 is not None:
            self.compress_to(phi0)

    def compress_to(self, phi0, rate=0.015):
        t0 = time.time()
        k = 0
        while self.phi < phi0 - 1e-12:
            target = min(phi0, self.phi * (1 + rate))
            s = (self.phi / target) ** (1.0 / 3.0)
            self.sim.affine_rescale(s)
            res = self.sim.step(self.dt, self.eps, self.tol, raise_on_error=False)
            if res["status"] != 0:
                self.sim.affine_rescale(1.0 / s)
                rate *= 0.5
                if rate < 1e-5:
                    raise RuntimeError("compression stalled at phi %.4f (status %d)" % (self.phi, res["status"]))
                continue
            self.box *= s
            self.phi = target
            k += 1
            if k % 20 == 0:
                self.log("compression: step %d phi %.4f contacts %d (%.1fs)" %
                         (k, self.phi, res["n_contacts_final"], time.time() - t0))
        return k

    def steps(self, nsteps, dphi=5e-5, on_step=None):
        """nsteps steps, each raising the volume fraction by dphi; returns
        the per-step statistics."""
        out = []
        for _ in range(nsteps):
            target = self.phi + dphi
            s = (self.phi / target) ** (1.0 / 3.0)
            self.sim.affine_rescale(s)
            self.box *= s
            self.phi = target
            res = self.sim.step(self.dt, self.eps, self.tol)
            out.append(res)
            if on_step is not None:
                on_step(self.sim, res)
        return out

    def state(self):
        x, q, U = self.sim.get_state()
        return dict(x=x, q=q, U=U, kind=self.kind, shape=self.shape, rho_xi=self.rho_xi, box=self.box.copy())
