"""Growing colony of spherocylinders in a monolayer (Sec. 5.3 workload):
every cell's length grows linearly and all cells divide together when they
reach the division length; each division splits a cell into its two halves
(tip to tip), each turned in the plane by a small random angle.  Host
orchestration only: growth, division and every ReLCP step run in
librelcp.

Lengths are total (tip-to-tip) lengths; the library's shape holds the
cylinder length l = length - 2 r.
"""
from __future__ import annotations

import time

import numpy as np

from . import inputs as I
from . import relcp as R


class Colony:
    """One cell of total length `length0` (diameter 2 r) at the origin,
    growing at `rate` (length per unit time) and dividing at `length_div`
    into two cells of half its length, jitter angles N(0, jitter^2) (seeded);
    overdamped (drag xi), open plane, dt, overlap tolerance eps, LCP
    tolerance tol.  The skin is 0.2: cells at the rim of a large colony move
    by up to a few hundredths per step as the interior grows, and a trial
    may move a surface point by at most skin / 2."""

    def __init__(self, seed=2, *, radius=0.5, length0=1.0, length_div=2.0, rate=0.01, dt=1e-2, eps=1e-3,
                 tol=1e-6, precision=64, skin=0.2, xi=1.0, jitter=0.01, lcp_max_iters=0, state=None):
        self.r, self.length_div, self.rate, self.dt = radius, length_div, rate, dt
        self.eps, self.tol, self.jitter = eps, tol, jitter
        self.xi, self.precision, self.lcp_max_iters = xi, precision, lcp_max_iters
        self.rng = I.rng_for(seed)
        if state is None:
            x = np.zeros((1, 3))
            q = I.planar_quaternions(np.array([0.0]))
            self.l = length0 - 2.0 * radius
            shape = np.array([[radius, self.l, 0.0]])
            rho = np.array([xi])
        else:
            x, q, shape, rho = state["x"], state["q"], state["shape"], state["rho_xi"]
            self.l = float(shape[0, 1])
        self.sim = R.Simulation(x, q, np.full(len(x), I.SPHEROCYLINDER, np.int32), shape, rho, np.zeros(3),
                                precision=precision, skin=skin, planar=True, warm_start=R.WS_PREV,
                                lcp_max_iters=lcp_max_iters)
        self.divisions = 0

    @property
    def n(self):
        return self.sim.n

    def reskin(self, skin, lcp_max_iters=None):
        """Continue from the current state in a new context with another
        skin (a larger one lets a set-up grow faster; warm-start history is
        not carried over) and, if given, another LCP iteration cap."""
        if lcp_max_iters is not None:
            self.lcp_max_iters = lcp_max_iters
        x, q, _ = self.sim.get_state()
        n = len(x)
        shape = np.tile([self.r, self.l, 0.0], (n, 1))
        self.sim.close()
        self.sim = R.Simulation(x, q, np.full(n, I.SPHEROCYLINDER, np.int32), shape, np.full(n, self.xi),
                                np.zeros(3), precision=self.precision, skin=skin, planar=True, warm_start=R.WS_PREV,
                                lcp_max_iters=self.lcp_max_iters)

    @property
    def l_div(self):
        return self.length_div - 2.0 * self.r

    def step(self, rate=None, raise_on_error=True):
        """Grow by rate dt, divide if the cells reached the division length,
        then one ReLCP step.  Returns the step statistics."""
        dl = (self.rate if rate is None else rate) * self.dt
        self.sim.grow(dl)
        self.l += dl
        self._divided = False
        if self.l >= self.l_div:
            jit = self.rng.normal(0.0, self.jitter, 2 * self.n)
            self.sim.divide(self.l_div, jit)
            self.l = 0.5 * self.l - self.r
            self.divisions += 1
            self._divided = True
        return self.sim.step(self.dt, self.eps, self.tol, raise_on_error=raise_on_error)

    def grow_to(self, n_cells, rate=0.1, log=None):
        """Steps until the colony holds at least n_cells cells: the set-up of
        a timed window, at a faster growth (`rate`).  A step that fails
        because the rim moved too far for the candidate list (skin) or
        whose LCP did not converge within the iteration cap (an overlap too
        large for one step) is taken again with half its growth undone and
        the growth rate halved (never below the benchmarked rate; the
        failed step left the state unchanged), and the rate recovers by a
        quarter every 1,000 steps."""
        k, ok, r = 0, 0, rate
        t_log = time.time()
        while self.n < n_cells:
            res = self.step(r, raise_on_error=False)
            back = r * self.dt
            while res["status"] in (R.E_SKIN, R.E_LCP_MAXITER) and not self._divided and back > 1e-6 * self.dt:
                back *= 0.5
                self.sim.grow(-back)
                self.l -= back
                r = max(self.rate, 0.5 * r)
                res = self.sim.step(self.dt, self.eps, self.tol, raise_on_error=False)
            if res["status"] != 0:
                raise R.RelcpError(res["status"], "colony set-up step failed")
            k += 1
            ok += 1
            if ok >= 1000:
                r, ok = min(rate, 1.25 * r), 0
            if log and time.time() - t_log > 15.0:
                t_log = time.time()
                log("colony: step %d, %d cells, length %.3f, set-up rate %.4f" % (k, self.n, self.l + 2 * self.r,
                                                                                    r))
        return k
