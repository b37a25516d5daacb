"""The two-ellipsoid sliding collision of Sec. 5.1 on the oracle (CPU).

* Pin of the narrowphase against a closed form: two identical, parallel
  ellipsoids touch exactly when the centre offset d lies on the boundary of
  their Minkowski difference, the same ellipsoid scaled by 2, i.e. when
  d^T (4 Sigma)^-1 d = 1 (Sigma = R diag(a^2, b^2, c^2) R^T).  So Phi is zero
  there, negative inside and positive outside, in every direction.
* The study's set-up touches at a centre separation of exactly 3 along y.
* Reduction (Corollary on the reduction to SNSD-LCP): through the contact
  of the study, ReLCP appends constraints at dt = 0.1 and none at dt = 0.01,
  where its steps are those of LCP-SNSD."""
import numpy as np
import pytest

import oracle as O
from paper_2506_14097_amd import inputs as I


def _sigma(q, e):
    R = O.quat_to_R(q)
    return R @ np.diag(np.asarray(e) ** 2) @ R.T


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_parallel_ellipsoids_touch_on_the_doubled_ellipsoid(seed):
    rng = np.random.default_rng(seed)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    e = rng.uniform(0.5, 2.0, 3)
    M = np.linalg.inv(4.0 * _sigma(q, e))
    for _ in range(6):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        s = 1.0 / np.sqrt(u @ M @ u)  # d = s u satisfies d^T (4 Sigma)^-1 d = 1
        phi0 = O.snsd_ellipsoid(s * u, q, e, q, e)[0]
        assert abs(phi0) < 1e-9 * s
        assert O.snsd_ellipsoid(0.9 * s * u, q, e, q, e)[0] < 0
        assert O.snsd_ellipsoid(1.1 * s * u, q, e, q, e)[0] > 0


def test_study_pair_touches_at_separation_three():
    S = I.glancing_ellipsoids()
    q, e = S["q"][0], S["shape"][0]
    assert abs(O.snsd_ellipsoid(np.array([1.0, 3.0, 0.0]), q, e, q, e)[0]) < 1e-9
    # the long axes lie in the x-y plane at 45 degrees
    assert np.allclose(O.quat_to_R(q)[:, 2], [np.sqrt(0.5), np.sqrt(0.5), 0.0], atol=1e-12)


def _recursing_steps(dt, t_end=120.0):
    S = I.glancing_ellipsoids()
    x, q = S["x"].copy(), S["q"].copy()
    n = int(round((t_end - S["t0"]) / dt))
    rec, rows = 0, 0
    for _ in range(n):
        r = O.relcp_step(x, q, S["kind"], S["shape"], S["rho_xi"], S["box"], dt=dt, eps=1e-5, tol=1e-12, skin=0.5,
                         fext=S["fext"])
        assert r["status"] == 0
        assert r["max_overlap"] <= 1e-5
        x, q = r["x"], r["q"]
        rec += r["recursions"] > 0
        rows += r["n_rows"] > 0
    return rec, rows


def test_relcp_reduces_to_snsd_lcp_at_small_timesteps():
    rec1, rows1 = _recursing_steps(0.1)
    rec2, rows2 = _recursing_steps(0.01)
    assert rows1 > 0 and rows2 > 0  # the bodies are in contact
    assert rec1 > 0                 # large steps need appended constraints
    assert rec2 == 0                # small steps are LCP-SNSD steps
