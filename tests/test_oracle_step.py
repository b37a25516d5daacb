"""Pins of the oracle's ReLCP time-step (Alg. 1, Eq. relcp, Eq.
relcp_inertial) against closed forms, conservation laws and the theorems'
invariants:

* head-on inertial collision of two spheres (closed form, momentum);
* overdamped drift and a pressed pair (closed forms of the local-drag law,
  Eq. ellipsoid_mobility);
* the work W_n = gamma_n^T A_n gamma_n is non-decreasing over recursions
  (proof of Thm. ReLCP solvability, monotone f_n(x_n*)) and the accepted
  configuration satisfies the stopping rule (Eq. gap_stopping_rule);
* the paper's incremental form (Eq. relcp) and the per-row-constant form
  give the same step;
* sphere-only systems never augment (orthogonal motion cannot cause overlap
  between spheres, Sec. 2.1.4);
* timestep refinement drives the augmentation count to zero (Cor. reduction
  to the SNSD LCP; Sec. 5.1);
* the three-capsule toy of Fig. 2: augmentation resolves the overlap that
  the single-constraint SNSD LCP leaves.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2506_14097_amd import inputs as I

from states import compressed_packing, compressed_monolayer

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def sphere_shape(r):
    return [r, r, r]


def test_head_on_inertial_spheres_closed_form():
    r1, r2, rho1, rho2 = 0.5, 0.4, 1.0, 2.5
    m1 = rho1 * 4 / 3 * np.pi * r1 ** 3
    m2 = rho2 * 4 / 3 * np.pi * r2 ** 3
    gap, v1, v2, dt = 0.01, 1.0, -0.5, 0.1
    x = np.array([[0, 0, 0], [r1 + r2 + gap, 0, 0]], float)
    q = np.array([[1, 0, 0, 0], [1, 0, 0, 0]], float)
    u = np.zeros((2, 6))
    u[0, 0], u[1, 0] = v1, v2
    shape = np.array([sphere_shape(r1), sphere_shape(r2)])
    res = O.relcp_step(x, q, np.zeros(2, np.int32), shape, np.array([rho1, rho2]), np.zeros(3), dt=dt, eps=1e-9,
                       tol=1e-14, skin=0.5, u=u, dynamics=1)
    assert res["status"] == 0 and res["recursions"] == 0
    gam = -(gap + dt * (v2 - v1)) / (dt * dt * (1 / m1 + 1 / m2))
    assert abs(res["gamma"][0] - gam) < 1e-12 * gam
    U = res["U"]
    # post-step relative velocity closes exactly the initial gap
    assert abs((U[1, 0] - U[0, 0]) - (-gap / dt)) < 1e-12
    # linear momentum conserved
    assert abs(m1 * U[0, 0] + m2 * U[1, 0] - (m1 * v1 + m2 * v2)) < 1e-13
    # bodies end exactly touching
    np.testing.assert_allclose(res["x"][1, 0] - res["x"][0, 0], r1 + r2, atol=1e-13)


def test_overdamped_free_drift_closed_form():
    """One ellipsoid under a constant wrench, no contacts: x += dt F / (xi L),
    rotation angle dt 12 |T| / (xi L^3) about T (Eq. ellipsoid_mobility)."""
    with open(os.path.join(GOLDEN, "ellipsoid_mobility.json")) as f:
        g = json.load(f)
    shape = np.array([g["semiaxes"]])
    xi = g["xi"]
    F = np.array([[0.3, -0.2, 0.1, 0.0, 0.0, 0.7]])
    dt = 0.01
    res = O.relcp_step(np.zeros((1, 3)), np.array([[1.0, 0, 0, 0]]), np.zeros(1, np.int32), shape, np.array([xi]),
                       np.zeros(3), dt=dt, eps=1e-6, tol=1e-12, skin=0.1, fext=F)
    assert res["status"] == 0
    np.testing.assert_allclose(res["U"][0, :3], F[0, :3] * g["translational_mobility"], rtol=1e-15)
    np.testing.assert_allclose(res["U"][0, 3:], F[0, 3:] * g["rotational_mobility"], rtol=1e-15)
    ang = dt * 0.7 * g["rotational_mobility"]
    np.testing.assert_allclose(res["q"][0], [np.cos(ang / 2), 0, 0, np.sin(ang / 2)], atol=1e-15)


def test_overdamped_pressed_pair():
    """Two touching spheres pushed together by equal and opposite forces F:
    the multiplier is exactly F and the bodies stay touching."""
    r, F = 0.5, 0.8
    x = np.array([[0, 0, 0], [2 * r, 0, 0]], float)
    q = np.array([[1, 0, 0, 0], [1, 0, 0, 0]], float)
    fext = np.zeros((2, 6))
    fext[0, 0], fext[1, 0] = F, -F
    res = O.relcp_step(x, q, np.zeros(2, np.int32), np.array([sphere_shape(r)] * 2), np.array([1.0, 3.0]),
                       np.zeros(3), dt=0.05, eps=1e-9, tol=1e-14, skin=0.1, fext=fext)
    assert res["status"] == 0
    assert abs(res["gamma"][0] - F) < 1e-13
    np.testing.assert_allclose(res["U"], 0.0, atol=1e-14)


def test_inertial_free_rotation():
    """Free flight of a spinning body: x += dt u, q = exp(dt w) q (world w)."""
    u = np.array([[0.1, 0.2, -0.3, 0.0, 0.0, 2.0]])
    q0 = np.array([[np.cos(0.2), np.sin(0.2), 0, 0]])
    res = O.relcp_step(np.zeros((1, 3)), q0, np.zeros(1, np.int32), np.array([[1.0, 0.5, 0.5]]), np.ones(1),
                       np.zeros(3), dt=0.01, eps=1e-6, tol=1e-12, skin=1.0, u=u, dynamics=1)
    np.testing.assert_allclose(res["x"][0], 0.01 * u[0, :3], atol=1e-16)
    e = np.array([np.cos(0.01), 0, 0, np.sin(0.01)])
    s1, w1, s2, w2 = e[0], e[1:], q0[0, 0], q0[0, 1:]
    ref = np.concatenate([[s1 * s2 - w1 @ w2], s1 * w2 + s2 * w1 + np.cross(w1, w2)])
    np.testing.assert_allclose(res["q"][0], ref, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1])
def test_step_invariants_on_compressed_packing(seed):
    S = compressed_packing(seed, 150, 26)
    x, box = S["x"] * 0.99, S["box"] * 0.99
    kw = dict(dt=5e-3, eps=1e-5, tol=1e-10, skin=0.2, prev=S["prev"])
    r = O.relcp_step(x, S["q"], S["kind"], S["shape"], S["rho_xi"], box, **kw)
    assert r["status"] == 0
    # the stopping rule holds at the accepted configuration
    assert r["max_overlap"] <= 1e-5
    # recursion work is monotone (proof of Thm. ReLCP solvability, part 3)
    W = r["W"]
    assert np.all(np.diff(W) >= -1e-12 * (1 + W.max()))
    # the incremental form of Eq. relcp and the per-row-constant form agree
    r2 = O.relcp_step(x, S["q"], S["kind"], S["shape"], S["rho_xi"], box, form=1, **kw)
    assert r2["status"] == 0
    assert list(r2["n_contacts"]) == list(r["n_contacts"])
    np.testing.assert_allclose(r2["U"], r["U"], atol=1e-7 * np.abs(r["U"]).max())
    # linear momentum: the contact wrench sums to zero (equal and opposite)
    kt, _ = O.body_K(0, 0, 5e-3, S["kind"], S["shape"], S["q"], S["rho_xi"])
    f = r["U"][:, :3] / kt
    assert np.abs(f.sum(0)).max() < 1e-9 * np.abs(f).sum()


def test_recursions_happen_and_resolve():
    S = compressed_packing(0, 150, 26)
    r = O.relcp_step(S["x"] * 0.99, S["q"], S["kind"], S["shape"], S["rho_xi"], S["box"] * 0.99, dt=5e-3, eps=1e-5,
                     tol=1e-10, skin=0.2, prev=S["prev"])
    assert r["recursions"] >= 1
    assert r["n_rows"] == r["n_contacts"][-1]
    assert np.all(r["rec"][r["n_contacts"][0]:] >= 1)


def test_spheres_never_augment():
    """Orthogonal motion between spheres cannot create overlap (Sec. 2.1.4):
    the first trial is always accepted, even at a tiny tolerance."""
    rng = np.random.default_rng(11)
    n = 60
    rad = rng.uniform(0.5, 1.0, n)
    box = np.full(3, 9.0)
    x = I.rsa_spheres(rng, rad, box) * 0.93
    res = O.relcp_step(x, np.tile([1.0, 0, 0, 0], (n, 1)), np.zeros(n, np.int32), np.repeat(rad[:, None], 3, 1),
                       np.ones(n), box * 0.93, dt=0.05, eps=1e-9, tol=1e-12, skin=1.0)
    assert res["status"] == 0
    assert res["recursions"] == 0
    assert res["n_contacts"][0] > 10


def _qmul(a, b):
    s1, w1, s2, w2 = a[0], a[1:], b[0], b[1:]
    return np.concatenate([[s1 * s2 - w1 @ w2], s1 * w2 + s2 * w1 + np.cross(w1, w2)])


def _two_ellipsoids_glancing(dt, T):
    """Sec. 5.1 set-up: r = (1, 1, 2) lying in the x-y plane (major axis
    in-plane), both rotated 45 deg about z, centres a unit apart in x, unit
    opposing vertical forces, overdamped local drag with xi = 1."""
    qy = np.array([np.cos(np.pi / 4), 0, np.sin(np.pi / 4), 0])   # body z -> world x
    qz = np.array([np.cos(np.pi / 8), 0, 0, np.sin(np.pi / 8)])   # 45 deg about z
    q = np.array([_qmul(qz, qy)] * 2)
    shape = np.array([[1.0, 1.0, 2.0]] * 2)
    kind = np.zeros(2, np.int32)
    # vertical offset: the two start a small gap apart (bisection on the
    # oracle SNSD is set-up here, not a check)
    lo, hi = 0.0, 6.0
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        phi = O.snsd_ellipsoid([1.0, mid, 0.0], q[0], shape[0], q[1], shape[1])[0]
        lo, hi = (mid, hi) if phi < 0.05 else (lo, mid)
    x = np.array([[0.0, 0.0, 0.0], [1.0, hi, 0.0]])
    fext = np.zeros((2, 6))
    fext[0, 1], fext[1, 1] = 1.0, -1.0
    aug = 0
    prev = None
    steps = int(round(T / dt))
    for _ in range(steps):
        r = O.relcp_step(x, q, kind, shape, np.ones(2), np.zeros(3), dt=dt, eps=2e-5, tol=1e-13, skin=1.0,
                         fext=fext, prev=prev)
        assert r["status"] == 0
        assert r["max_overlap"] <= 2e-5
        aug += r["recursions"]
        x, q = r["x"], r["q"]
        prev = O.pair_lambda(r)
    return aug / steps, x


def test_timestep_refinement_reduces_augmentation():
    """Augmentations per step fall to zero as dt is refined (overlap
    tolerance 1e-5 diameters, as in Sec. 5.1)."""
    a1, _ = _two_ellipsoids_glancing(0.1, 8.0)
    a2, _ = _two_ellipsoids_glancing(0.05, 8.0)
    a3, _ = _two_ellipsoids_glancing(0.01, 8.0)
    assert a1 > 0.1
    assert a1 >= a2 > 0
    assert a3 == 0


def test_three_capsule_toy():
    """Fig. 2: three overlapping capsules; augmentation resolves what the
    single-constraint SNSD LCP (max_recursions = 0) leaves overlapping."""
    rng = np.random.default_rng(0)
    th = rng.uniform(0, np.pi, 3)
    x = np.array([[0, 0, 0], [0.9, 0.2, 0], [0.4, 0.8, 0]]) + rng.normal(0, 0.1, (3, 3)) * [1, 1, 0]
    q = I.planar_quaternions(th)
    shape = np.array([[0.5, 2.0, 0]] * 3)
    kw = dict(dt=0.1, eps=1e-5, tol=1e-12, skin=5.0, planar=1)
    r = O.relcp_step(x, q, np.ones(3, np.int32), shape, np.ones(3), np.zeros(3), **kw)
    r0 = O.relcp_step(x, q, np.ones(3, np.int32), shape, np.ones(3), np.zeros(3), max_recursions=0, **kw)
    assert r["status"] == 0 and r0["status"] == 0
    assert r["recursions"] >= 1
    assert r["max_overlap"] <= 1e-5
    assert r0["max_overlap"] > 1e-2
    # planar: no out-of-plane motion
    assert np.abs(r["x"][:, 2]).max() == 0.0
    assert np.abs(r["U"][:, 2:5]).max() == 0.0


def test_monolayer_step():
    S = compressed_monolayer(3, 120, 20)
    box = S["box"] * [0.99, 0.99, 0]
    x = S["x"] * [0.99, 0.99, 1]
    r = O.relcp_step(x, S["q"], S["kind"], S["shape"], S["rho_xi"], box, dt=1e-2, eps=1e-5, tol=1e-10, skin=0.2,
                     planar=1, prev=S["prev"])
    assert r["status"] == 0
    assert r["max_overlap"] <= 1e-5
    assert r["n_contacts"][0] > 20


def test_error_paths():
    S = compressed_packing(0, 150, 26)
    x, box = S["x"] * 0.99, S["box"] * 0.99
    kw = dict(dt=5e-3, eps=1e-5, tol=1e-10, prev=S["prev"])
    r = O.relcp_step(x, S["q"], S["kind"], S["shape"], S["rho_xi"], box, skin=0.2, **kw)
    assert r["recursions"] >= 1
    # recursion cap
    rc = O.relcp_step(x, S["q"], S["kind"], S["shape"], S["rho_xi"], box, skin=0.2, max_recursions=1 if
                      r["recursions"] > 1 else 64, **kw)
    if r["recursions"] > 1:
        assert rc["status"] == O.E_RECURSION_CAP
    # skin too small for the motion of this step
    rs = O.relcp_step(x, S["q"], S["kind"], S["shape"], S["rho_xi"], box, skin=1e-4, **kw)
    assert rs["status"] == O.E_SKIN
    # LCP iteration cap
    rl = O.relcp_step(x, S["q"], S["kind"], S["shape"], S["rho_xi"], box, skin=0.2, lcp_mode=1, lcp_max_iters=1,
                      **kw)
    assert rl["status"] == O.E_LCP_MAXITER
