"""Pins of the oracle's inertial mobility (Sec. 2.1.2, Eq. law_inertia;
Eq. relcp_inertial) against quantities computed here without its formula:

* the inertia tensor of a rotated solid ellipsoid, integrated by a Gauss
  quadrature over the body (exact for the quadratic moments), against the
  inverse of the rotational block of ``body_K`` (which holds dt M^-1), and
  the mass against the quadrature's volume;
* angular momentum across an inertial contact step with off-centre lever
  arms and no recursion: the impulse on a pair is equal and opposite and
  acts along the shared normal through two points with p_b - p_a = Phi n
  (Lemma uniform interior tangent ball; Eq. collision_ft), so
  sum_b (m x_b x u_b + I_b w_b), with x and I at C^k, is unchanged by the
  velocity update.  A wrong principal moment or a transposed rotation in
  M^-1 breaks both.

The rotation matrices here come from scipy's quaternion routine, not from
the oracle.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle as O
from paper_2506_14097_amd import inputs as I


def rot(q):
    """World-from-body rotation of a scalar-first unit quaternion (scipy
    takes the scalar last)."""
    q = np.asarray(q, float)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def ellipsoid_inertia_quadrature(semi, q, rho, nr=6, nmu=8, nphi=16):
    """Mass and world-frame inertia tensor about the centre of a solid
    ellipsoid, I = rho int (|r|^2 1 - r r^T) dV, by quadrature: points of the
    unit ball in spherical coordinates (Gauss-Legendre in the radius and in
    cos(theta), uniform in phi), mapped to the body by diag(semi) and to the
    world by the rotation.  Exact up to rounding for the polynomial moments
    of degree <= 2 that the tensor needs."""
    Rm = rot(q)
    A = np.diag(semi)
    xr, wr = np.polynomial.legendre.leggauss(nr)
    rr, wr = 0.5 * (xr + 1.0), 0.5 * wr
    mu, wmu = np.polynomial.legendre.leggauss(nmu)
    ph = 2.0 * np.pi * np.arange(nphi) / nphi
    wph = np.full(nphi, 2.0 * np.pi / nphi)
    mass = 0.0
    J = np.zeros((3, 3))
    jac = np.prod(semi)  # dV = a b c ds
    for r, w1 in zip(rr, wr):
        for m_, w2 in zip(mu, wmu):
            st = np.sqrt(1.0 - m_ * m_)
            for p, w3 in zip(ph, wph):
                s = r * np.array([st * np.cos(p), st * np.sin(p), m_])
                x = Rm @ (A @ s)
                w = rho * jac * r * r * w1 * w2 * w3
                mass += w
                J += w * ((x @ x) * np.eye(3) - np.outer(x, x))
    return mass, J


def test_quaternion_convention_matches_scipy():
    rng = np.random.default_rng(0)
    for qq in I.shoemake_quaternions(rng, 20):
        assert np.abs(O.quat_to_R(qq) - rot(qq)).max() < 1e-14


def test_quadrature_sphere_closed_form():
    """The quadrature itself on a ball of radius r: m = rho 4/3 pi r^3 and
    I = 2/5 m r^2 (textbook)."""
    m, J = ellipsoid_inertia_quadrature([0.7, 0.7, 0.7], [1.0, 0, 0, 0], 2.0)
    m0 = 2.0 * 4.0 / 3.0 * np.pi * 0.7 ** 3
    assert abs(m - m0) < 1e-13 * m0
    np.testing.assert_allclose(J, 0.4 * m0 * 0.49 * np.eye(3), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("seed", range(4))
def test_inertial_mobility_against_quadrature(seed):
    rng = np.random.default_rng(100 + seed)
    n = 5
    semi = rng.uniform(0.3, 1.5, (n, 3))
    q = I.shoemake_quaternions(rng, n)
    rho = rng.uniform(0.5, 3.0, n)
    dt = 0.01
    kt, Kr = O.body_K(1, 0, dt, np.zeros(n, np.int32), semi, q, rho)
    for b in range(n):
        m, J = ellipsoid_inertia_quadrature(semi[b], q[b], rho[b])
        np.testing.assert_allclose(kt[b], dt / m, rtol=1e-13)
        Iw = np.linalg.inv(Kr[b] / dt)
        assert np.abs(Iw - J).max() < 1e-12 * np.abs(J).max(), (Iw, J)


def _touching_pair(rng, semi_a, semi_b, depth):
    """Two ellipsoids, b placed along a random direction from a with a random
    lateral offset, then moved along the SNSD normal so that Phi = -depth."""
    qa, qb = I.shoemake_quaternions(rng, 2)
    d = rng.normal(size=3)
    d *= 2.5 / np.linalg.norm(d)
    for _ in range(3):
        phi, nrm, _, _ = O.snsd_ellipsoid(d, qa, semi_a, qb, semi_b)
        d = d - (phi + depth) * nrm
    phi, nrm, _, _ = O.snsd_ellipsoid(d, qa, semi_a, qb, semi_b)
    assert abs(phi + depth) < 1e-10
    return d, qa, qb, nrm


def _angular_momentum(x, U, semi, q, rho):
    L = np.zeros(3)
    parts = 0.0
    for b in range(len(x)):
        m, J = ellipsoid_inertia_quadrature(semi[b], q[b], rho[b])
        t1 = m * np.cross(x[b], U[b, :3])
        t2 = J @ U[b, 3:]
        L += t1 + t2
    return L


@pytest.mark.parametrize("seed", range(4))
def test_inertial_contact_step_conserves_angular_momentum(seed):
    rng = np.random.default_rng(200 + seed)
    # a chain of three ellipsoids, each pair slightly overlapping and closing
    semi = rng.uniform(0.4, 1.2, (3, 3))
    d1, q0, q1, n1 = _touching_pair(rng, semi[0], semi[1], 0.01)
    q = [q0, q1]
    x = [np.zeros(3), d1]
    # third body touching the second
    for _ in range(20):
        d2, qa, qb, n2 = _touching_pair(rng, semi[1], semi[2], 0.008)
        # keep the orientation of body 1: rebuild the pair with body 1's q
        phi, nrm, _, _ = O.snsd_ellipsoid(d2, q1, semi[1], qb, semi[2])
        for _ in range(3):
            d2 = d2 - (phi + 0.008) * nrm
            phi, nrm, _, _ = O.snsd_ellipsoid(d2, q1, semi[1], qb, semi[2])
        x2 = d1 + d2
        gap02, _, _, _ = O.snsd_ellipsoid(x2, q0, semi[0], qb, semi[2])
        if gap02 > 0.3:
            break
    q.append(qb)
    x.append(x2)
    x, q = np.array(x), np.array(q)
    rho = rng.uniform(0.5, 2.0, 3)
    u = np.zeros((3, 6))
    u[:, :3] = rng.normal(0, 0.2, (3, 3))
    u[:, 3:] = rng.normal(0, 0.3, (3, 3))
    u[0, :3] += 0.5 * n1
    u[2, :3] -= 0.5 * nrm
    dt = 0.01
    r = O.relcp_step(x, q, np.zeros(3, np.int32), semi, rho, np.zeros(3), dt=dt, eps=1e-3, tol=1e-14, skin=0.3, u=u,
                     dynamics=1)
    assert r["status"] == 0 and r["recursions"] == 0
    assert np.sum(r["gamma"] > 0) >= 2, r["gamma"]
    L0 = _angular_momentum(x, u, semi, q, rho)
    L1 = _angular_momentum(x, r["U"], semi, q, rho)
    # the scale: the angular impulse the contacts deliver to each body
    imp = 0.0
    rot_imp = 0.0
    for b in range(3):
        m, J = ellipsoid_inertia_quadrature(semi[b], q[b], rho[b])
        du = r["U"][b] - u[b]
        imp += np.linalg.norm(m * np.cross(x[b], du[:3])) + np.linalg.norm(J @ du[3:])
        rot_imp += np.linalg.norm(J @ du[3:])
    assert rot_imp > 0.05 * imp  # the lever arms are off-centre
    assert np.linalg.norm(L1 - L0) <= 1e-12 * imp, (L1 - L0, imp)
    # linear momentum too
    m = np.array([ellipsoid_inertia_quadrature(semi[b], q[b], rho[b])[0] for b in range(3)])
    P0, P1 = (m[:, None] * u[:, :3]).sum(0), (m[:, None] * r["U"][:, :3]).sum(0)
    assert np.linalg.norm(P1 - P0) <= 1e-12 * np.abs(m[:, None] * (r["U"][:, :3] - u[:, :3])).sum()
