"""Pins of the oracle's shared-normal signed distance (SNSD).

Each check ties the oracle to something other than itself: closed forms
(spheres, a shared principal axis, segment geometry), an independent contact
function (Perram-Wertheim), an independent surface-distance minimisation, and
brute force over dense samples.  Paper: Sec. 2.1.4 (proxy surfaces), Lemma
uniform interior tangent ball (p_b - p_a = Phi n), Sec. 5.2 / 5.3 (ellipsoid
and spherocylinder SNSD).
"""
import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

import oracle as O
from paper_2506_14097_amd import inputs as I

Q0 = np.array([1.0, 0.0, 0.0, 0.0])


def rand_q(rng):
    return I.shoemake_quaternions(rng, 1)[0]


def sigma(q, e):
    R = O.quat_to_R(q)
    return R @ np.diag(np.asarray(e) ** 2) @ R.T


def pw_contact(d, Sa, Sb):
    """Perram-Wertheim contact function: < 1 overlap, = 1 touching, > 1 apart."""
    def negF(lam):
        Cm = (1 - lam) * Sa + lam * Sb
        return -lam * (1 - lam) * d @ np.linalg.solve(Cm, d)
    r = minimize_scalar(negF, bounds=(0.0, 1.0), method="bounded", options=dict(xatol=1e-13))
    return -r.fun


@pytest.mark.parametrize("d", [[3.0, 0, 0], [0.5, 0.3, -0.2], [1.2, 0.9, 0.4], [0.0, 0.0, 1.69]])
def test_sphere_closed_form(d):
    d = np.array(d)
    rng = np.random.default_rng(1)
    for qa, qb in [(Q0, Q0), (rand_q(rng), rand_q(rng))]:
        phi, n, ra, rb = O.snsd_ellipsoid(d, qa, [1, 1, 1], qb, [0.7, 0.7, 0.7])
        L = np.linalg.norm(d)
        assert abs(phi - (L - 1.7)) < 1e-13
        np.testing.assert_allclose(n, d / L, atol=1e-12)
        np.testing.assert_allclose(ra, d / L * 1.0, atol=1e-12)
        np.testing.assert_allclose(rb, -d / L * 0.7, atol=1e-12)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("gap", [1.4, 0.3, 0.0, -0.05, -0.1])
def test_shared_principal_axis(axis, gap):
    """Both bodies share a principal frame and d lies along axis i:
    Phi = |d| - a_i - b_i, for separation and shallow overlap."""
    ea, eb = np.array([1.0, 0.5, 0.7]), np.array([0.6, 0.9, 0.4])
    rng = np.random.default_rng(7)
    q = rand_q(rng)
    R = O.quat_to_R(q)
    L = ea[axis] + eb[axis] + gap
    d = R[:, axis] * L
    phi, n, ra, rb = O.snsd_ellipsoid(d, q, ea, q, eb)
    assert abs(phi - gap) < 1e-12
    np.testing.assert_allclose(n, R[:, axis], atol=1e-10)


def test_shared_normal_identity_and_surface_points():
    """p_b - p_a = Phi n (Lemma uniform interior tangent ball); p_a, p_b lie on
    the surfaces with outward normals +n and -n."""
    rng = np.random.default_rng(2)
    for _ in range(100):
        qa, qb = rand_q(rng), rand_q(rng)
        ea, eb = rng.uniform(0.3, 1.2, 3), rng.uniform(0.3, 1.2, 3)
        d = rng.normal(size=3) * 1.5
        phi, n, ra, rb = O.snsd_ellipsoid(d, qa, ea, qb, eb)
        np.testing.assert_allclose((d + rb) - ra, phi * n, atol=1e-11)
        assert abs(np.linalg.norm(n) - 1) < 1e-14
        Sa, Sb = sigma(qa, ea), sigma(qb, eb)
        assert abs(ra @ np.linalg.solve(Sa, ra) - 1) < 1e-10
        assert abs(rb @ np.linalg.solve(Sb, rb) - 1) < 1e-10
        na = np.linalg.solve(Sa, ra)
        nb = np.linalg.solve(Sb, rb)
        np.testing.assert_allclose(na / np.linalg.norm(na), n, atol=1e-9)
        np.testing.assert_allclose(nb / np.linalg.norm(nb), -n, atol=1e-9)


def _surface_distance(d, qa, ea, qb, eb, rng):
    """Independent: min over points of both surfaces of their distance."""
    Ra, Rb = O.quat_to_R(qa), O.quat_to_R(qb)

    def pt(R, e, t, p, c):
        u = np.array([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)])
        return c + R @ (e * u)

    def f(v):
        pa = pt(Ra, ea, v[0], v[1], np.zeros(3))
        pb = pt(Rb, eb, v[2], v[3], d)
        return np.sum((pa - pb) ** 2)
    def facing(R, v):
        w = R.T @ v
        w /= np.linalg.norm(w)
        return [np.arccos(np.clip(w[2], -1, 1)), np.arctan2(w[1], w[0])]
    starts = [facing(Ra, d) + facing(Rb, -d)]
    starts += [list(rng.uniform([0, 0, 0, 0], [np.pi, 2 * np.pi, np.pi, 2 * np.pi])) for _ in range(3)]
    best = np.inf
    for v0 in starts:
        r = minimize(f, np.array(v0, float), method="BFGS", options=dict(gtol=1e-13))
        best = min(best, r.fun)
    return np.sqrt(best)


def test_separated_pairs_match_surface_distance():
    rng = np.random.default_rng(3)
    done = 0
    while done < 12:
        qa, qb = rand_q(rng), rand_q(rng)
        ea, eb = rng.uniform(0.5, 1.0, 3), rng.uniform(0.5, 1.0, 3)
        d = rng.normal(size=3)
        d *= rng.uniform(1.6, 2.6) / np.linalg.norm(d)
        phi, n, ra, rb = O.snsd_ellipsoid(d, qa, ea, qb, eb)
        if phi <= 0.02:
            continue
        ref = _surface_distance(d, qa, ea, qb, eb, rng)
        assert abs(phi - ref) < 1e-6, (phi, ref)
        done += 1


def test_perram_wertheim_sign_and_touching_translation():
    """Sign of Phi agrees with the Perram-Wertheim contact function, and
    translating b by -Phi n leaves the pair exactly touching (F = 1)."""
    rng = np.random.default_rng(4)
    for _ in range(60):
        qa, qb = rand_q(rng), rand_q(rng)
        ea, eb = rng.uniform(0.5, 1.0, 3), rng.uniform(0.5, 1.0, 3)
        d = rng.normal(size=3)
        d *= rng.uniform(0.9, 2.4) / np.linalg.norm(d)
        phi, n, ra, rb = O.snsd_ellipsoid(d, qa, ea, qb, eb)
        Sa, Sb = sigma(qa, ea), sigma(qb, eb)
        F = pw_contact(d, Sa, Sb)
        if abs(F - 1) > 1e-6:
            assert (phi < 0) == (F < 1)
        F1 = pw_contact(d - phi * n, Sa, Sb)
        assert abs(F1 - 1.0) < 1e-8, (phi, F1)


def test_global_maximum_by_dense_sampling():
    """Phi is the maximum of the support gap over all directions (reading of
    'the' SNSD pair): no sampled direction beats it, and samples approach it."""
    rng = np.random.default_rng(5)
    m = 200000
    z = 1 - (2 * np.arange(m) + 1) / m
    r = np.sqrt(1 - z * z)
    ph = np.arange(m) * np.pi * (3 - np.sqrt(5))
    N = np.stack([r * np.cos(ph), r * np.sin(ph), z], axis=1)
    for _ in range(20):
        qa, qb = rand_q(rng), rand_q(rng)
        ea, eb = rng.uniform(0.5, 1.0, 3), rng.uniform(0.5, 1.0, 3)
        d = rng.normal(size=3)
        d *= rng.uniform(0.2, 2.0) / np.linalg.norm(d)
        phi, n, ra, rb = O.snsd_ellipsoid(d, qa, ea, qb, eb)
        Sa, Sb = sigma(qa, ea), sigma(qb, eb)
        f = N @ d - np.sqrt(np.einsum("ij,jk,ik->i", N, Sa, N)) - np.sqrt(np.einsum("ij,jk,ik->i", N, Sb, N))
        assert f.max() <= phi + 1e-12
        assert f.max() >= phi - 1e-4


# --------------------------------------------------------------------------
# spherocylinders
# --------------------------------------------------------------------------
def _brute_segments(d, ta, la, tb, lb, k=2001):
    s = np.linspace(-la / 2, la / 2, k)
    u = np.linspace(-lb / 2, lb / 2, k)
    P = s[:, None] * ta[None, :]
    Q = d[None, :] + u[:, None] * tb[None, :]
    best = np.inf
    for i in range(0, k, 250):
        D = Q[None, :, :] - P[i:i + 250, None, :]
        best = min(best, np.sqrt((D ** 2).sum(-1)).min())
    return best


def test_spherocylinder_brute_force():
    rng = np.random.default_rng(6)
    for _ in range(15):
        ta, tb = rng.normal(size=3), rng.normal(size=3)
        ta /= np.linalg.norm(ta)
        tb /= np.linalg.norm(tb)
        la, lb = rng.uniform(0.5, 2.5, 2)
        d = rng.normal(size=3) * 1.2
        phi, n, ra, rb = O.snsd_spherocyl(d, ta, la, 0.5, tb, lb, 0.4)
        ref = _brute_segments(d, ta, la, tb, lb) - 0.9
        # grid spacing <= 2.5/2000; distance error is second order except at clamps
        assert phi <= ref + 1e-12
        assert phi >= ref - 2e-3
        np.testing.assert_allclose((d + rb) - ra, phi * n, atol=1e-12)


def test_spherocylinder_closed_forms():
    ex, ey, ez = np.eye(3)
    # parallel, side by side with offset along the axis: distance = lateral gap
    phi, n, ra, rb = O.snsd_spherocyl(np.array([0.3, 1.5, 0.0]), ex, 2.0, 0.5, ex, 2.0, 0.5)
    assert abs(phi - 0.5) < 1e-14
    np.testing.assert_allclose(n, ey, atol=1e-14)
    # reading: midpoint of the overlap of the projections, s = (0.3 - 1 + 1) / 2
    np.testing.assert_allclose(ra, [0.15, 0.5, 0.0], atol=1e-14)
    # collinear, end to end
    phi, n, ra, rb = O.snsd_spherocyl(np.array([3.5, 0.0, 0.0]), ex, 2.0, 0.5, ex, 2.0, 0.5)
    assert abs(phi - 0.5) < 1e-14
    np.testing.assert_allclose(n, ex, atol=1e-14)
    # perpendicular, crossing at distance 1.2 along z
    phi, n, ra, rb = O.snsd_spherocyl(np.array([0.0, 0.0, 1.2]), ex, 2.0, 0.5, ey, 2.0, 0.5)
    assert abs(phi - 0.2) < 1e-14
    np.testing.assert_allclose(n, ez, atol=1e-14)
    # perpendicular T: end of b's axis at distance 1.0 from a's axis
    phi, n, ra, rb = O.snsd_spherocyl(np.array([0.2, 2.0, 0.0]), ex, 2.0, 0.5, ey, 2.0, 0.5)
    assert abs(phi - 0.0) < 1e-14
    np.testing.assert_allclose(n, ey, atol=1e-14)
    # crossing axes (touching segments): normal along t_a x t_b, signed towards d
    phi, n, ra, rb = O.snsd_spherocyl(np.array([0.0, 0.0, 0.0]), ex, 2.0, 0.5, ey, 2.0, 0.5)
    assert abs(phi + 1.0) < 1e-14
    assert abs(abs(n[2]) - 1) < 1e-14
