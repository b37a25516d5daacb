"""Pins of the oracle's torus SNSD (Sec. 6, non-convex rings: the distance
between the two centre circles minus the two minor radii) and of a ReLCP
step between rings:

* closed forms: coplanar rings side by side, coaxial rings (a continuum of
  closest pairs: only Phi is unique), a point against a circle (major radius
  0: the torus is a sphere), two circles that pass through each other's
  centre (a continuum again);
* brute force over a grid of both circle angles on random pairs, with the
  first-order conditions at the returned points (the segment between them
  is normal to both circles) and the points on their circles;
* symmetries: exchanging the bodies, a rigid rotation of the pair;
* a step: two interlaced rings pulled apart by equal and opposite forces
  (a taut chain link), and two coplanar rings pressed together, where the
  multiplier is exactly the force and the rings stay touching;
* the chainmail input (linked, apart, the slack exact), the extensile field,
  and the contrast of Sec. 6: ReLCP within the overlap tolerance where the
  single-constraint SNSD LCP overlaps beyond it.
"""
import numpy as np
import pytest

import oracle as O


def rot(seed):
    q = np.random.default_rng(seed).normal(size=4)
    q /= np.linalg.norm(q)
    return O.quat_to_R(q)


def check_contact(d, Ra, ra, Rb, rb, ea, eb, res):
    """Points on the tube surfaces, Phi = separation along n, centre-circle
    points on their circles."""
    phi, n, pa, pb = res[:4]
    assert abs(np.linalg.norm(n) - 1) < 1e-12
    # (x_b + r_b) - (x_a + r_a) = Phi n
    np.testing.assert_allclose(d + pb - pa, phi * n, atol=1e-11)
    ca = pa - ra * n                 # centre-circle point of a (relative to x_a)
    cb = pb + rb * n                 # centre-circle point of b (relative to x_b)
    assert abs(ca @ ea) < 1e-11 and abs(np.linalg.norm(ca) - Ra) < 1e-11
    assert abs(cb @ eb) < 1e-11 and abs(np.linalg.norm(cb) - Rb) < 1e-11
    return ca, cb


@pytest.mark.parametrize("seed", range(4))
def test_coplanar_rings_closed_form(seed):
    rng = np.random.default_rng(seed)
    R = rot(seed)
    Ra, Rb, ra, rb = rng.uniform(0.5, 1.5, 2).tolist() + rng.uniform(0.02, 0.2, 2).tolist()
    D = Ra + Rb + ra + rb + rng.uniform(0.01, 1.0)
    ang = rng.uniform(0, 2 * np.pi)
    dh = np.array([np.cos(ang), np.sin(ang), 0.0])
    e = np.array([0, 0, 1.0])
    d = D * dh
    phi, n, pa, pb, margin = O.snsd_torus(R @ d, R @ e, Ra, ra, R @ e, Rb, rb)
    assert abs(phi - (D - Ra - Rb - ra - rb)) < 1e-12
    np.testing.assert_allclose(n, R @ dh, atol=1e-12)
    np.testing.assert_allclose(pa, (Ra + ra) * (R @ dh), atol=1e-12)
    np.testing.assert_allclose(pb, -(Rb + rb) * (R @ dh), atol=1e-12)
    assert margin > D - Ra - Rb + 0.1  # the next local minimum is far worse


@pytest.mark.parametrize("seed", range(3))
def test_coaxial_rings_closed_form(seed):
    rng = np.random.default_rng(10 + seed)
    R = rot(10 + seed)
    Ra, Rb, ra, rb, h = rng.uniform(0.4, 1.2, 2).tolist() + rng.uniform(0.02, 0.1, 2).tolist() + [0.7]
    e = R @ np.array([0, 0, 1.0])
    res = O.snsd_torus(h * e, e, Ra, ra, e, Rb, rb)
    assert abs(res[0] - (np.hypot(h, Ra - Rb) - ra - rb)) < 1e-12
    check_contact(h * e, Ra, ra, Rb, rb, e, e, res)
    assert res[4] - (res[0] + ra + rb) < 1e-9  # a continuum: no unique minimum


@pytest.mark.parametrize("seed", range(4))
def test_point_against_circle(seed):
    """Major radius 0: body a is a sphere of radius r_a; the distance from its
    centre to circle b is sqrt(h^2 + (rho - R_b)^2)."""
    rng = np.random.default_rng(20 + seed)
    eb = rot(20 + seed)[:, 2]
    d = rng.uniform(-2, 2, 3)
    Rb, ra, rb = 1.1, 0.15, 0.05
    w = -d                             # the sphere centre seen from x_b
    h = w @ eb
    rho = np.linalg.norm(w - h * eb)
    phi, n, pa, pb, _ = O.snsd_torus(d, np.array([0, 0, 1.0]), 0.0, ra, eb, Rb, rb)
    assert abs(phi - (np.hypot(h, rho - Rb) - ra - rb)) < 1e-12
    # both radii 0: two spheres
    phi2, n2, _, _, _ = O.snsd_torus(d, np.array([0, 0, 1.0]), 0.0, ra, eb, 0.0, rb)
    assert abs(phi2 - (np.linalg.norm(d) - ra - rb)) < 1e-12
    np.testing.assert_allclose(n2, d / np.linalg.norm(d), atol=1e-12)


def test_circles_through_each_others_centre():
    """Circle a in the xy-plane at 0, circle b in the xz-plane at (R, 0, 0):
    |c_a - c_b|^2 = R^2 (3 - 2X + 2Y - 2XY) with X = cos(t_a), Y = cos(t_b),
    smallest (R^2) along Y = -1 for every X: Phi = R - r_a - r_b."""
    R, r = 1.0, 0.1
    res = O.snsd_torus(np.array([R, 0, 0]), np.array([0, 0, 1.0]), R, r, np.array([0, 1.0, 0]), R, r)
    assert abs(res[0] - (R - 2 * r)) < 1e-12
    check_contact(np.array([R, 0, 0]), R, r, R, r, np.array([0, 0, 1.0]), np.array([0, 1.0, 0]), res)


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_grid_and_stationarity(seed):
    rng = np.random.default_rng(30 + seed)
    Ma, Mb = rot(30 + seed), rot(60 + seed)
    Ra, Rb = rng.uniform(0.6, 1.2, 2)
    ra, rb = 0.1, 0.08
    d = rng.uniform(-1.5, 1.5, 3)
    # grid over both angles, each circle in its own body frame
    t = np.linspace(0, 2 * np.pi, 1600, endpoint=False)
    ca = Ra * (np.outer(np.cos(t), Ma[:, 0]) + np.outer(np.sin(t), Ma[:, 1]))
    cb = d + Rb * (np.outer(np.cos(t), Mb[:, 0]) + np.outer(np.sin(t), Mb[:, 1]))
    dist = np.sqrt(((ca[:, None, :] - cb[None, :, :]) ** 2).sum(-1)).min()
    res = O.snsd_torus(d, Ma[:, 2], Ra, ra, Mb[:, 2], Rb, rb)
    dc = res[0] + ra + rb
    step = 2 * np.pi / 1600
    assert dc <= dist + 1e-12
    assert dist - dc <= 0.5 * (Ra + Rb) * step
    ca, cb = check_contact(d, Ra, ra, Rb, rb, Ma[:, 2], Mb[:, 2], res)
    w = d + cb - ca
    if np.linalg.norm(w) > 1e-6:
        # first-order conditions: the segment between the centre-circle
        # points is normal to both circles' tangents there
        ta, tb = np.cross(Ma[:, 2], ca), np.cross(Mb[:, 2], cb)
        assert abs(w @ ta) < 1e-12 and abs(w @ tb) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_exchange_and_rotation(seed):
    rng = np.random.default_rng(90 + seed)
    Ma, Mb, Q = rot(90 + seed), rot(120 + seed), rot(150 + seed)
    d = rng.uniform(-1.5, 1.5, 3)
    A = (Ma[:, 2], 1.0, 0.1)
    B = (Mb[:, 2], 0.8, 0.07)
    phi, n, pa, pb, margin = O.snsd_torus(d, A[0], A[1], A[2], B[0], B[1], B[2])
    phi2, n2, pa2, pb2, _ = O.snsd_torus(-d, B[0], B[1], B[2], A[0], A[1], A[2])
    phi3, n3, pa3, pb3, _ = O.snsd_torus(Q @ d, Q @ A[0], A[1], A[2], Q @ B[0], B[1], B[2])
    assert abs(phi - phi2) < 1e-12 and abs(phi - phi3) < 1e-12
    if margin - (phi + 0.17) > 1e-6:   # unique closest pair: the points agree too
        np.testing.assert_allclose(n2, -n, atol=1e-9)
        np.testing.assert_allclose(pa2, pb, atol=1e-9)
        np.testing.assert_allclose(n3, Q @ n, atol=1e-9)
        np.testing.assert_allclose(pa3, Q @ pa, atol=1e-9)


def _ring_q(axis):
    """Quaternion taking the body z axis to the given coordinate axis."""
    if axis == "z":
        return [1.0, 0, 0, 0]
    if axis == "y":   # rotation by -90 degrees about x: z -> y
        return [np.cos(-np.pi / 4), np.sin(-np.pi / 4), 0, 0]
    return [np.cos(np.pi / 4), 0, np.sin(np.pi / 4), 0]  # +90 about y: z -> x


def test_quaternion_helper_axes():
    for ax, e in (("z", [0, 0, 1]), ("y", [0, 1, 0]), ("x", [1, 0, 0])):
        np.testing.assert_allclose(O.quat_to_R(_ring_q(ax))[:, 2], e, atol=1e-15)


def test_interlaced_rings_pulled_apart():
    """Ring a flat at 0, ring b (axis y) threaded through it at (s, 0, 0) with
    s = 2 (R - r): the tubes touch at (R - r, 0, 0) with n = -x.  Pulled
    apart by F, the multiplier is F and both rings stop."""
    R, r, F = 1.0, 0.1, 0.6
    s = 2 * (R - r)
    x = np.array([[0, 0, 0], [s, 0, 0]], float)
    q = np.array([_ring_q("z"), _ring_q("y")])
    shape = np.array([[R, r, 0.0]] * 2)
    kind = np.full(2, 2, np.int32)
    snsd = O.snsd_pairs([0], [1], x, q, kind, shape, np.zeros(3))[0]
    assert abs(snsd[0]) < 1e-12
    np.testing.assert_allclose(snsd[1:4], [-1, 0, 0], atol=1e-12)
    fext = np.zeros((2, 6))
    fext[0, 0], fext[1, 0] = -F, F
    res = O.relcp_step(x, q, kind, shape, np.array([1.0, 2.0]), np.zeros(3), dt=0.05, eps=1e-9, tol=1e-14,
                       skin=0.1, fext=fext)
    assert res["status"] == 0
    assert abs(res["gamma"].sum() - F) < 1e-13
    np.testing.assert_allclose(res["U"], 0.0, atol=1e-14)


def test_coplanar_rings_pressed_together():
    R, r, F = 1.0, 0.1, 0.4
    x = np.array([[0, 0, 0], [2 * (R + r), 0, 0]], float)
    q = np.array([_ring_q("z")] * 2)
    fext = np.zeros((2, 6))
    fext[0, 0], fext[1, 0] = F, -F
    res = O.relcp_step(x, q, np.full(2, 2, np.int32), np.array([[R, r, 0.0]] * 2), np.array([1.0, 1.0]),
                       np.zeros(3), dt=0.05, eps=1e-9, tol=1e-14, skin=0.1, fext=fext)
    assert res["status"] == 0
    assert abs(res["gamma"].sum() - F) < 1e-13
    np.testing.assert_allclose(res["U"], 0.0, atol=1e-14)


def test_torus_mobility_length():
    """Overdamped local drag with L = 2 (R + r), the outer diameter."""
    R, r, xi = 1.0, 0.1, 2.0
    kt, Kr = O.body_K(0, 0, 0.01, np.array([2], np.int32), np.array([[R, r, 0.0]]), np.array([[1.0, 0, 0, 0]]),
                      np.array([xi]))
    L = 2 * (R + r)
    np.testing.assert_allclose(np.ravel(kt)[:3], 1 / (xi * L), rtol=1e-15)
    np.testing.assert_allclose(np.ravel(Kr)[[0, 4, 8]], 12 / (xi * L ** 3), rtol=1e-15)


def test_chainmail_lattice_linked_and_apart():
    """The chainmail input: no two rings overlap (oracle SNSD over every pair
    within reach), each connector's centre circle crosses the plane of the
    node rings inside the holes of both rings of its edge, and stretching an
    edge closes exactly the stated slack before the tubes touch."""
    from paper_2506_14097_amd import inputs as I
    for slack in (0.45, 0.05):
        S = I.chainmail(3, 3, slack=slack)
        x, q, shape = S["x"], S["q"], S["shape"]
        pa, pb = O.broadphase(x, S["kind"], shape, S["box"], 0.5)
        phi = O.snsd_pairs(pa, pb, x, q, S["kind"], shape, S["box"])[:, 0]
        assert phi.min() > 0 and abs(phi.min() - min(slack, np.sqrt(2) * (S["spacing"] / 2 - 1) - 0.2)) < 1e-12
        nodes = x[:S["n_nodes"]]
        R, r = shape[0, 0], shape[0, 1]
        for k in range(S["n_nodes"], len(x)):
            e = O.quat_to_R(q[k])[:, 2]
            u = np.cross(e, [0, 0, 1.0])          # horizontal, in the connector's plane
            for p in (x[k] + R * u, x[k] - R * u):   # where its centre circle meets z = 0
                dn = np.linalg.norm(nodes - p, axis=1).min()
                assert dn < R - 2 * r
        # the link of the first edge: node 0 and its connector, gap along x
        k = S["n_nodes"]
        out = O.snsd_pairs([0], [k], x, q, S["kind"], shape, S["box"])[0]
        assert abs(out[0] - slack) < 1e-12


def test_extensile_field():
    from paper_2506_14097_amd import inputs as I
    x = np.array([[0, 0, 0], [3.0, 4.0, 0.0], [0, 0, 9.99e-4], [0, 0, 1.001e-3]])
    f = I.extensile_field(x)
    np.testing.assert_array_equal(f[0], 0.0)
    np.testing.assert_allclose(f[1, :3], x[1] * (5 - np.sin(5)) / 25, rtol=1e-15)
    assert np.all(f[:, 3:] == 0)
    # the series and the direct form meet smoothly at |x| = 1e-3
    assert abs(f[2, 2] / 9.99e-4 ** 2 - f[3, 2] / 1.001e-3 ** 2) < 1e-6


def test_chainmail_augmentation_holds_the_tolerance():
    """Sec. 6: on a chainmail pulled taut at a timestep outside the linear
    regime, ReLCP keeps every accepted configuration within the overlap
    tolerance by appending constraints, while the single-constraint SNSD LCP
    (no recursions) overlaps beyond it (3 x 3 nodes, drag 0.1, dt 1e-3)."""
    from paper_2506_14097_amd import inputs as I
    out = {}
    for mr in (64, 0):
        S = I.chainmail(3, 3, slack=0.05, xi=0.1, jitter=0.05)
        x, q, prev, worst, nrec = S["x"], S["q"], None, 0.0, 0
        for _ in range(50):
            ref = O.relcp_step(x, q, S["kind"], S["shape"], S["rho_xi"], S["box"], dt=1e-3, eps=1e-5, tol=1e-9,
                               skin=0.1, fext=I.extensile_field(x), max_recursions=mr, prev=prev)
            assert ref["status"] == 0
            x, q, prev = ref["x"], ref["q"], O.pair_lambda(ref)
            worst = max(worst, ref["max_overlap"])
            nrec += ref["recursions"] > 0
        out[mr] = (worst, nrec)
    assert out[64][0] <= 1e-5 and out[64][1] >= 10
    assert out[0][0] > 2e-5 and out[0][1] == 0
