"""Pins of the FP64 MLP oracle (learned warm start): identities of GELU,
bfloat16 rounding on representable neighbours, the analytic
gradient against central finite differences, the first Adam step in closed
form, and that plain training lowers the loss."""
import math

import numpy as np
import pytest

from oracle import mlp as M


def test_gelu_identities():
    t = np.linspace(-6, 6, 241)
    # x Phi(x) with Phi(x) + Phi(-x) = 1  =>  GELU(x) - GELU(-x) = x
    np.testing.assert_allclose(M.gelu(t) - M.gelu(-t), t, atol=1e-14)
    assert M.gelu(0.0) == 0.0
    assert abs(M.gelu_prime(0.0) - 0.5) < 1e-15
    assert abs(M.gelu(40.0) - 40.0) < 1e-12 and abs(M.gelu(-40.0)) < 1e-12
    # derivative against central differences
    h = 1e-6
    np.testing.assert_allclose(M.gelu_prime(t), (M.gelu(t + h) - M.gelu(t - h)) / (2 * h), atol=1e-8)



def test_bf16_rounding():
    one = 1.0
    ulp = 2.0 ** -7
    assert M.bf16(one) == one
    assert M.bf16(one + ulp / 2) == one                     # tie -> even
    assert M.bf16(one + 3 * ulp / 2) == one + 2 * ulp       # tie -> even (up)
    assert M.bf16(one + 0.75 * ulp) == one + ulp
    assert M.bf16(math.pi) == 3.140625
    assert M.bf16(-2.0) == -2.0


def _batch(seed, B=40):
    rng = np.random.default_rng(seed)
    flat = M.init_params(seed)
    flat = flat + 0.05 * rng.normal(size=flat.size)  # nonzero biases
    X = rng.normal(size=(B, M.F))
    y = np.abs(rng.normal(size=B))
    return flat, X, y


def test_gradient_matches_finite_differences():
    flat, X, y = _batch(0)
    g = M.grad(flat, X, y)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(np.arange(0, 1024), 30, replace=False),     # W1
                          rng.choice(np.arange(1024, 1152), 10, replace=False),  # b1
                          rng.choice(np.arange(1152, 17536), 40, replace=False),  # W2
                          rng.choice(np.arange(17536, 17664), 10, replace=False),  # b2
                          rng.choice(np.arange(17664, 17792), 10, replace=False),  # w3
                          [17792]])                                                # b3
    h = 1e-6
    for k in idx:
        e = np.zeros_like(flat)
        e[k] = h
        fd = (M.loss(flat + e, X, y) - M.loss(flat - e, X, y)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])) + 1e-10, (k, fd, g[k])
    assert M.NPARAM == 17793 and g.size == 17793


def test_emulated_gradient_is_close_to_exact():
    flat, X, y = _batch(2)
    g0 = M.grad(flat, X, y)
    g1 = M.grad(flat, X, y, emulate=True)
    assert np.linalg.norm(g1 - g0) < 3e-2 * np.linalg.norm(g0)


def test_first_adam_step_closed_form():
    flat = np.zeros(5)
    g = np.array([0.3, -2.0, 1e-3, -1e-5, 7.0])
    new, m, v = M.adam(flat, g, np.zeros(5), np.zeros(5), 1, 0.01)
    # bias-corrected moments are g and g^2 on the first step: update = -lr g/(|g| + eps)
    np.testing.assert_allclose(new, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_lowers_loss():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(256, M.F))
    y = np.log1p(np.exp(0.5 * X[:, 0] - 0.3 * X[:, 2]))  # a smooth target
    flat = M.init_params(4)
    m = np.zeros_like(flat)
    v = np.zeros_like(flat)
    l0 = M.loss(flat, X, y)
    for t in range(1, 151):
        flat, m, v = M.adam(flat, M.grad(flat, X, y), m, v, t, 3e-3)
    assert M.loss(flat, X, y) < 0.2 * l0


# --------------------------------------------------------------------------
# features of the iteration-0 rows
# --------------------------------------------------------------------------
import oracle as O  # noqa: E402


def _qaxis(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    return np.concatenate([[math.cos(ang / 2)], math.sin(ang / 2) * axis])


def test_semi_extents():
    np.testing.assert_allclose(M._semi_extents(0, [1.0, 0.5, 0.25]), [1.0, 0.5, 0.25])
    # spherocylinder (r, l): l/2 + r along the axis, r across
    np.testing.assert_allclose(M._semi_extents(1, [0.5, 2.0, 0]), [1.5, 0.5, 0.5])


def test_features_three_spheres_by_hand():
    """Sphere 0 (r = 1) touches spheres 1 and 2 (r = 0.5) at gaps 0.1 and
    0.2; sphere 0 moved along +x at speed 2 in the previous step."""
    x = np.array([[0.0, 0, 0], [1.6, 0, 0], [0, 1.7, 0]])
    q = np.tile([1.0, 0, 0, 0], (3, 1))
    shape = np.array([[1.0, 1, 1], [0.5, 0.5, 0.5], [0.5, 0.5, 0.5]])
    kind = np.zeros(3, np.int32)
    dt = 1e-3
    step = O.relcp_step(x, q, kind, shape, np.ones(3), np.zeros(3), dt=dt, eps=1e-6, tol=1e-12, skin=0.5)
    assert step["status"] == 0
    u_prev = np.zeros((3, 6))
    u_prev[0, 0] = 2.0
    prev = (np.array([0], np.int32), np.array([1], np.int32), np.array([0.25]))
    ia, ib, X, rs = M.features(q, kind, shape, np.ones(3), u_prev, prev, step, dt)
    order = np.argsort(ib)
    ia, ib, X, rs = ia[order], ib[order], X[order], rs[order]
    assert list(ia) == [0, 0] and list(ib) == [1, 2]
    abar = 0.75
    # spheres: no lever arm, overdamped mobility 1 / (xi L), L = diameter,
    # so A_aa = dt (1/2 + 1/1)
    np.testing.assert_allclose(rs, abar / (1.5 * dt), rtol=1e-12)
    np.testing.assert_allclose(X[:, 0], [0.1 / abar, 0.2 / abar], atol=1e-12)
    # D^T U along (0,1) = -(n . u_0) = -2 ; along (0,2) n = e_y: 0
    np.testing.assert_allclose(X[:, 1], [-2 * dt / abar, 0.0], atol=1e-14)
    np.testing.assert_allclose(X[:, 2], [0.25 * 1.5 * dt / abar, 0.0], rtol=1e-12)
    # separated spheres: no multiplier, so zero targets
    np.testing.assert_allclose(M.targets(step, rs[np.argsort(order)]), 0.0)
    np.testing.assert_allclose(X[:, 3:5], [[2, 1], [2, 1]])
    np.testing.assert_allclose(X[:, 5:7], 1.0)
    np.testing.assert_allclose(X[:, 7], 0.0)           # no overlaps around


def test_features_orientation_by_index():
    """Relabelling the bodies swaps the a/b features of a row and inverts
    the support ratio; the symmetric features stay."""
    x = np.array([[0.0, 0, 0], [1.45, 0.2, 0]])
    q = np.array([_qaxis([0, 0, 1], 0.3), _qaxis([1, 1, 0], 1.1)])
    shape = np.array([[1.0, 0.6, 0.5], [0.7, 0.5, 0.45]])
    kind = np.zeros(2, np.int32)
    u = np.array([[0.3, 0, 0.1, 0, 0.2, 0], [-0.1, 0.2, 0, 0.5, 0, 0]])
    s1 = O.relcp_step(x, q, kind, shape, np.ones(2), np.zeros(3), dt=1e-3, eps=1e-6, tol=1e-12, skin=0.5)
    s2 = O.relcp_step(x[::-1], q[::-1], kind, shape[::-1], np.ones(2), np.zeros(3), dt=1e-3, eps=1e-6, tol=1e-12,
                      skin=0.5)
    _, _, X1, r1 = M.features(q, kind, shape, np.ones(2), u, None, s1, 1e-3)
    _, _, X2, r2 = M.features(q[::-1], kind, shape[::-1], np.ones(2), u[::-1], None, s2, 1e-3)
    np.testing.assert_allclose(r1, r2, rtol=1e-9)
    assert X1.shape == (1, 8) and X2.shape == (1, 8)
    np.testing.assert_allclose(X1[0, :3], X2[0, :3], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(X1[0, [3, 5]], X2[0, [4, 6]])
    np.testing.assert_allclose(X1[0, [4, 6]], X2[0, [3, 5]])
    assert X1[0, 5] != X1[0, 6]


def test_target_of_one_overlapping_pair():
    """One row: the LCP gives gamma = -Phi_0 / A_aa, so the target in length
    units is -Phi_0 / abar, whatever the mobility."""
    for r_b, xi in ((1.0, 1.0), (0.5, 3.0)):
        x = np.array([[0.0, 0, 0], [1.0 + r_b - 0.01, 0, 0]])
        shape = np.array([[1.0, 1, 1], [r_b, r_b, r_b]])
        q = np.tile([1.0, 0, 0, 0], (2, 1))
        step = O.relcp_step(x, q, np.zeros(2, np.int32), shape, np.full(2, xi), np.zeros(3), dt=1e-3, eps=1e-9,
                            tol=1e-14, skin=0.1, max_recursions=0)
        _, _, X, rs = M.features(q, np.zeros(2, np.int32), shape, np.full(2, xi), None, None, step, 1e-3)
        abar = 0.5 * (1.0 + r_b)
        np.testing.assert_allclose(X[0, 0], -0.01 / abar, rtol=1e-9)
        np.testing.assert_allclose(M.targets(step, rs), [0.01 / abar], rtol=1e-8)


def test_neighbourhood_overlap_load():
    """Sphere 0 (r = 1) overlaps spheres 1 and 2 (r = 0.5) by 0.01 and 0.02,
    and sphere 1 overlaps sphere 3 by 0.03: each row sees the overlaps of
    the other rows at its two bodies."""
    x = np.array([[0.0, 0, 0], [1.49, 0, 0], [0, 1.48, 0], [2.46, 0, 0]])
    q = np.tile([1.0, 0, 0, 0], (4, 1))
    shape = np.array([[1.0, 1, 1], [0.5, 0.5, 0.5], [0.5, 0.5, 0.5], [0.5, 0.5, 0.5]])
    kind = np.zeros(4, np.int32)
    step = O.relcp_step(x, q, kind, shape, np.ones(4), np.zeros(3), dt=1e-3, eps=1e-6, tol=1e-12, skin=0.2,
                        max_recursions=0)
    assert step["status"] == 0
    ia, ib, X, _ = M.features(q, kind, shape, np.ones(4), None, None, step, 1e-3)
    got = {(int(a), int(b)): X[k] for k, (a, b) in enumerate(zip(ia, ib))}
    assert set(got) == {(0, 1), (0, 2), (1, 3)}
    np.testing.assert_allclose(got[(0, 1)][7], (0.02 + 0.03) / 0.75, rtol=1e-9)
    np.testing.assert_allclose(got[(0, 2)][7], 0.01 / 0.75, rtol=1e-9)
    np.testing.assert_allclose(got[(1, 3)][7], 0.01 / 0.5, rtol=1e-9)
    np.testing.assert_allclose([got[k][3] for k in ((0, 1), (0, 2), (1, 3))], [2, 2, 2])
    np.testing.assert_allclose([got[k][4] for k in ((0, 1), (0, 2), (1, 3))], [2, 1, 1])


def test_start_reduces_to_previous_multiplier_and_clips():
    """With a zero output layer (z = 0) the start is the previous-step
    multiplier; a negative correction clips at zero."""
    rng = np.random.default_rng(9)
    X = np.abs(rng.normal(size=(20, M.F)))
    norm = np.concatenate([np.zeros(8), np.ones(8), [0.5]])
    P = M.unpack(M.init_params(1))
    P["w3"] = np.zeros(M.H)
    P["b3"] = 0.0
    np.testing.assert_allclose(M.predict(M.pack(P), X, norm), X[:, 2])
    P["b3"] = -1e3
    np.testing.assert_allclose(M.predict(M.pack(P), X, norm), 0.0)
    P["b3"] = 0.25
    np.testing.assert_allclose(M.predict(M.pack(P), X, norm), X[:, 2] + 0.125)
    np.testing.assert_allclose(M.correction_target(X, X[:, 2] + 0.125, norm), 0.25)
