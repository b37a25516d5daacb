"""Pins of the colony's growth and division (Sec. 5.3) as the oracle's side
of the colony tests writes them: a divided cell's halves fill the parent
tip to tip (outer tips at the parent's tips, inner tips meeting at its
centre, checked with the oracle's spherocylinder SNSD: the halves touch,
Phi = 0), lengths halve, the jitter turns each half about z, and a single
growing cell does not move."""
import numpy as np
import pytest

import oracle as O
from paper_2506_14097_amd import inputs as I

from colony_ref import divide, grow, same_rotation


@pytest.mark.parametrize("l,r", [(1.0, 0.5), (3.5, 0.25), (2.0, 0.5)])
def test_halves_fill_the_parent(l, r):
    th = 0.7
    x = np.array([[1.0, -2.0, 0.0]])
    q = I.planar_quaternions(np.array([th]))
    shape = np.array([[r, l, 0.0]])
    x2, q2, s2, rho2, nd = divide(x, q, shape, np.ones(1), l, np.zeros(2))
    assert nd == 1 and len(x2) == 2
    t = np.array([np.cos(th), np.sin(th), 0.0])
    ld = 0.5 * l - r
    assert np.allclose(s2[:, 1], ld) and np.allclose(s2[:, 0], r)
    # outer tips at the parent's tips, inner tips at the parent's centre
    tip = 0.5 * l + r
    half = 0.5 * ld + r
    assert np.allclose(x2[0] + half * t, x[0] + tip * t, atol=1e-14)
    assert np.allclose(x2[1] - half * t, x[0] - tip * t, atol=1e-14)
    assert np.allclose(x2[0] - half * t, x[0], atol=1e-14) and np.allclose(x2[1] + half * t, x[0], atol=1e-14)
    assert same_rotation(q2, np.repeat(q, 2, 0)) < 1e-15
    # the halves touch: the oracle's SNSD of the pair is zero
    out = O.snsd_pairs([0], [1], x2, q2, np.ones(2, np.int32), s2, np.zeros(3), planar=1)
    assert abs(out[0, 0]) < 1e-12


def test_jitter_turns_each_half_about_z():
    q = I.planar_quaternions(np.array([0.3]))
    x2, q2, s2, _, _ = divide(np.zeros((1, 3)), q, np.array([[0.5, 1.0, 0.0]]), np.ones(1), 1.0, [0.01, -0.02])
    assert same_rotation(q2[:1], I.planar_quaternions(np.array([0.31]))) < 1e-15
    assert same_rotation(q2[1:], I.planar_quaternions(np.array([0.28]))) < 1e-15
    # several parents: halves appended in parent order, short cells kept
    x = np.array([[0.0, 0, 0], [5.0, 0, 0], [10.0, 0, 0]])
    q = I.planar_quaternions(np.zeros(3))
    shape = np.array([[0.5, 1.0, 0], [0.5, 0.4, 0], [0.5, 1.2, 0]])
    x2, q2, s2, _, nd = divide(x, q, shape, np.ones(3), 1.0, np.zeros(4))
    assert nd == 2 and len(x2) == 5
    assert np.allclose(x2[:, 0], [0.5, 5.0, 10.55, -0.5, 9.45])
    assert np.allclose(s2[:, 1], [0.0, 0.4, 0.1, 0.0, 0.1])


def test_single_growing_cell_does_not_move():
    x = np.zeros((1, 3))
    q = I.planar_quaternions(np.array([0.4]))
    shape = np.array([[0.5, 0.2, 0.0]])
    for _ in range(5):
        shape = grow(shape, 1e-3)
        r = O.relcp_step(x, q, np.ones(1, np.int32), shape, np.ones(1), np.zeros(3), dt=1e-2, eps=1e-3, tol=1e-12,
                         skin=0.05, planar=1)
        assert r["status"] == 0 and r["n_rows"] == 0
        assert np.array_equal(r["x"], x) and same_rotation(r["q"], q) == 0
    assert abs(shape[0, 1] - 0.205) < 1e-15
