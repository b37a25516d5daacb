"""Pins of the oracle's LCP solvers (Sec. 2.2: Lemma monotone LCP <-> CQP,
Lemma uniqueness: D gamma unique even when gamma is not).

The exact active-set enumeration is checked against an independent bounded
QP solver (scipy L-BFGS-B on the equivalent CQP) and against the KKT
conditions; the BB projected gradient is checked against the enumeration.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O


def random_rows(rng, n, m, planar=False):
    ia = rng.integers(0, n - 1, m)
    ib = np.array([rng.integers(a + 1, n) for a in ia])
    nrm = rng.normal(size=(m, 3))
    if planar:
        nrm[:, 2] = 0
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    ra = rng.normal(size=(m, 3)) * 0.5
    rb = rng.normal(size=(m, 3)) * 0.5
    ta, tb = np.cross(ra, nrm), np.cross(rb, nrm)
    return ia.astype(np.int32), ib.astype(np.int32), nrm, ta, tb


def random_K(rng, n):
    kt = np.repeat(rng.uniform(0.2, 2.0, (n, 1)), 3, axis=1)
    Kr = np.zeros((n, 3, 3))
    for b in range(n):
        G = rng.normal(size=(3, 3))
        Kr[b] = G @ G.T + 0.1 * np.eye(3)
    return kt, Kr


def scatter(n, ia, ib, nrm, ta, tb, g):
    """Wrench D gamma (Eq. collision_ft), written with numpy index-add."""
    W = np.zeros((n, 6))
    np.add.at(W, ia, -np.concatenate([nrm, ta], 1) * g[:, None])
    np.add.at(W, ib, np.concatenate([nrm, tb], 1) * g[:, None])
    return W


def qp_reference(A, qv):
    """Independent: min_{g >= 0} 1/2 g^T A g + qv^T g by L-BFGS-B."""
    f = lambda g: 0.5 * g @ A @ g + qv @ g
    jac = lambda g: A @ g + qv
    r = minimize(f, np.zeros(qv.size), jac=jac, method="L-BFGS-B", bounds=[(0, None)] * qv.size,
                 options=dict(ftol=1e-15, gtol=1e-13, maxiter=20000))
    return r.x, r.fun


def test_one_constraint_closed_form():
    for a, q in [(2.0, -1.0), (0.5, 0.3), (3.0, 0.0), (1e-3, -1e-6)]:
        g = O.lcp_enumerate(np.array([[a]]), np.array([q]))
        assert abs(g[0] - max(0.0, -q / a)) < 1e-15


@pytest.mark.parametrize("seed", range(8))
def test_enumeration_kkt_and_independent_qp(seed):
    rng = np.random.default_rng(seed)
    n, m = 5, int(rng.integers(3, 11))
    ia, ib, nrm, ta, tb = random_rows(rng, n, m)
    kt, Kr = random_K(rng, n)
    A = O.dense_A(n, ia, ib, nrm, ta, tb, kt, Kr, 0.1)
    assert np.allclose(A, A.T, atol=1e-14)
    assert np.linalg.eigvalsh(A).min() > -1e-12
    qv = rng.normal(size=m)
    g = O.lcp_enumerate(A, qv)
    w = A @ g + qv
    assert g.min() >= 0
    assert w.min() >= -1e-10
    assert abs(g @ w) < 1e-10
    gref, fref = qp_reference(A, qv)
    f = 0.5 * g @ A @ g + qv @ g
    assert f <= fref + 1e-9
    # the wrench D gamma is unique (Lemma uniqueness, Case 2)
    W1 = scatter(n, ia, ib, nrm, ta, tb, g)
    W2 = scatter(n, ia, ib, nrm, ta, tb, gref)
    assert np.abs(W1 - W2).max() < 1e-4 * (1 + np.abs(W1).max())


@pytest.mark.parametrize("seed", range(8))
def test_bbpgd_matches_enumeration(seed):
    """BB-PGD converges to the LCP solution: same wrench D gamma as the exact
    enumeration, including rank-deficient systems (more rows than body DOF)."""
    rng = np.random.default_rng(100 + seed)
    n = 3 if seed % 2 else 6
    m = 12 if seed % 2 else int(rng.integers(4, 12))
    ia, ib, nrm, ta, tb = random_rows(rng, n, m)
    kt, Kr = random_K(rng, n)
    dt = 0.05
    A = O.dense_A(n, ia, ib, nrm, ta, tb, kt, Kr, dt)
    qv = rng.normal(size=m) * 0.1
    g_ex = O.lcp_enumerate(A, qv)
    g_bb, it, res = O.lcp_bbpgd_rows(n, ia, ib, nrm, ta, tb, kt, Kr, dt, qv, tol=1e-13)
    assert it >= 0 and res <= 1e-13
    w = A @ g_bb + qv
    assert g_bb.min() >= 0 and w.min() >= -1e-12
    W1 = scatter(n, ia, ib, nrm, ta, tb, g_ex)
    W2 = scatter(n, ia, ib, nrm, ta, tb, g_bb)
    assert np.abs(W1 - W2).max() < 1e-8 * (1 + np.abs(W1).max())
    # where the active block is nonsingular gamma itself is unique
    act = g_ex > 1e-12
    if act.any() and np.linalg.matrix_rank(A[np.ix_(act, act)]) == act.sum():
        assert np.abs(g_ex - g_bb).max() < 1e-7 * (1 + np.abs(g_ex).max())


def test_bbpgd_warm_start_and_zero_rhs():
    rng = np.random.default_rng(9)
    n, m = 4, 8
    ia, ib, nrm, ta, tb = random_rows(rng, n, m)
    kt, Kr = random_K(rng, n)
    qv = np.abs(rng.normal(size=m))  # separating: solution gamma = 0
    g, it, res = O.lcp_bbpgd_rows(n, ia, ib, nrm, ta, tb, kt, Kr, 0.1, qv, gamma0=np.ones(m), tol=1e-14)
    assert np.all(g == 0.0)
    # a converged warm start needs no iteration
    qv = rng.normal(size=m)
    g1, it1, _ = O.lcp_bbpgd_rows(n, ia, ib, nrm, ta, tb, kt, Kr, 0.1, qv, tol=1e-12)
    g2, it2, _ = O.lcp_bbpgd_rows(n, ia, ib, nrm, ta, tb, kt, Kr, 0.1, qv, gamma0=g1, tol=1e-12)
    assert it2 == 0 and np.array_equal(g1, g2)
