"""The oracle's cell-grid candidate search against its all-pairs search.

The step switches to the cell grid for large systems; the two must give the
same pairs in the same order (every a < b with bounding-sphere gap <= skin,
sorted by (a, b); the near-contacting pairs of Alg. 1).  Cases: periodic
packings, boxes of one or two cells per direction (neighbour cells wrap onto
themselves), open domains (sparse and dense), rods in a monolayer, mixed
sizes, a single body, and bodies on cell boundaries.
"""
import numpy as np
import pytest

import oracle as O
from paper_2506_14097_amd import inputs as I


def _same(x, kind, shape, box, skin):
    a0, b0 = O.broadphase(x, kind, shape, box, skin)
    a1, b1 = O.broadphase(x, kind, shape, box, skin, cells=True)
    assert np.array_equal(a0, a1) and np.array_equal(b0, b1)
    return a0.size


@pytest.mark.parametrize("seed", [0, 1])
def test_cells_periodic_packing(seed):
    P = I.ellipsoid_packing(seed, 3000, sphere_phi=0.3, compress=0.97)
    assert _same(P["x"], P["kind"], P["shape"], P["box"], 0.05) > 1000
    assert _same(P["x"], P["kind"], P["shape"], P["box"], 0.4) > 3000


@pytest.mark.parametrize("edge", [1.7, 2.9, 4.5])
def test_cells_small_periodic_boxes(edge):
    rng = np.random.default_rng(4)
    nb = 60
    x = rng.uniform(-edge, 2 * edge, (nb, 3))  # positions outside the box wrap
    shape = rng.uniform(0.3, 0.6, (nb, 3))
    assert _same(x, np.zeros(nb, np.int32), shape, np.full(3, edge), 0.1) > 0


def test_cells_open_domains():
    rng = np.random.default_rng(5)
    for spread, nb in ((20.0, 700), (400.0, 900), (6.0, 500)):
        x = rng.uniform(-spread, spread, (nb, 3))
        _same(x, np.zeros(nb, np.int32), rng.uniform(0.5, 1.0, (nb, 3)), np.zeros(3), 0.2)
    # a slab open along z, periodic along x and y
    x = rng.uniform(0, 15, (800, 3)) * [1, 1, 0.2]
    assert _same(x, np.zeros(800, np.int32), rng.uniform(0.5, 1.0, (800, 3)), np.array([15.0, 15.0, 0.0]), 0.1) > 0


def test_cells_rods_mixed_sizes_and_edges():
    S = I.spherocylinder_monolayer(3, 400, disk_fraction=0.4)
    assert _same(S["x"], S["kind"], S["shape"], S["box"], 0.2) > 0
    rng = np.random.default_rng(6)
    nb = 500
    shape = np.where(rng.random((nb, 1)) < 0.1, 3.0, 0.5) * np.ones((nb, 3))
    x = rng.uniform(0, 30, (nb, 3))
    assert _same(x, np.zeros(nb, np.int32), shape, np.full(3, 30.0), 0.3) > 0
    # bodies exactly on cell boundaries and on the box faces
    h = 2.0 + 0.1
    g = np.arange(0, 4) * h
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    assert _same(x, np.zeros(len(x), np.int32), np.ones((len(x), 3)), np.full(3, 4 * h), 0.1) > 0
    assert _same(np.zeros((1, 3)), np.zeros(1, np.int32), np.ones((1, 3)), np.zeros(3), 0.1) == 0


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_pair_snsd_independent_of_threads(kind):
    """The oracle shares pairs among OpenMP threads; every pair's result is
    the same with one thread and with several (no state shared between
    pairs)."""
    rng = np.random.default_rng(1)
    nb = 250
    x = rng.uniform(0, 6.0, (nb, 3))
    q = I.shoemake_quaternions(rng, nb)
    if kind == 0:
        shape = rng.uniform(0.5, 1.0, (nb, 3))
    elif kind == 1:
        shape = np.stack([np.full(nb, 0.5), rng.uniform(0.0, 2.0, nb), np.zeros(nb)], 1)
    else:
        shape = np.stack([rng.uniform(0.6, 1.2, nb), rng.uniform(0.05, 0.15, nb), np.zeros(nb)], 1)
    k = np.full(nb, kind, np.int32)
    pa, pb = O.broadphase(x, k, shape, np.zeros(3), 0.3)
    assert pa.size > 100
    was = O.threads()
    try:
        O.threads(1)
        a = O.snsd_pairs(pa, pb, x, q, k, shape, np.zeros(3))
        O.threads(4)
        b = O.snsd_pairs(pa, pb, x, q, k, shape, np.zeros(3))
    finally:
        O.threads(was)
    assert np.array_equal(a, b)
