"""GPU: tori (the rings of Sec. 6) through the C ABI against the oracle.

* SNSD of random torus pairs, of linked or nearly linked pairs (competing
  local minima) and of special configurations: Phi (the
  centre-circle distance minus the minor radii) to 1e-11; where the closest
  pair is unique (the oracle's next local minimum is 1e-6 worse), the normal
  and both contact points to 1e-9;
* a chainmail of interlaced rings pulled by the extensile field, step by
  step against the oracle's step from the GPU's own state: the same contact
  sets per recursion, velocities to 1e-8 of their scale, positions and
  orientations to 1e-10;
* a context holding an ellipsoid packing and a chainmail (the narrowphase
  kernel for every kind), each packing against its own oracle step;
* the contrast of Sec. 6 on a small chainmail at drag 0.1, dt 1e-3: ReLCP
  within the overlap tolerance, LCP-SNSD beyond it;
* shape checks: tori are refused in a monolayer, under inertial dynamics and
  with a negative major radius.
"""
import numpy as np
import pytest

import oracle as O
from paper_2506_14097_amd import inputs as I
from paper_2506_14097_amd import relcp as R

from states import compressed_packing

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def soa(a, dev, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(np.asarray(a).T), dtype=dtype, device=dev).contiguous()


def tens(a, dev, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device=dev)


def gpu_snsd(dev, x, q, kind, shape, pa, pb):
    return R.snsd_device(soa(x, dev), soa(q, dev), tens(kind, dev, torch.int32), soa(shape, dev),
                         tens(pa, dev, torch.int32), tens(pb, dev, torch.int32), np.zeros(3)).cpu().numpy().T


def oracle_with_margin(x, q, shape, pa, pb):
    """Oracle SNSD per pair and the margin of uniqueness of its minimum."""
    out, unique = [], []
    for a, b in zip(pa, pb):
        ea, eb = O.quat_to_R(q[a])[:, 2], O.quat_to_R(q[b])[:, 2]
        phi, n, ra, rb, second = O.snsd_torus(x[b] - x[a], ea, shape[a, 0], shape[a, 1], eb, shape[b, 0],
                                               shape[b, 1])
        out.append(np.concatenate([[phi], n, ra, rb]))
        unique.append(second - (phi + shape[a, 1] + shape[b, 1]) > 1e-6)
    return np.array(out), np.array(unique)


@pytest.mark.parametrize("seed", [0, 1])
def test_snsd_tori_random_pairs(dev, seed):
    rng = np.random.default_rng(seed)
    nb = 300
    x = rng.uniform(0, 7.0, (nb, 3))
    q = I.shoemake_quaternions(rng, nb)
    shape = np.stack([rng.uniform(0.6, 1.2, nb), rng.uniform(0.05, 0.15, nb), np.zeros(nb)], 1)
    kind = np.full(nb, I.TORUS, np.int32)
    pa, pb = O.broadphase(x, kind, shape, np.zeros(3), 0.3)
    print("torus SNSD seed", seed, "pairs", pa.size, flush=True)
    out = gpu_snsd(dev, x, q, kind, shape, pa, pb)
    ref, unique = oracle_with_margin(x, q, shape, pa, pb)
    # the bodies of the table agree with the oracle's own pair routine
    np.testing.assert_array_equal(ref, O.snsd_pairs(pa, pb, x, q, kind, shape, np.zeros(3)))
    assert pa.size > 300 and unique.sum() > 0.9 * pa.size
    assert np.abs(out[:, 0] - ref[:, 0]).max() < 1e-11
    assert np.abs(out[unique, 1:] - ref[unique, 1:]).max() < 1e-9
    # every result is a valid contact: (x_b + r_b) - (x_a + r_a) = Phi n
    d = x[pb] - x[pa]
    np.testing.assert_allclose(d + out[:, 7:10] - out[:, 4:7], out[:, :1] * out[:, 1:4], atol=1e-11)


def test_snsd_tori_special_cases(dev):
    e = I.RING_FLAT
    cases = [  # (x_b, q_a, q_b, R_a, r_a, R_b, r_b, closed-form Phi or None)
        ((3.0, 0, 0), e, e, 1.0, 0.1, 0.8, 0.05, 3.0 - 1.95),            # coplanar
        ((0, 0, 0.5), e, e, 1.0, 0.1, 0.7, 0.1, np.hypot(0.5, 0.3) - 0.2),  # coaxial (continuum)
        ((1.0, 0, 0), e, I.RING_AXIS_Y, 1.0, 0.1, 1.0, 0.1, 0.8),          # through each other's centre
        ((1.8, 0, 0), e, I.RING_AXIS_Y, 1.0, 0.1, 1.0, 0.1, 0.0),          # taut link
        ((0.3, -0.4, 1.2), e, e, 0.0, 0.2, 0.0, 0.3, 1.3 - 0.5),           # R = 0: spheres
        ((0.6, 0.2, 0.1), e, I.RING_AXIS_X, 1.0, 0.1, 0.9, 0.1, None),
    ]
    x = np.zeros((2 * len(cases), 3))
    q = np.zeros((2 * len(cases), 4))
    shape = np.zeros((2 * len(cases), 3))
    for k, (xb, qa, qb, Ra, ra, Rb, rb, _) in enumerate(cases):
        x[2 * k + 1] = xb
        q[2 * k], q[2 * k + 1] = qa, qb
        shape[2 * k, :2], shape[2 * k + 1, :2] = (Ra, ra), (Rb, rb)
    kind = np.full(len(x), I.TORUS, np.int32)
    pa, pb = np.arange(0, len(x), 2, dtype=np.int32), np.arange(1, len(x), 2, dtype=np.int32)
    out = gpu_snsd(dev, x, q, kind, shape, pa, pb)
    ref, unique = oracle_with_margin(x, q, shape, pa, pb)
    for k, c in enumerate(cases):
        if c[-1] is not None:
            assert abs(out[k, 0] - c[-1]) < 1e-12, k
        assert abs(out[k, 0] - ref[k, 0]) < 1e-12, k
        if unique[k]:
            assert np.abs(out[k, 1:] - ref[k, 1:]).max() < 1e-9, k
    np.testing.assert_allclose(out[3, 1:4], [-1, 0, 0], atol=1e-12)  # the taut link pulls along -x


def test_chainmail_steps_follow_oracle(dev):
    S = I.chainmail(3, 3, slack=0.02)
    kw = dict(dt=0.01, eps=1e-5, skin=0.2)
    sim = R.Simulation(S["x"], S["q"], S["kind"], S["shape"], S["rho_xi"], S["box"], precision=64, skin=kw["skin"])
    compared = contacts = recs = 0
    for k in range(60):
        x, q, _ = sim.get_state()
        f = I.extensile_field(x)
        sim.set_external(f)
        ref = O.relcp_step(x, q, S["kind"], S["shape"], S["rho_xi"], S["box"], dt=kw["dt"], eps=kw["eps"],
                           tol=1e-12, skin=kw["skin"], fext=f)
        res = sim.step(kw["dt"], kw["eps"], 1e-12)
        assert res["status"] == 0 and ref["status"] == 0, k
        xg, qg, Ug = sim.get_state()
        if np.any(ref["margin"] < 1e-9):
            continue
        assert res["recursions"] == ref["recursions"], k
        assert list(res["n_contacts"]) == list(ref["n_contacts"]), k
        assert np.abs(Ug - ref["U"]).max() < 1e-8 * max(1.0, np.abs(ref["U"]).max()), k
        assert np.abs(xg - ref["x"]).max() < 1e-10, k
        assert np.abs(qg - ref["q"]).max() < 1e-10, k
        assert res["max_overlap"] <= kw["eps"]
        compared += 1
        contacts += res["n_contacts_final"] > 0
        recs += res["recursions"]
    print("chainmail steps compared", compared, "with contacts", contacts, "recursions", recs, flush=True)
    sim.close()
    assert compared > 50 and contacts > 30


def test_torus_shape_checks(dev):
    S = I.chainmail(2, 2)
    args = (S["x"], S["q"], S["kind"], S["shape"], S["rho_xi"], S["box"])
    for kw in (dict(planar=True), dict(dynamics=R.INERTIAL)):
        with pytest.raises(R.RelcpError):
            R.Simulation(*args, **kw)
    bad = S["shape"].copy()
    bad[0, 0] = -1.0
    with pytest.raises(R.RelcpError):
        R.Simulation(S["x"], S["q"], S["kind"], bad, S["rho_xi"], S["box"])


def test_chainmail_relcp_against_snsd(dev):
    """The contrast of Sec. 6 through the library: ReLCP within the overlap
    tolerance with recursions, LCP-SNSD beyond it (the oracle shows the same
    on this input)."""
    out = {}
    for mr in (64, 0):
        S = I.chainmail(3, 3, slack=0.05, xi=0.1, jitter=0.05)
        sim = R.Simulation(S["x"], S["q"], S["kind"], S["shape"], S["rho_xi"], S["box"], precision=64, skin=0.1,
                           max_recursions=mr)
        worst = nrec = 0
        for _ in range(50):
            x, _, _ = sim.get_state()
            sim.set_external(I.extensile_field(x))
            res = sim.step(1e-3, 1e-5, 1e-9)
            worst = max(worst, res["max_overlap"])
            nrec += res["recursions"] > 0
        sim.close()
        out[mr] = (worst, nrec)
    print("chainmail ReLCP", out[64], "LCP-SNSD", out[0], flush=True)
    assert out[64][0] <= 1e-5 and out[64][1] >= 10
    assert out[0][0] > 2e-5 and out[0][1] == 0


def test_snsd_tori_linked_pairs(dev):
    """Pairs whose second ring is centred near the first ring's centre circle
    (linked or nearly so, random axes): several local minima compete, so the
    sampled search must still find the global one."""
    rng = np.random.default_rng(7)
    m = 2000
    qa, qb = I.shoemake_quaternions(rng, m), I.shoemake_quaternions(rng, m)
    Ra, Rb = rng.uniform(0.6, 1.2, m), rng.uniform(0.6, 1.2, m)
    t = rng.uniform(0, 2 * np.pi, m)
    x = np.zeros((2 * m, 3))
    q = np.zeros((2 * m, 4))
    shape = np.zeros((2 * m, 3))
    for k in range(m):
        Ma = O.quat_to_R(qa[k])
        c = Ra[k] * (np.cos(t[k]) * Ma[:, 0] + np.sin(t[k]) * Ma[:, 1])
        x[2 * k] = (10.0 * k, 0, 0)
        x[2 * k + 1] = x[2 * k] + c + rng.normal(0, 0.25, 3)
        q[2 * k], q[2 * k + 1] = qa[k], qb[k]
        shape[2 * k, :2], shape[2 * k + 1, :2] = (Ra[k], 0.1), (Rb[k], 0.08)
    kind = np.full(2 * m, I.TORUS, np.int32)
    pa, pb = np.arange(0, 2 * m, 2, dtype=np.int32), np.arange(1, 2 * m, 2, dtype=np.int32)
    out = gpu_snsd(dev, x, q, kind, shape, pa, pb)
    ref, unique = oracle_with_margin(x, q, shape, pa, pb)
    err = np.abs(out[:, 0] - ref[:, 0])
    print("linked pairs: max |dPhi| %.3g, unique %d of %d" % (err.max(), unique.sum(), m), flush=True)
    assert err.max() < 1e-11
    assert np.abs(out[unique, 1:] - ref[unique, 1:]).max() < 1e-9


def test_mixed_batch_of_ellipsoids_and_rings(dev):
    """One context holding a periodic ellipsoid packing and an open chainmail
    (one kind per packing): the narrowphase kernel for every kind then
    handles the rings.  Each packing's step against the oracle's step of
    that packing alone, from the GPU's own state, over 20 steps."""
    P = compressed_packing(3, 120, 24)
    Cm = I.chainmail(3, 3, slack=0.02)
    parts = [dict(P, x=P["x"] * 0.99, box=P["box"] * 0.99), Cm]
    off = np.cumsum([0] + [len(p["x"]) for p in parts]).astype(np.int32)
    cat = lambda k: np.concatenate([p[k] for p in parts])
    sim = R.Simulation(cat("x"), cat("q"), cat("kind"), cat("shape"), cat("rho_xi"), np.stack([p["box"] for p in parts]),
                       batch_off=off, precision=64, skin=0.2, warm_start=R.WS_COLD)
    ring = slice(off[1], off[2])
    compared = 0
    for k in range(20):
        x, q, _ = sim.get_state()
        f = np.zeros((len(x), 6))
        f[ring] = I.extensile_field(x[ring])
        sim.set_external(f)
        refs = []
        for j, p in enumerate(parts):
            sl = slice(off[j], off[j + 1])
            refs.append(O.relcp_step(x[sl], q[sl], p["kind"], p["shape"], p["rho_xi"], p["box"], dt=0.01, eps=1e-5,
                                     tol=1e-12, skin=0.2, fext=f[sl], lcp_mode=1, prev=None))
        res = sim.step(0.01, 1e-5, 1e-12)
        assert res["status"] == 0 and all(r["status"] == 0 for r in refs), k
        xg, qg, Ug = sim.get_state()
        if any(np.any(r["margin"] < 1e-9) for r in refs):
            continue
        for j, r in enumerate(refs):
            sl = slice(off[j], off[j + 1])
            assert np.abs(Ug[sl] - r["U"]).max() < 1e-8 * max(1.0, np.abs(r["U"]).max()), (k, j)
            assert np.abs(xg[sl] - r["x"]).max() < 1e-10, (k, j)
            assert np.abs(qg[sl] - r["q"]).max() < 1e-10, (k, j)
        compared += 1
    print("mixed batch: steps compared", compared, flush=True)
    sim.close()
    assert compared > 15
