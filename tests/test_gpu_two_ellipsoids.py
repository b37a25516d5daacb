"""GPU: the two-ellipsoid sliding collision of Sec. 5.1, step by step
through the contact against the oracle's step from the GPU's own state, for
ReLCP and for LCP-SNSD (the same step with no recursions), at dt = 0.1,
where ReLCP appends constraints: the same recursions and constraint counts,
velocities to 1e-8 of their scale, positions to 1e-10."""
import numpy as np
import pytest

import oracle as O
from paper_2506_14097_amd import inputs as I
from paper_2506_14097_amd import relcp as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("max_rec", [64, 0], ids=["relcp", "snsd-lcp"])
def test_glancing_pair_follows_the_oracle(dev, max_rec):
    S = I.glancing_ellipsoids()
    sim = R.Simulation(S["x"], S["q"], S["kind"], S["shape"], S["rho_xi"], S["box"], precision=64, skin=0.5,
                       max_recursions=max_rec)
    sim.set_external(S["fext"])
    recs = contacts = 0
    for k in range(400):  # t = 98 to 138: contact from about 99 to 137
        x, q, _ = sim.get_state()
        ref = O.relcp_step(x, q, S["kind"], S["shape"], S["rho_xi"], S["box"], dt=0.1, eps=1e-5, tol=1e-12,
                           skin=0.5, fext=S["fext"], max_recursions=max_rec)
        res = sim.step(0.1, 1e-5, 1e-12)
        assert res["status"] == 0 and ref["status"] == 0
        xg, qg, Ug = sim.get_state()
        if np.any(ref["margin"] < 1e-9):
            continue  # the oracle saw a pair within 1e-9 of the overlap threshold
        assert res["recursions"] == ref["recursions"], k
        assert list(res["n_contacts"]) == list(ref["n_contacts"]), k
        assert np.abs(Ug - ref["U"]).max() < 1e-8 * max(1.0, np.abs(ref["U"]).max()), k
        assert np.abs(xg - ref["x"]).max() < 1e-10, k
        assert np.abs(qg - ref["q"]).max() < 1e-10, k
        recs += res["recursions"]
        contacts += res["n_contacts_final"] > 0
    sim.close()
    assert contacts > 300
    if max_rec:
        assert recs > 0
