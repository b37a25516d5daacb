"""The prefix-sum entry point that allocates nothing (for callers that
cannot allocate device memory), through the C ABI, against the allocating
entry point and numpy: two calls in a row, the second smaller (the shared
scratch keeps the first call's tile totals), an empty call, and a size
above the maximum refused before anything runs."""
import numpy as np
import pytest

from paper_2506_14097_amd import relcp as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_noalloc_scan_matches_the_allocating_scan():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(0)
    for n in (5_000_000, 2_100_000, 3000):
        h = rng.integers(0, 50, n, dtype=np.int32)
        x = torch.tensor(h, device=dev)
        ref, tot_ref = R.exclusive_scan_device(x)
        out = torch.full_like(x, -7)
        tot = torch.full((1,), -7, dtype=torch.int32, device=dev)
        print("noalloc scan n", n, flush=True)
        assert R.exclusive_scan_device_noalloc(x, out, tot) == R.OK
        torch.cuda.synchronize()
        assert torch.equal(out, ref) and int(tot.item()) == tot_ref
        expect = np.concatenate([[0], np.cumsum(h, dtype=np.int64)[:-1]])
        assert np.array_equal(out.cpu().numpy(), expect) and tot_ref == int(h.sum())
    e = torch.zeros(0, dtype=torch.int32, device=dev)
    tot = torch.full((1,), -7, dtype=torch.int32, device=dev)
    assert R.exclusive_scan_device_noalloc(e, e, tot) == R.OK
    torch.cuda.synchronize()
    assert int(tot.item()) == 0
    # above the maximum: refused by the host check, nothing launched
    small = torch.zeros(4, dtype=torch.int32, device=dev)
    rc = R.lib().relcp_exclusive_scan_device_noalloc(R._tptr(small), R._tptr(small), R.NOALLOC_SCAN_MAX + 1,
                                                       R._tptr(tot), None)
    assert rc == R.E_CAPACITY
