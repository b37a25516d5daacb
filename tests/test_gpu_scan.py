"""GPU: the prefix sum and the flag compaction the step is built on (pair
selection of A_0 and of each augmentation, incidence offsets, cell lists,
row-graph slice bases), through the C ABI, against numpy.  Integer work:
bit-exact.  Sizes cover each path: empty, one block (up to 8192 items), two
passes with offsets summed per block (up to 4096 tiles of 2048), and past
that with the tile totals scanned first; compaction with the group offsets
summed per block (up to 4096 groups of 256) and scanned first."""
import numpy as np
import pytest

from paper_2506_14097_amd import relcp as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


SCAN_SIZES = [0, 1, 2, 255, 2047, 2048, 2049, 8191, 8192, 8193, 300_001, 2048 * 4096, 2048 * 4096 + 1, 9_000_003]


@pytest.mark.parametrize("n", SCAN_SIZES)
def test_exclusive_scan_matches_cumsum(dev, n):
    rng = np.random.Generator(np.random.PCG64(n + 7))
    x = rng.integers(0, 9, n).astype(np.int32)
    print("scan n", n, flush=True)
    out, tot = R.exclusive_scan_device(torch.tensor(x, device=dev))
    ref = np.concatenate([[0], np.cumsum(x, dtype=np.int64)[:-1]]) if n else np.zeros(0, np.int64)
    assert tot == int(x.sum(dtype=np.int64))
    assert np.array_equal(out.cpu().numpy().astype(np.int64), ref)


def test_exclusive_scan_in_place(dev):
    rng = np.random.Generator(np.random.PCG64(3))
    x = rng.integers(0, 5, 100_000).astype(np.int32)
    t = torch.tensor(x, device=dev)
    out, tot = R.exclusive_scan_device(t, out=t)
    assert out.data_ptr() == t.data_ptr()
    assert tot == int(x.sum())
    assert np.array_equal(t.cpu().numpy(), np.concatenate([[0], np.cumsum(x)[:-1]]).astype(np.int32))


COMPACT_SIZES = [0, 1, 255, 256, 257, 2048, 2049, 300_000, 1_048_576, 1_048_577, 3_000_001]


@pytest.mark.parametrize("n", COMPACT_SIZES)
@pytest.mark.parametrize("density", [0.0, 0.03, 0.5, 1.0])
def test_compact_flags_matches_nonzero(dev, n, density):
    rng = np.random.Generator(np.random.PCG64(n * 4 + int(density * 100)))
    f = (rng.random(n) < density).astype(np.int32) * rng.integers(1, 4, n).astype(np.int32)
    print("compact n", n, "density", density, flush=True)
    idx = R.compact_flags_device(torch.tensor(f, device=dev))
    assert np.array_equal(idx.cpu().numpy(), np.nonzero(f)[0].astype(np.int32))


def test_scan_and_compact_reject_bad_arguments(dev):
    x = torch.zeros(4, dtype=torch.int32, device=dev)
    assert R.lib().relcp_exclusive_scan_device(R._tptr(x), R._tptr(x), -1, None, None) == R.E_INVALID
    assert R.lib().relcp_compact_flags_device(R._tptr(x), 4, R._tptr(x), None, None) == R.E_INVALID
    assert R.lib().relcp_compact_flags_device(None, 4, None, None, None) == R.E_INVALID
