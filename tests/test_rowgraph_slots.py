"""Bounds of the row graph's entry slots under an overflow, on the CPU.

The row graph stores the off-diagonal entries of A over rows in sliced ELL
with a fixed stride S: slice s holds rows [64 s, 64 s + 64), and entry k of
row r sits in slot 64 (s S + k) + r % 64, for k below the row's count (the
other rows at its two bodies); no slot past a row's count is written by the
fill or read by a pass.  The allocation holds 64 S slots per slice.  A row
whose count exceeds S does not fit: the fill (k_rowgraph_fill_entries)
writes none of its entries, raises the device's overflow count to the row's
count and flags the overflow; the passes (row_preload_b) read no entry of
it.  The step then raises S to at least half again that count and restarts.
This test restates that slot arithmetic and walks every slot the fill would
write and every slot a pass would read, on the rows of A_0 of real oracle
steps, with the first stride forced down to one slot per row
(RELCP_RG_SLOTS_PER_ROW = 1): all stay inside their own row's slots and the
allocation, the overflow is flagged exactly when a row does not fit, and
with the raised stride every row fits."""
import numpy as np
import pytest

import oracle as O

from states import compressed_packing

W = 64


def counts(ia, ib, nb):
    deg = np.bincount(np.concatenate([ia, ib]), minlength=nb)
    return deg[ia] + deg[ib] - 2


def walk(ia, ib, nb, S):
    """Slots touched by the fill and by a pass at stride S; returns (max slot
    + 1 written, max slot + 1 read, allocation, overflow flag, overflow count)."""
    wrow = counts(ia, ib, nb)
    ns = (len(ia) + W - 1) // W
    cap = W * ns * S
    hi_w = hi_r = 0
    overflow, need = False, 0
    owner = {}
    for r in range(len(ia)):
        s, lane = r // W, r % W
        if wrow[r] > S:  # the fill leaves this row and flags it; passes read no entry of it
            overflow, need = True, max(need, int(wrow[r]))
            continue
        for k in range(wrow[r]):
            at = W * (s * S + k) + lane
            assert owner.setdefault(at, r) == r  # no two rows share a slot
            hi_w = max(hi_w, at + 1)
            hi_r = max(hi_r, at + 1)
    return hi_w, hi_r, cap, overflow, need


@pytest.mark.parametrize("seed", [0, 3])
def test_slots_stay_inside_the_allocation_when_the_stride_is_low(seed):
    S = compressed_packing(seed, 150, 26)
    r = O.relcp_step(S["x"] * 0.99, S["q"], S["kind"], S["shape"], S["rho_xi"], S["box"] * 0.99, dt=5e-3, eps=1e-5,
                     tol=1e-9, skin=0.2, lcp_mode=1)
    ia, ib = r["ia"][r["rec"] == 0], r["ib"][r["rec"] == 0]
    nb = len(S["x"])
    stride = 1
    hi_w, hi_r, cap, overflow, need = walk(ia, ib, nb, stride)
    print("rows", len(ia), "largest count", counts(ia, ib, nb).max(), "allocated", cap, "overflow", overflow)
    assert hi_w <= cap and hi_r <= cap
    assert overflow == (counts(ia, ib, nb).max() > stride) and overflow
    assert need == counts(ia, ib, nb).max()
    # the re-size: half again the largest count of a row that did not fit
    stride = max(stride + 1, need + need // 2)
    hi_w, hi_r, cap, overflow, _ = walk(ia, ib, nb, stride)
    assert not overflow and hi_w <= cap
