"""Bounds of the row graph's entry slots under an overflow, on the CPU.

The row graph stores the off-diagonal entries of A over rows in sliced ELL:
slice s holds rows [64 s, 64 s + 64), its width w_s is the largest count of
other rows at a row's two bodies in the slice, and entry k of row r sits in
slot 64 (base_s + k) + r % 64 (base = exclusive scan of the widths); the
slots past a row's own entries (up to the slice's width) are neither
written by the fill nor read by a pass, which takes each row's count.  The
step sizes the slots from an estimate per row (RELCP_RG_SLOTS_PER_ROW, with
half again as much headroom) before the widths are known; the fill
(k_rowgraph_fill_entries) skips a slice whose end 64 (base_s + w_s) passes the
allocation and flags the overflow, and the passes (row_preload_b) treat such
a slice as empty.  This test restates that slot arithmetic and walks every
slot the fill would write and every slot a pass would read, on the rows of
A_0 of real oracle steps, with the estimate forced down to one slot per row:
all stay below the allocation, the overflow is flagged exactly when a slice
does not fit, and with the re-sized allocation (twice the slots needed)
every slice fits."""
import numpy as np
import pytest

import oracle as O

from states import compressed_packing

W = 64


def slices(ia, ib, nb):
    m = len(ia)
    deg = np.bincount(np.concatenate([ia, ib]), minlength=nb)
    wrow = deg[ia] + deg[ib] - 2
    ns = (m + W - 1) // W
    width = np.array([wrow[s * W:(s + 1) * W].max() for s in range(ns)], np.int64)
    base = np.concatenate([[0], np.cumsum(width)])
    return deg, wrow, width, base


def walk(ia, ib, nb, cap):
    """Slots touched by the fill and by a pass; returns (max slot + 1 written,
    max slot + 1 read, overflow flag)."""
    deg, wrow, width, base = slices(ia, ib, nb)
    hi_w = hi_r = 0
    overflow = False
    for r in range(len(ia)):
        s, lane = r // W, r % W
        b0, w = base[s], width[s]
        if W * (b0 + w) > cap:  # the fill leaves this slice and flags it; passes read no entry
            overflow = True
            continue
        assert wrow[r] <= w
        for k in range(wrow[r]):  # the row's entries (the slots past them are neither written nor read)
            at = W * (b0 + k) + lane
            hi_w = max(hi_w, at + 1)
            hi_r = max(hi_r, at + 1)
    return hi_w, hi_r, overflow, base[-1]


@pytest.mark.parametrize("seed", [0, 3])
def test_slots_stay_inside_the_allocation_when_the_estimate_is_low(seed):
    S = compressed_packing(seed, 150, 26)
    r = O.relcp_step(S["x"] * 0.99, S["q"], S["kind"], S["shape"], S["rho_xi"], S["box"] * 0.99, dt=5e-3, eps=1e-5,
                     tol=1e-9, skin=0.2, lcp_mode=1)
    ia, ib = r["ia"][r["rec"] == 0], r["ib"][r["rec"] == 0]
    nb = len(S["x"])
    ns = (len(ia) + W - 1) // W
    est = W * ns * 1
    cap = est + est // 2  # the buffers' headroom
    hi_w, hi_r, overflow, need = walk(ia, ib, nb, cap)
    print("rows", len(ia), "slots needed", W * need, "allocated", cap, "overflow", overflow)
    assert hi_w <= cap and hi_r <= cap
    assert overflow == (W * need > cap) and overflow
    # the re-size: twice the slots the fill reported
    cap2 = 2 * W * need
    hi_w, hi_r, overflow, _ = walk(ia, ib, nb, cap2)
    assert not overflow and hi_w <= W * need <= cap2
