"""Host-side model of the dense condensation's LDS ring (the index arithmetic
of prep_band_body, restated step by step): positions stream through a ring
of R = min(nf, CH + band_w) slots in chunks of CH rows; the global loads of
the positions chunk c + 1 brings in are issued before chunk c's products and
stored after them.  The model replays every read and write of a workgroup
for many sizes and checks that each read finds the position it asks for
(no slot is overwritten while a later row still needs it), that every slot
index stays below R, and that the wrap's argument stays below 2R (its one
conditional subtraction).  No GPU: this checks the indexing scheme the
kernel uses, for the chunk sizes it is built with (128, 256, 512)."""
import numpy as np
import pytest


def _wrap(t, R):
    assert 0 <= t < 2 * R, (t, R)
    return t if t < R else t - R


def _replay(nf, bw, CH, upper):
    """upper[p]: the band positions k >= p row p reads (p itself first)."""
    R = min(nf, CH + bw)
    ring = [None] * R
    for pos in range(R):                        # first fill: slot = position
        ring[pos] = pos
    lo, lo_slot, p0_slot = R, 0, 0
    for p0 in range(0, nf, CH):
        nhi = min(nf, p0 + 2 * CH + bw)
        pre = [lo + tid for tid in range(CH) if lo + tid < nhi]
        cshift = p0_slot - p0
        for p in range(p0, min(p0 + CH, nf)):
            for k in upper[p]:
                assert p <= k <= min(nf - 1, p + bw)
                s = _wrap(k + cshift, R)
                assert ring[s] == k, (nf, bw, CH, p0, p, k, s, ring[s])
        for tid, pos in enumerate(pre):         # after the chunk's reads
            ring[_wrap(lo_slot + tid, R)] = pos
        if nhi > lo:
            lo_slot = _wrap(lo_slot + (nhi - lo), R)
            lo = nhi
        if p0 + CH < nf:                        # the next chunk's start
            p0_slot = _wrap(p0_slot + CH, R)
    return R


def _band(nf, bw, rng, density=0.3):
    """Upper neighbours of each position within the band width, the
    diagonal first and the far edge of the band present somewhere."""
    upper = []
    for p in range(nf):
        ks = [p] + [k for k in range(p + 1, min(nf, p + bw + 1)) if rng.random() < density]
        upper.append(ks)
    if nf > bw:
        upper[0] = sorted(set(upper[0]) | {bw})
    return upper


@pytest.mark.parametrize("CH", [128, 256, 512])
def test_ring_reads_find_their_positions(CH):
    rng = np.random.default_rng(CH)
    cases = [(1, 0), (5, 3), (CH - 1, 40), (CH, 121), (CH + 1, 121), (3 * CH + 17, 121),
             (2 * CH, CH + 50), (1960, 121), (1960, 482), (4 * CH + 3, 1)]
    for nf, bw in cases:
        bw = min(bw, max(nf - 1, 0))
        R = _replay(nf, bw, CH, _band(nf, bw, rng))
        assert R == min(nf, CH + bw)


def test_ring_structured_grid_band():
    """A bar's band rows: each position reads the grid neighbours ahead of
    it within one cross-section and the next (the widest band the exact
    basis layout produces is one cross-section plus a little)."""
    nx, ny, nz = 23, 7, 7
    nf = nx * ny * nz
    section = ny * nz
    upper = []
    for p in range(nf):
        ks = {p}
        for d in (1, ny, ny + 1, section, section + 1, section + ny, section + ny + 1):
            if p + d < nf:
                ks.add(p + d)
        upper.append(sorted(ks))
    bw = max(max(u) - p for p, u in enumerate(upper))
    for CH in (128, 256, 512):
        _replay(nf, bw, CH, upper)
