"""Host checks of index maps: the compile-time row ranges of the folded zero-padded FFT pass at N_z = 512
and 128, the workgroup order of the one-pass sums, and the XCD order of the padded passes' tiles.

A padded axis (Sec. 3.3) embeds N data points at offset s = (N_z - N)/2 of an N_z-point transform,
N_z = 2 L2^2 (L2 = 16 or 8, L1 = 2 L2). Thread t of a line holds the first-stage inputs at data indices
m0 + L2 r (r < L1/2) with m0 = L2 ceil((s - t)/L2) + t - s, and writes the outputs k1 = 2t + p,
k2 of phase p at data index 2t + p - s + L1 k2. For a band 4 L2 KW <= N < 4 L2 (KW + 1) the kernel
treats input rows r < 4 KW and outputs k2 = L2/2 + d, d in [-KW, KW), as in the data on every lane,
and input rows r >= 4 KW + 4 and outputs with d < -KW - 1 or d > KW as in the data on no lane. This
test enumerates every even N of the instantiated bands and every lane and checks both claims.
"""
from __future__ import annotations

import pytest

# (L2, instantiated bands KW)
SPLITS = [(16, (1, 2, 3, 4)), (8, (1, 2))]


def _lanes(n, L2):
    NZ = 2 * L2 * L2
    s = (NZ - n) // 2
    for t in range(L2):
        a0 = (s - t + L2 - 1) // L2
        m0 = L2 * a0 + t - s
        assert 0 <= m0 < L2
        yield t, s, m0


@pytest.mark.parametrize("L2,bands", SPLITS)
def test_band_rows_and_outputs(L2, bands):
    L1, NZ = 2 * L2, 2 * L2 * L2
    H = L1 // 2
    checked = 0
    for n in range(2, NZ // 2 + 1, 2):
        kw = n // (4 * L2)
        if kw not in bands:
            continue
        ra, rz = 4 * kw, 4 * kw + 4
        assert ra <= H
        for t, s, m0 in _lanes(n, L2):
            for r in range(H):
                inside = m0 + L2 * r < n
                if r < ra:
                    assert inside, (n, t, r)
                if r >= rz:
                    assert not inside, (n, t, r)
            for p in range(2):
                for k2 in range(L2):
                    m = 2 * t + p - s + L1 * k2
                    d = k2 - L2 // 2
                    inside = 0 <= m < n
                    if -kw <= d < kw:
                        assert inside, (n, t, p, k2)
                    if not (-kw - 1 <= d <= kw):
                        assert not inside, (n, t, p, k2)
                    checked += 1
    assert checked == (NZ // 2 - 4 * L2) // 2 * L2 * 2 * L2 + L2 * 2 * L2  # every even N from 4 L2 to N_z / 2


@pytest.mark.parametrize("L2,sizes", [(16, (64, 100, 126, 128, 136, 190, 192, 200, 254, 256)),
                                      (8, (32, 48, 60, 62, 64))])
def test_every_data_point_is_read_and_written_once(L2, sizes):
    """Over the lanes and rows of one line, the inputs cover [0, N) once and the outputs cover [0, N) once."""
    L1 = 2 * L2
    H = L1 // 2
    for n in sizes:
        reads, writes = [], []
        for t, s, m0 in _lanes(n, L2):
            reads += [m0 + L2 * r for r in range(H) if m0 + L2 * r < n]
            writes += [2 * t + p - s + L1 * k2 for p in range(2) for k2 in range(L2)
                       if 0 <= 2 * t + p - s + L1 * k2 < n]
        assert sorted(reads) == list(range(n))
        assert sorted(writes) == list(range(n))


@pytest.mark.parametrize("gx", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("gy", [8, 16, 64, 256])
def test_one_pass_block_order(gx, gy):
    """The one-pass sums of a group of one entry remap the linear workgroup index l (dealt to XCD l mod 8)
    to (column tile, slab range) = ((l / 8) mod gx, l mod 8 + 8 (l / (8 gx))): a bijection onto the grid in
    which every column tile of a slab range has the same l mod 8."""
    seen = set()
    for l in range(gx * gy):
        x, y = (l // 8) % gx, l % 8 + 8 * (l // (8 * gx))
        assert 0 <= x < gx and 0 <= y < gy
        assert y % 8 == l % 8
        seen.add((x, y))
    assert len(seen) == gx * gy


def _xcd_tiles(G, b, tiles):
    """The padded passes' tile range of workgroup b in a grid of G: (first, end, step)."""
    x, r = b % 8, G % 8
    below = (G // 8) * x + min(r, x)
    upto = (G // 8) * (x + 1) + min(r, x + 1)
    return tiles * below // G + b // 8, tiles * upto // G, upto - below


@pytest.mark.parametrize("G", [1, 3, 7, 8, 9, 13, 64, 100, 777, 4096])
def test_xcd_tile_order_is_a_partition(G):
    """Every tile is taken by exactly one workgroup (grid G = min(tiles, 4096) as launched, and larger
    tile counts), each XCD's share is contiguous, and the shares differ by at most one tile per workgroup."""
    for tiles in sorted({G, G + 1, 2 * G + 5, 8 * G + 3, 10 * G, 12345}):
        if tiles < G:
            continue
        seen = [0] * tiles
        shares = {}
        for b in range(G):
            first, end, step = _xcd_tiles(G, b, tiles)
            assert step >= 1
            for t in range(first, end, step):
                seen[t] += 1
                shares.setdefault(b % 8, []).append(t)
        assert all(c == 1 for c in seen), (G, tiles)
        for x, ts in shares.items():
            assert sorted(ts) == list(range(min(ts), max(ts) + 1)), (G, tiles, x)
        per_wg = [len(range(*_xcd_tiles(G, b, tiles))) for b in range(G)]
        assert max(per_wg) - min(per_wg) <= 2, (G, tiles)
