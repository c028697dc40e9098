"""Host check of the compile-time row ranges of the folded zero-padded FFT pass at N_z = 512.

A padded axis (Sec. 3.3) embeds N data points at offset s = (N_z - N)/2 of an N_z-point transform,
N_z = 2 L2^2 (L2 = 16, L1 = 32). Thread t of a line holds the first-stage inputs at data indices
m0 + L2 r (r < L1/2) with m0 = L2 ceil((s - t)/L2) + t - s, and writes the outputs k1 = 2t + p,
k2 of phase p at data index 2t + p - s + L1 k2. For a band 4 L2 KW <= N < 4 L2 (KW + 1) the kernel
treats input rows r < 4 KW and outputs k2 = L2/2 + d, d in [-KW, KW), as in the data on every lane,
and input rows r >= 4 KW + 4 and outputs with d < -KW - 1 or d > KW as in the data on no lane. This
test enumerates every even N of the instantiated bands and every lane and checks both claims.
"""
from __future__ import annotations

L2, L1, NZ = 16, 32, 512
H = L1 // 2


def _lanes(n):
    s = (NZ - n) // 2
    for t in range(L2):
        a0 = (s - t + L2 - 1) // L2
        m0 = L2 * a0 + t - s
        assert 0 <= m0 < L2
        yield t, s, m0


def test_band_rows_and_outputs():
    checked = 0
    for n in range(2, NZ // 2 + 1, 2):
        kw = n // (4 * L2)
        if kw not in (1, 2, 3, 4):
            continue
        ra, rz = 4 * kw, 4 * kw + 4
        for t, s, m0 in _lanes(n):
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
    assert checked == 97 * L2 * 2 * L2  # N = 64, 66, ..., 256


def test_every_data_point_is_read_and_written_once():
    """Over the lanes and rows of one line, the inputs cover [0, N) once and the outputs cover [0, N) once."""
    for n in (64, 100, 126, 128, 136, 190, 192, 200, 254, 256):
        reads, writes = [], []
        for t, s, m0 in _lanes(n):
            reads += [m0 + L2 * r for r in range(H) if m0 + L2 * r < n]
            writes += [2 * t + p - s + L1 * k2 for p in range(2) for k2 in range(L2)
                       if 0 <= 2 * t + p - s + L1 * k2 < n]
        assert sorted(reads) == list(range(n))
        assert sorted(writes) == list(range(n))
