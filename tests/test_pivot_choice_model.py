"""CPU model of how the factorization kernels choose a pivot row across the
waves of a workgroup (partial pivoting: the largest |Re| + |Im| in the
column among the rows not yet used, lowest row on ties).

Every wave reduces the 32-bit keys of its rows (the magnitude's float bits
with the low mantissa bits dropped, then the complement of the row, so that
equal magnitudes go to the lowest row) to its best one and offers it, with
its row, in LDS.  The kernels take the pivot from the largest offered key
and the offering wave from the pivot row itself (the wave that holds that
row), instead of searching the offers for the first largest one.  That is
the same choice whenever the offered keys are distinct and the best one is
positive; this model checks it against the search on random columns with
many magnitude ties, zeros and NaNs, for the 2D line-block layout (two
threads per row, 32 rows per wave, 8 waves, 8-bit row field) and the 3D
plane-block layout (row i in thread i mod 1024, 64 threads per wave, 16
waves, 13-bit row field)."""

import numpy as np
import pytest


def _key(m, row, bits):
    # NaN magnitude: the row stays a candidate with magnitude 0
    m = np.float32(0.0) if np.isnan(m) else np.float32(m)
    b = int(m.view(np.uint32))
    mask = (1 << bits) - 1
    return (b & ~mask & 0xFFFFFFFF) | (mask - row)


def _rows_of_threads(layout, n):
    # (thread, row) pairs as the kernels lay rows out over their threads
    if layout == "2d":                      # threads 2 r and 2 r + 1 hold row r
        return [(t, t >> 1) for t in range(2 * n)]
    return [(t, t + 1024 * s) for s in range(2) for t in range(1024)   # thread t holds rows t + 1024 s
            if t + 1024 * s < n]


def _wave_offers(keys, layout, nwaves):
    # each wave (64 threads) offers the best key among the rows it holds
    offers = [0] * nwaves
    for t, r in _rows_of_threads(layout, len(keys)):
        offers[t >> 6] = max(offers[t >> 6], keys[r])
    return offers


def _search(offers):
    # the first wave holding the largest offer
    best, bw = offers[0], 0
    for w in range(1, len(offers)):
        if offers[w] > best:
            best, bw = offers[w], w
    return best, bw


def _column(rng, n):
    # magnitudes from a few distinct values (ties after the bit truncation),
    # zeros and NaNs
    base = rng.choice([0.0, 1e-3, 0.5, 0.5000001, 1.0, 2.0, 3.0], size=n)
    col = base * np.exp(1j * rng.uniform(0, 2 * np.pi, size=n))
    col[rng.random(n) < 0.05] = np.nan
    return col


@pytest.mark.parametrize("layout", ["2d", "3d"])
def test_pivot_from_best_offer_equals_search(layout):
    rng = np.random.default_rng(20030258 + (layout == "3d"))
    # the offering wave as the kernels compute it from the pivot row
    if layout == "2d":
        bits, nwaves = 8, 8
        wave_of = lambda p: p >> 5                       # noqa: E731
        sizes = (16, 96, 144, 160)
    else:
        bits, nwaves = 13, 16
        wave_of = lambda p: (p & 1023) >> 6              # noqa: E731
        sizes = (100, 1024, 1936, 2048)
    checked = 0
    for n in sizes:
        for _ in range(40):
            col = _column(rng, n)
            used = rng.random(n) < rng.uniform(0.0, 0.9)
            used[rng.integers(n)] = False                # a candidate exists
            keys = [0 if used[r] else
                    _key(abs(col[r].real) + abs(col[r].imag), r, bits)
                    for r in range(n)]
            offers = _wave_offers(keys, layout, nwaves)
            nz = [k for k in offers if k]
            assert len(nz) == len(set(nz)), "offered keys must be distinct"
            best_s, bw_s = _search(offers)
            best = max(offers)
            p = ((1 << bits) - 1) - (best & ((1 << bits) - 1))
            assert best == best_s and best > 0
            assert wave_of(p) == bw_s
            # the pivot is the largest magnitude among unused rows, lowest
            # row on ties (NaN counted as zero), at the key's precision
            mags = {r: (0.0 if np.isnan(abs(col[r])) else
                        np.float32(abs(col[r].real) + abs(col[r].imag)))
                    for r in range(n) if not used[r]}
            top = max((int(np.float32(m).view(np.uint32)) >> bits) for m in mags.values())
            rows = [r for r, m in mags.items()
                    if (int(np.float32(m).view(np.uint32)) >> bits) == top]
            assert p == min(rows)
            checked += 1
    assert checked == 160
