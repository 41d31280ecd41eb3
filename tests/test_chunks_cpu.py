"""Beam-by-beam chunking of D (the paper's small-card mode): range selection on the host."""
import numpy as np
import pytest

from paper_0908_4417_amd.plan import chunk_ranges


def _check(ranges, per, cap_bytes, n):
    assert ranges[0][0] == 0 and ranges[-1][1] == n
    for (a, b), (c, _) in zip(ranges, ranges[1:]):
        assert b == c and a < b
    for a, b in ranges:
        assert 8 * (per[b] - per[a]) <= cap_bytes


def test_whole_beams_when_they_fit():
    beam_rows = [4, 4, 4]
    per = np.concatenate([[0], np.cumsum(np.full(12, 10))])   # 80 bytes per row, 320 per beam
    r = chunk_ranges(per, beam_rows, 700)
    assert r == [(0, 8), (8, 12)]                               # two beams, then one
    _check(r, per, 700, 12)
    assert chunk_ranges(per, beam_rows, 10**9) == [(0, 12)]


def test_split_inside_a_large_beam():
    rng = np.random.default_rng(0)
    counts = rng.integers(0, 50, 30)
    per = np.concatenate([[0], np.cumsum(counts)])
    r = chunk_ranges(per, [30], 8 * 120)
    _check(r, per, 8 * 120, 30)
    r2 = chunk_ranges(per, [30], 8 * 120, by_beam=False)
    assert r == r2
    # every range is maximal: adding the next row would exceed the budget
    for a, b in r[:-1]:
        assert 8 * (per[b + 1] - per[a]) > 8 * 120


def test_row_too_large_and_empty_rows():
    per = np.array([0, 0, 0, 500, 500])
    with pytest.raises(ValueError, match="row 2"):
        chunk_ranges(per, [4], 8 * 100)
    r = chunk_ranges(np.zeros(6, dtype=np.int64), [2, 3], 8)
    assert r == [(0, 5)]


def test_row_ranges_c_contract():
    """fspb_row_ranges through the C ABI: size query, capacity and argument errors."""
    import ctypes as C
    import paper_0908_4417_amd as m
    L = m.lib()
    per = np.concatenate([[0], np.cumsum(np.full(12, 10))]).astype(np.int64)
    beams = np.array([4, 4, 4], dtype=np.int32)
    P64, P32 = C.POINTER(C.c_int64), C.POINTER(C.c_int32)
    pp, bp = per.ctypes.data_as(P64), beams.ctypes.data_as(P32)
    n = C.c_int32(-1)
    assert L.fspb_row_ranges(pp, 12, bp, 3, 700, None, 0, C.byref(n)) == m.FSPB_ERR_CAPACITY and n.value == 2
    small = np.full(2, -9, dtype=np.int32)
    assert L.fspb_row_ranges(pp, 12, bp, 3, 700, small.ctypes.data_as(P32), 1, C.byref(n)) == m.FSPB_ERR_CAPACITY
    assert (small == -9).all()                                  # nothing written
    out = np.zeros(3, dtype=np.int32)
    assert L.fspb_row_ranges(pp, 12, bp, 3, 700, out.ctypes.data_as(P32), 2, C.byref(n)) == m.FSPB_OK
    assert out.tolist() == [0, 8, 12]
    bad = np.array([4, 4, 3], dtype=np.int32)                   # beams do not cover the rows
    assert L.fspb_row_ranges(pp, 12, bad.ctypes.data_as(P32), 3, 700, None, 0, C.byref(n)) == m.FSPB_ERR_INVALID
    dec = per.copy()
    dec[5] = dec[4] - 1                                         # row pointers decrease
    assert L.fspb_row_ranges(dec.ctypes.data_as(P64), 12, None, 0, 700, None, 0, C.byref(n)) == m.FSPB_ERR_INVALID
    assert "decreases" in m.fspb_last_error()
    assert L.fspb_row_ranges(pp, 0, None, 0, 8, out.ctypes.data_as(P32), 2, C.byref(n)) == m.FSPB_OK and n.value == 0


def test_row_ranges_match_brute_force():
    """Greedy maximal ranges against an exhaustive scan on random row counts."""
    rng = np.random.default_rng(3)
    for trial in range(40):
        nb = int(rng.integers(1, 5))
        beam_rows = rng.integers(1, 9, nb).tolist()
        n = sum(beam_rows)
        per = np.concatenate([[0], np.cumsum(rng.integers(0, 30, n))]).astype(np.int64)
        budget = 8 * int(max(np.diff(per).max(), 1) * rng.uniform(1, 6))
        units = np.concatenate([[0], np.cumsum(beam_rows)])
        for by_beam in (True, False):
            got = chunk_ranges(per, beam_rows, budget, by_beam)
            j0, want = 0, []
            while j0 < n:
                fits = lambda j: 8 * (per[j] - per[j0]) <= budget
                ub = [u for u in units if u > j0 and fits(u)] if by_beam else []
                j1 = max(ub) if ub else max(j for j in range(j0 + 1, n + 1) if fits(j))
                want.append((j0, int(j1)))
                j0 = int(j1)
            assert got == want, (trial, by_beam)
