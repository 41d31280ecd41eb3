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
