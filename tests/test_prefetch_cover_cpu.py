"""The solve kernel's fetch-ahead of cost-matrix rows, checked on the CPU.

While k <= 960 the last wavefront loads, for the unit two allotments ahead,
word min(16 * lane, k - 1) of its row on every lane 0..62 with
16 * lane < k + 15, and the unit's most suitable center on lane 63.  These
tests check that those words touch every 64-byte line the row spans, for
every alignment a row can start at, and never read outside the row or use
lane 63 for a row word."""
import pytest


def touched_lines(k, start):
    lanes = [lane for lane in range(63) if 16 * lane < k + 15]
    words = [min(16 * lane, k - 1) for lane in lanes]
    assert max(lanes) < 63 and all(0 <= w < k for w in words)
    return {(start + 4 * w) // 64 for w in words}


@pytest.mark.parametrize("k", list(range(1, 130)) + [255, 256, 257, 500, 511, 512, 513, 959, 960])
def test_every_line_of_the_row_is_touched(k):
    for start in range(0, 64, 4):                 # rows start at any 4-byte alignment
        spanned = set(range(start // 64, (start + 4 * k - 1) // 64 + 1))
        assert touched_lines(k, start) == spanned, (k, start)
