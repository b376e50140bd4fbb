"""The comparison (Hudgin) extension of Sec. 3.2 in the oracle (CPU only): slopes repeated from
the pupil edge along columns (x) and rows (y), the nearest in-pupil cell filling every other
cell of the line, measurement kept, Eq. 5 imposed."""
import numpy as np

from oracle import fwr_oracle as O
from paper_1705_04298_amd import inputs as I


def _ext(n, N, mask, seed):
    slopes = I.random_slopes(1, n, seed=seed)[0] * mask
    s0x, s0y, P = O.padded_measurement(slopes, mask, N)
    return s0x, s0y, P, O.hudgin_extend(s0x, s0y, P)


def test_edge_repetition_and_measurement():
    n, N = 40, 80
    mask = I.pupil_mask(n)
    s0x, s0y, P, (sx, sy) = _ext(n, N, mask, 1)
    assert np.array_equal(sx[P], s0x[P]) and np.array_equal(sy[P], s0y[P])
    for c in range(N - 1):  # Eq. 5 rewrites column N-1 of s_x only
        rows = np.flatnonzero(P[:, c])
        if rows.size == 0:
            assert np.all(sx[:, c] == 0.0)
            continue
        assert np.all(sx[:rows[0], c] == s0x[rows[0], c])      # repeated up from the top edge
        assert np.all(sx[rows[-1] + 1:, c] == s0x[rows[-1], c])  # and down from the bottom edge
    for r in range(N - 1):
        cols = np.flatnonzero(P[r, :])
        if cols.size == 0:
            assert np.all(sy[r, :] == 0.0)
            continue
        assert np.all(sy[r, :cols[0]] == s0y[r, cols[0]])
        assert np.all(sy[r, cols[-1] + 1:] == s0y[r, cols[-1]])


def test_obstruction_filled_from_the_nearest_cell():
    n, N = 8, 12
    mask = np.ones((n, n), dtype=np.uint8)
    mask[2:6, 3] = 0  # a gap of 4 cells in column 3 (grid column 5)
    s0x, s0y, P, (sx, sy) = _ext(n, N, mask, 2)
    c, o = 3 + 2, 2
    top, bottom = s0x[o + 1, c], s0x[o + 6, c]  # rows 1 and 6 of the window bound the gap
    assert sx[o + 2, c] == top and sx[o + 3, c] == top      # nearer to the top edge, or a tie
    assert sx[o + 4, c] == bottom and sx[o + 5, c] == bottom


def test_periodicity_imposed():
    s0x, s0y, P, (sx, sy) = _ext(24, 48, I.pupil_mask(24), 3)
    assert np.abs(sx.sum(axis=1)).max() < 1e-12 and np.abs(sy.sum(axis=0)).max() < 1e-12
