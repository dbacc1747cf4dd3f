"""Host check of the colouring behind the reproducible-sums flush (no GPU).

Each raster work item of tile (tp, tt) deposits into the region of rows
[tp TP, tp TP + TP + 32) and ticks [tt TT, tt TT + TT + 16) (the tile plus the
halo of the tile shapes in wcsim.h).  The owner flush adds the regions of one
colour (tp mod CP, tt mod CT) side by side with plain read-add-writes, which
is only race-free if two tiles of one colour never share a cell, and it
reaches every cell of a region only if the colours tile the grid.  Checked by
brute force over every cell of a grid of several colour periods."""
import itertools

import numpy as np
import pytest

HALO_P, HALO_T = 32, 16
SHAPES = [(32, 8), (32, 32), (64, 8)]  # tile shape ids 0, 1, 2


def colours(tp_size, tt_size):
    rp, rt = tp_size + HALO_P, tt_size + HALO_T
    return -(-rp // tp_size), -(-rt // tt_size)  # ceil


@pytest.mark.parametrize("shape", SHAPES)
def test_tiles_of_one_colour_never_share_a_cell(shape):
    TP, TT = shape
    CP, CT = colours(TP, TT)
    RP, RT = TP + HALO_P, TT + HALO_T
    ntp, ntt = 3 * CP + 1, 3 * CT + 2
    owner = {}  # (colour, cell) -> tile
    cover = np.zeros((ntp * TP + RP, ntt * TT + RT), np.int32)
    for tp, tt in itertools.product(range(ntp), range(ntt)):
        col = (tp % CP, tt % CT)
        cover[tp * TP:tp * TP + RP, tt * TT:tt * TT + RT] += 1
        for r in range(tp * TP, tp * TP + RP, 4):
            for c in range(tt * TT, tt * TT + RT, 4):
                key = (col, r, c)
                assert key not in owner, (shape, (tp, tt), owner.get(key))
                owner[key] = (tp, tt)
    # a cell is reached by at most one tile per colour: CP * CT tiles at most
    assert cover.max() <= CP * CT


@pytest.mark.parametrize("shape", SHAPES)
def test_fewer_colours_would_share_cells(shape):
    """The colour counts are the least that work: with one colour fewer along
    either axis, two tiles of one colour overlap."""
    TP, TT = shape
    CP, CT = colours(TP, TT)
    RP, RT = TP + HALO_P, TT + HALO_T
    assert (CP - 1) * TP < RP and (CT - 1) * TT < RT
    assert (CP, CT) == {(32, 8): (2, 3), (32, 32): (2, 2), (64, 8): (2, 3)}[shape]
