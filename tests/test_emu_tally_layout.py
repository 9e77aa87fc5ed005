"""The library's layout of the forward's absorbed-luminosity tally, checked
on every cell by the CPU harness with the library's own grid set-up: units
of whole bricks (at least one 64-byte segment of FP64 values) scattered by a
multiplicative permutation over a power-of-two unit count.  Every bricked
cell gets its own slot, the inverse map returns it, cells keep their order
inside a unit, and the slots per wavelength stay below twice the bricked
cells.  The end-to-end effect -- the same absorbed tally as the oracle's --
is pinned by the parity tests of every grid kind."""
import pytest

from paper_1410_1629_amd import binding
from test_emu_tree import _tree

BOX = (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0)


@pytest.mark.parametrize("n, prec, brick, want_tb", [
    ((8, 8, 8), 1, 0, 5),          # 32 FP32 cells per brick
    ((13, 7, 5), 0, 0, 4),         # ragged, 16 FP64 cells per brick, padded bricks
    ((256, 256, 64), 1, 0, 5),     # the spiral's grid: 2^17 bricks, no padding
    ((9, 3, 17), 1, (0, 0, 0), 3), # one-cell bricks: units of 8 cells
    ((5, 40, 6), 0, (1, 2, 0), 3),
])
def test_regular_grid_tally_layout(E, n, prec, brick, want_tb):
    shape = binding.brick(*brick) if brick else 0
    ntal, tb = E.tally_layout(BOX, n, prec, brick_shape=shape)
    assert tb == want_tb
    if n == (256, 256, 64):
        assert ntal == 256 * 256 * 64


def test_rectilinear_grid_tally_layout(E, W):
    planes = [W.power_law_planes(-1.0, 1.0, m, r) for m, r in ((12, 4.0), (7, 2.0), (30, 8.0))]
    ntal, tb = E.tally_layout(BOX, (12, 7, 30), 1, planes=planes)
    assert tb == 5 and ntal >= 12 * 7 * 30


@pytest.mark.parametrize("kind", ["kd", "oct", "regular"])
def test_tree_grid_tally_layout(E, W, kind):
    T = _tree(W, kind)
    ntal, tb = E.tally_layout(BOX, (T.n_cells, 1, 1), 1, tree=T.tree())
    assert tb == 3 and T.n_cells <= ntal < 2 * (T.n_cells + 8)
    assert ntal & (ntal - 1) == 0
