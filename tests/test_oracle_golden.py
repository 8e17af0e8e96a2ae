"""Oracle counts against the grid table the paper prints (Sec. 4.1, Table 1).

Only the coarsest row of the driven-cavity hierarchy is a uniform grid (three
uniform refinements of the unit square).  The printed n_DoF of that row is
three unknowns per grid vertex (an equal-order count), so it pins the oracle's
cell and vertex numbering: n_e = N^2 cells and n_DoF = 3 (N+1)^2.  The
Taylor-Hood space has 2 (2N+1)^2 + (N+1)^2 unknowns on the same grid.  The
finer, adaptively refined rows pin the quadtree grids and the hanging-node
rule of oracle/adaptive.py.
"""
import os

import numpy as np

from oracle.grid import Grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_coarse_grid.txt")


def _rows():
    return [tuple(int(v) for v in line.split()) for line in open(GOLDEN)
            if line.strip() and not line.startswith("#")]


def test_table1_coarsest_grid_counts():
    (refinements, n_e, n_dof), = _rows()
    N = 2 ** refinements
    g = Grid(2, N, 0b1111)
    assert N * N == n_e
    assert 3 * g.nP == n_dof                      # pressure space = grid vertices
    assert g.nP == int(np.prod([N + 1] * 2))
    assert g.n == 2 * (2 * N + 1) ** 2 + (N + 1) ** 2 == 659


GRIDS = os.path.join(os.path.dirname(__file__), "golden", "table1_grids.txt")


def test_table1_adaptive_hierarchy_counts():
    """All ten rows of Table 1.  The band widths of the refinement rule are a
    reading chosen to give the element counts; the DoF counts (three per
    regular vertex, hanging nodes excluded, Sec. 2 / Fig. 2) are not used to
    choose them and must follow: they do for every grid, up to 3,063,075 DoFs
    on Omega^10.  Every grid is 2:1 balanced (checked up to Omega^7)."""
    from oracle import adaptive as ad
    rows = [tuple(int(v) for v in line.split()) for line in open(GRIDS)
            if line.strip() and not line.startswith("#")]
    grids = ad.cavity_grids(len(rows))
    for (k, n_e, n_dof), leaves in zip(rows, grids):
        _, _, regular = ad.vertex_counts(leaves)
        assert len(leaves) == n_e, k
        assert 3 * regular == n_dof, (k, 3 * regular, n_dof)
        if k <= 7:
            assert ad.is_balanced(leaves), k
