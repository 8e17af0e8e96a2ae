"""Oracle counts against the grid table the paper prints (Sec. 4.1, Table 1).

Only the coarsest row of the driven-cavity hierarchy is a uniform grid (three
uniform refinements of the unit square); the finer rows are adaptive and out
of scope.  The printed n_DoF of that row is three unknowns per grid vertex
(an equal-order count), so it pins the oracle's cell and vertex numbering:
n_e = N^2 cells and n_DoF = 3 (N+1)^2.  The Taylor-Hood space the path uses
has 2 (2N+1)^2 + (N+1)^2 unknowns on the same grid.
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
