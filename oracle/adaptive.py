"""Vertex and hanging-node counts of the adaptively refined quadrilateral grids
of the driven-cavity hierarchy (Sec. 4.1, Table 1; Sec. 2, Fig. 2).  Test
infrastructure: plain Python/numpy.  The leaf lists themselves come from the
input generator (rav_inputs.cavity_grids).

A grid is a list of leaf cells of a quadtree over [0,1]^2 whose root level is
the uniform 8 x 8 grid; a leaf is (x0, y0, s) in integer units of half the
finest possible cell (side 1 / (16 * 2^L)), so that edge midpoints are lattice
points too.  Refining a leaf replaces it by its four children.

Refinement rule (a reading; the paper states only that the grids are refined
towards the boundary and that the refined region shrinks at every step): step
l refines every leaf of the current finest size that lies within w_l such
cells of the boundary.  The band widths w = 2, 3, 5, 8, 13, 19, 27, 31, 17 are
the ones for which the element counts follow; the number of degrees of
freedom then follows independently from the hanging-node rule below.

Degrees of freedom (equal-order Q1-Q1, three per vertex): every leaf corner
that is not a hanging node.  With the 2:1 balance of these grids a hanging
node is the midpoint of a leaf edge whose neighbouring leaf is refined: it is
a corner of the finer neighbours but its value is constrained by the two
endpoints of the coarse edge, so it carries no unknown (Fig. 2).
"""
from __future__ import annotations

import numpy as np

from rav_inputs import BANDS, BASE, cavity_grids, lattice  # noqa: F401  (the grids are inputs)


def _points(leaves, which):
    x0, y0, s = leaves[:, 0], leaves[:, 1], leaves[:, 2]
    h = s // 2
    if which == "corners":
        offs = [(0, 0), (1, 0), (0, 1), (1, 1)]
        pts = [(x0 + a * s, y0 + b * s) for a, b in offs]
    else:   # edge midpoints
        pts = [(x0 + h, y0), (x0 + h, y0 + s), (x0, y0 + h), (x0 + s, y0 + h)]
    M = int((leaves[:, 0] + leaves[:, 2]).max()) + 1
    return np.unique(np.concatenate([px * M + py for px, py in pts]))


def vertex_counts(leaves):
    """(all leaf corners, hanging nodes, regular vertices) of a grid."""
    corners = _points(leaves, "corners")
    mids = _points(leaves, "mids")
    hanging = np.intersect1d(corners, mids, assume_unique=True)
    return len(corners), len(hanging), len(corners) - len(hanging)


def is_balanced(leaves):
    """2:1 balance: leaves that share an edge segment differ by at most one level.
    Checked through the midpoints: a corner of a leaf that lies strictly inside
    another leaf's edge must be that edge's midpoint."""
    M = int((leaves[:, 0] + leaves[:, 2]).max()) + 1
    corners = _points(leaves, "corners")
    x0, y0, s = leaves[:, 0], leaves[:, 1], leaves[:, 2]
    for frac in (1, 3):                     # quarter points of every edge
        q = s * frac // 4
        for px, py in ((x0 + q, y0), (x0 + q, y0 + s), (x0, y0 + q), (x0 + s, y0 + q)):
            ok = s >= 4
            if np.isin((px * M + py)[ok], corners).any():
                return False
    return True


def uniform_refinement_counts(n_vertices: int, n_cells: int, holes: int, steps: int):
    """(cells, vertices) of a conforming quadrilateral mesh of a planar domain
    with `holes` holes after each of `steps` uniform refinements.  Euler's
    formula V - E + F = 1 - holes gives the edge count; one refinement adds a
    vertex per edge and per cell, splits every edge in two and every cell in
    four (four new interior edges)."""
    V, F = n_vertices, n_cells
    E = V + F - (1 - holes)
    out = []
    for _ in range(steps):
        V, E, F = V + E + F, 2 * E + 4 * F, 4 * F
        out.append((F, V))
    return out
