"""Vanka subdomains, their restricted (owned) sets and the MV colouring (Sec. 3).

Vertex patch k (pressure-oriented subdomain, Sec. 3): the pressure DoF p_k and
every free velocity DoF coupled to it by B^T, i.e. all components at the Q2
nodes of the elements that contain vertex k: nodes a in [2k-2, 2k+2]^d.
Element patch e: all free velocity DoFs at the 3^d Q2 nodes of element e plus
its 2^d pressure vertices.
Local order: component-major, then lexicographic over nodes (x fastest), then
the pressure DoF(s).  L_i = R_i L R_i^T is the principal submatrix (Sec. 3).

Owned set of RAV (the rows kept by the modified prolongation of eq. 13).  In
Sec. 3 a patch keeps its own pressure unknown together with the velocity
unknowns located at that same vertex; this partitions the DoFs only when
velocity lives on vertices (Q1-Q1).  For
Q2/Q1 this oracle uses the floor rule, which agrees with the paper's rule on
vertex nodes and also assigns edge/face/cell nodes so that sum_i G_i = I:
* vertex patches: velocity node a is owned by vertex floor(a/2); pressure k by k;
* element patches: node a by element min(floor(a/2), N-1); pressure k by
  element min(k, N-1) (componentwise).

MV order: patches in ascending colour, lexicographic within a colour.  Vertex
patches use colour sum_d (k_d mod 4) 4^d, element patches sum_d (e_d mod 3) 3^d;
two patches of one colour never touch each other's residual rows, so the
sequential product of eq. (11) in this order equals the colour-parallel form.
"""
from __future__ import annotations

import itertools

import numpy as np

from .grid import Grid

VERTEX = 0
ELEMENT = 1


def _box(lo, hi, dim):
    """Integer points of the box [lo, hi] (per dim), lexicographic x fastest."""
    ranges = [range(lo[d], hi[d] + 1) for d in range(dim)]
    pts = [p[::-1] for p in itertools.product(*ranges[::-1])]
    return np.asarray(pts, dtype=np.int64).reshape(-1, dim)


def n_patches(grid: Grid, kind: int) -> int:
    return grid.nP if kind == VERTEX else grid.N ** grid.dim


def patch_anchor(grid: Grid, kind: int, i: int):
    """Vertex k or element e of patch i (lexicographic, x fastest)."""
    base = grid.np1 if kind == VERTEX else grid.N
    out = []
    for _ in range(grid.dim):
        out.append(i % base)
        i //= base
    return np.asarray(out, dtype=np.int64)


def patch_dofs(grid: Grid, kind: int, i: int) -> np.ndarray:
    """Global DoF list I_i in local order (free DoFs only)."""
    k = patch_anchor(grid, kind, i)
    d = grid.dim
    if kind == VERTEX:
        lo = np.maximum(2 * k - 2, 0)
        hi = np.minimum(2 * k + 2, 2 * grid.N)
        pverts = k[None, :]
    else:
        lo = 2 * k
        hi = 2 * k + 2
        pverts = _box(k, k + 1, d)
    nodes = _box(lo, hi, d)
    dofs = []
    for c in range(d):
        g = grid.vel(c, nodes)
        dofs.append(g[grid.free[g]])
    dofs.append(grid.pres(pverts))
    return np.concatenate(dofs)


def owner_of_dofs(grid: Grid, kind: int) -> np.ndarray:
    """Owning patch of every DoF (floor rule); -1 for masked DoFs."""
    d = grid.dim
    own = np.full(grid.n, -1, dtype=np.int64)
    base = grid.np1 if kind == VERTEX else grid.N
    if kind == VERTEX:
        vo = grid.vnode // 2
        po = grid.pnode
    else:
        vo = np.minimum(grid.vnode // 2, grid.N - 1)
        po = np.minimum(grid.pnode, grid.N - 1)
    strides = base ** np.arange(d)
    vidx = vo @ strides
    pidx = po @ strides
    for c in range(d):
        own[c * grid.nV:(c + 1) * grid.nV] = vidx
    own[d * grid.nV:] = pidx
    own[~grid.free] = -1
    return own


def owned_local(grid: Grid, kind: int, i: int, dofs: np.ndarray, owner: np.ndarray) -> np.ndarray:
    """Local indices (into I_i) of the DoFs owned by patch i."""
    return np.nonzero(owner[dofs] == i)[0]


def colour(grid: Grid, kind: int, i: int) -> int:
    k = patch_anchor(grid, kind, i)
    m = 4 if kind == VERTEX else 3
    return int(sum(int(k[d] % m) * m ** d for d in range(grid.dim)))


def n_colours(grid: Grid, kind: int) -> int:
    return (4 if kind == VERTEX else 3) ** grid.dim


def mv_order(grid: Grid, kind: int) -> np.ndarray:
    """Canonical MV order: ascending colour, lexicographic within a colour."""
    npt = n_patches(grid, kind)
    cols = np.asarray([colour(grid, kind, i) for i in range(npt)])
    return np.lexsort((np.arange(npt), cols))


class PatchSet:
    """All patches of one level with their DoF lists and owned local indices."""

    def __init__(self, grid: Grid, kind: int):
        self.grid = grid
        self.kind = kind
        self.count = n_patches(grid, kind)
        self.owner = owner_of_dofs(grid, kind)
        self.dofs = [patch_dofs(grid, kind, i) for i in range(self.count)]
        self.owned = [owned_local(grid, kind, i, self.dofs[i], self.owner) for i in range(self.count)]
        self.order = mv_order(grid, kind)
