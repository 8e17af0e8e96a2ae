"""Stabilized Q1-Q1 Stokes on adaptively refined quadtree grids with hanging
nodes, and its multigrid hierarchy (Sec. 2, eqs. 5-8 and Fig. 2; Sec. 3,
eq. 13; Sec. 4.1).  Test infrastructure: plain, slow, fp64 (scipy.sparse).

Grid: leaf cells (x0, y0, s) in integer lattice units inside the rectangle
[0, M] x [0, My] (My = M: the unit square of the driven cavity,
rav_inputs.cavity_grids; the channel of the cylinder benchmark,
rav_inputs.channel_grids), lengths in units of the height My.  The domain is
the union of the leaves: cells of the rectangle that no leaf covers are holes.  Vertices are leaf corners; a corner that is the
midpoint of an edge of a larger neighbouring leaf is a hanging node: its value
is the mean of that edge's two endpoints (recursively, if an endpoint hangs
itself), so the discrete space is the conforming Q1 space on the grid.  The
unknowns are three per regular vertex, numbered [u_x; u_y; p] with the regular
vertices in lexicographic order (x fastest), as on uniform grids.

Operator: the element matrices of oracle.q1q1 (2-point Gauss; A with viscosity
eta, B = -(div v, q), stabilization C = -beta diam_e^2 (grad q, grad p)_e with
each leaf's own diameter) assembled over the leaves with their corners, then
restricted to the conforming space: L = T^T L_corners T with T the constraint
map from regular unknowns to all corner values.  Velocity is Dirichlet on the
boundary of holes and on the sides of the rectangle set in dmask (bit 0:
x = 0, 1: x = M, 2: y = 0, 3: y = My), free on the other sides (the natural
outflow condition, Sec. 4.2); data enter through the lifting
b = -L_all[free, masked] u_D (the driven cavity's lid, Sec. 4.1; the
channel's parabolic inflow, eq. 14).  With every side Dirichlet the pressure
is fixed only up to a constant (the coarse solve then imposes zero mean).

Vanka patches (Sec. 3): the patch of regular vertex i holds p_i and every free
velocity unknown of the leaves around vertex i (the structural nonzeros of row
i of B^T), a hanging corner standing for the regular vertices that constrain
it (the paper's implicit inclusion of hanging nodes, Fig. 2); RAV owns p_i and
the velocity at vertex i.  MV order: greedy colouring in patch order by
vertex sets (mv_colouring: a patch may not write x where a same-colour patch
reads it), colour-major.

Transfer between consecutive grids (each refines the previous): the coarse FE
function evaluated at the fine regular vertices (bilinear on the coarse leaf
that contains the vertex, hanging coarse corners through their constraints);
restriction is the transpose; masked rows and columns zero.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import mg
from . import smoothers as sm
from .q1q1 import RefQ1


class AdaptiveGrid:
    def __init__(self, leaves, M: int, beta: float, eta: float = 1.0, My: int | None = None, dmask: int = 0xF):
        self.leaves = np.asarray(leaves, dtype=np.int64)
        self.M = M
        self.My = My = M if My is None else My
        self.dmask = dmask
        self.dim = 2
        x0, y0, s = self.leaves[:, 0], self.leaves[:, 1], self.leaves[:, 2]
        h = s // 2
        corners = np.stack([np.stack([x0 + a * s, y0 + b * s], 1) for b in (0, 1) for a in (0, 1)], 1)   # (n,4,2), local a = ax + 2 ay
        key = lambda p: p[..., 0] * (My + 1) + p[..., 1]
        ckey = key(corners)
        mids = np.stack([[x0 + h, y0], [x0 + h, y0 + s], [x0, y0 + h], [x0 + s, y0 + h]], 0).transpose(2, 0, 1)   # (n,4,2)
        ends = [((x0, y0), (x0 + s, y0)), ((x0, y0 + s), (x0 + s, y0 + s)), ((x0, y0), (x0, y0 + s)),
                ((x0 + s, y0), (x0 + s, y0 + s))]
        mkey = key(mids)
        allc = np.unique(ckey)
        hang = np.intersect1d(allc, np.unique(mkey), assume_unique=True)
        # endpoints of the coarse edge of every hanging node
        self.hang_ends = {}
        for e in range(4):
            hit = np.isin(mkey[:, e], hang)
            for li in np.nonzero(hit)[0]:
                (ax, ay), (bx, by) = ends[e]
                self.hang_ends[int(mkey[li, e])] = (int(ax[li] * (My + 1) + ay[li]), int(bx[li] * (My + 1) + by[li]))
        reg = np.setdiff1d(allc, hang, assume_unique=True)
        rx, ry = reg // (My + 1), reg % (My + 1)
        order = np.lexsort((rx, ry))            # y slowest, x fastest
        self.reg_keys = reg[order]
        self.rx, self.ry = rx[order], ry[order]
        self.nV = len(self.reg_keys)
        self.n = 3 * self.nV
        self.reg_index = {int(k): i for i, k in enumerate(self.reg_keys)}
        self.corner_keys = ckey
        self.beta, self.eta = beta, eta
        self.h_leaf = s / My
        on_b = self._dirichlet(ckey)
        self.dirichlet_node = on_b
        self.free = np.ones(self.n, dtype=bool)
        self.free[: self.nV] = ~on_b
        self.free[self.nV: 2 * self.nV] = ~on_b
        self.all_dirichlet = dmask == 0xF

    def _dirichlet(self, ckey):
        """Dirichlet flag per regular vertex.  The leaves that have vertex v as
        a corner fill some of the four quadrants around v; v is on the boundary
        when a quadrant is empty, and Dirichlet when an empty quadrant lies in
        the rectangle (a hole) or beyond a side whose dmask bit is set."""
        filled = np.zeros((self.nV, 2, 2), dtype=bool)   # [v, quadrant on +x side, quadrant on +y side]
        for li in range(len(self.leaves)):
            for a in range(4):
                v = self.reg_index.get(int(ckey[li, a]))
                if v is not None:
                    filled[v, 1 - (a & 1), 1 - (a >> 1)] = True
        out = np.zeros(self.nV, dtype=bool)
        for v in range(self.nV):
            x, y = int(self.rx[v]), int(self.ry[v])
            for qx in (0, 1):
                for qy in (0, 1):
                    if filled[v, qx, qy]:
                        continue
                    beyond = []
                    if qx == 0 and x == 0:
                        beyond.append(0)
                    if qx == 1 and x == self.M:
                        beyond.append(1)
                    if qy == 0 and y == 0:
                        beyond.append(2)
                    if qy == 1 and y == self.My:
                        beyond.append(3)
                    if not beyond or any((self.dmask >> side) & 1 for side in beyond):
                        out[v] = True
        return out

    def pressure_slice(self):
        return slice(2 * self.nV, self.n)

    def weights(self, key):
        """Regular-vertex weights of the value at lattice point `key`."""
        if key in self.reg_index:
            return {self.reg_index[key]: 1.0}
        a, b = self.hang_ends[key]
        out = {}
        for k in (a, b):
            for j, w in self.weights(k).items():
                out[j] = out.get(j, 0.0) + 0.5 * w
        return out

    def constraint(self):
        """T: (3 * n_corner_slots) x n map; corner slot = (leaf, local corner)."""
        nl = len(self.leaves)
        rows, cols, vals = [], [], []
        cache = {}
        for li in range(nl):
            for a in range(4):
                k = int(self.corner_keys[li, a])
                w = cache.get(k)
                if w is None:
                    w = cache[k] = self.weights(k)
                for j, v in w.items():
                    rows.append(li * 4 + a); cols.append(j); vals.append(v)
        T1 = sp.csr_matrix((vals, (rows, cols)), shape=(nl * 4, self.nV))
        return sp.block_diag([T1] * 3, format="csr")

    def corner_matrix(self):
        """Block-diagonal element matrices over the (leaf, corner) slots, fields
        [u_x; u_y; p] each of 4 n_leaves slots."""
        ref = RefQ1(2)
        nl = len(self.leaves)
        rows, cols, vals = [], [], []
        base = np.arange(nl) * 4
        for li in range(nl):
            hl = self.h_leaf[li]
            Ae = ref.stiffness(hl, np.full(4, self.eta))
            Be = ref.divergence(hl)
            Ce = ref.stabilization(hl, self.beta)
            o = base[li]
            for a in range(4):
                for b in range(4):
                    for c in range(2):
                        rows.append(c * 4 * nl + o + a); cols.append(c * 4 * nl + o + b); vals.append(Ae[a, b])
                        rows.append(c * 4 * nl + o + a); cols.append(2 * 4 * nl + o + b); vals.append(Be[c, a, b])
                        rows.append(2 * 4 * nl + o + b); cols.append(c * 4 * nl + o + a); vals.append(Be[c, a, b])
                    rows.append(2 * 4 * nl + o + a); cols.append(2 * 4 * nl + o + b); vals.append(Ce[a, b])
        return sp.csr_matrix((vals, (rows, cols)), shape=(12 * nl, 12 * nl))

    def assemble(self, keep_masked=False):
        T = self.constraint()
        L = (T.T @ self.corner_matrix() @ T).tocsr()
        if not keep_masked:
            D = sp.diags(self.free.astype(np.float64))
            L = (D @ L @ D).tocsr()
        L.eliminate_zeros()
        return L

    def lid_velocity(self, U=1.0):
        """Lid data: u_x = U on the top side strictly between the corners."""
        assert (self.dmask >> 3) & 1, "the lid needs a Dirichlet top side"
        u = np.zeros(self.n)
        top = (self.ry == self.My) & (self.rx > 0) & (self.rx < self.M)
        u[: self.nV][top] = U
        return u

    def inflow_velocity(self, ubar):
        """Inflow data of the channel (eq. 14): u_x = 4 ubar y (H - y) / H^2,
        u_y = 0 on the side x = 0, H the height (1 in these units)."""
        u = np.zeros(self.n)
        y = self.ry / self.My
        inflow = (self.rx == 0) & self.dirichlet_node
        u[: self.nV][inflow] = 4.0 * ubar * y[inflow] * (1.0 - y[inflow])
        return u

    def lifting(self, uD):
        """b = -L_all[free, masked] uD for Dirichlet data uD on the masked DoFs."""
        L_all = self.assemble(keep_masked=True)
        b = -(L_all @ np.where(self.free, 0.0, uD))
        b[~self.free] = 0.0
        return b

    def lid_rhs(self, U=1.0):
        return self.lifting(self.lid_velocity(U))

    def patches(self, L=None):
        """Vanka patch of every regular vertex i: p_i and the free velocity at the
        vertices of the leaves that have i as a corner, a hanging corner standing
        for the regular vertices that constrain it.  Local order: velocity
        component-major, vertices by id; p_i last.  Owned: velocity at i and p_i."""
        nV = self.nV
        touch = [[] for _ in range(nV)]
        for li in range(len(self.leaves)):
            for a in range(4):
                j = self.reg_index.get(int(self.corner_keys[li, a]))
                if j is not None:
                    touch[j].append(li)
        cache = {}
        dofs, owned = [], []
        for i in range(nV):
            verts = set()
            for li in touch[i]:
                for a in range(4):
                    k = int(self.corner_keys[li, a])
                    w = cache.get(k)
                    if w is None:
                        w = cache[k] = self.weights(k)
                    verts.update(w.keys())
            verts = np.array(sorted(verts), dtype=np.int64)
            I = np.concatenate([verts, nV + verts, [2 * nV + i]])
            I = I[self.free[I]]
            dofs.append(I)
            own = [np.nonzero(I == c * nV + i)[0] for c in range(2)] + [np.array([len(I) - 1])]
            owned.append(np.concatenate(own).astype(np.int64))
        return dofs, owned

    def locate(self, px, py):
        """Leaf containing lattice point (px, py) (the first one found)."""
        x0, y0, s = self.leaves[:, 0], self.leaves[:, 1], self.leaves[:, 2]
        hit = np.nonzero((x0 <= px) & (px <= x0 + s) & (y0 <= py) & (py <= y0 + s))[0]
        return int(hit[0])


def prolongation(fine: AdaptiveGrid, coarse: AdaptiveGrid):
    """Coarse FE function at the fine regular vertices (all three fields)."""
    rows, cols, vals = [], [], []
    for i in range(fine.nV):
        px, py = int(fine.rx[i]), int(fine.ry[i])
        li = coarse.locate(px, py)
        x0, y0, s = coarse.leaves[li]
        tx, ty = (px - x0) / s, (py - y0) / s
        for a in range(4):
            ax, ay = a & 1, a >> 1
            w = (tx if ax else 1 - tx) * (ty if ay else 1 - ty)
            if w == 0.0:
                continue
            k = int(coarse.corner_keys[li, a])
            for j, v in coarse.weights(k).items():
                rows.append(i); cols.append(j); vals.append(w * v)
    P1 = sp.csr_matrix((vals, (rows, cols)), shape=(fine.nV, coarse.nV))
    P = sp.block_diag([P1] * 3, format="csr")
    P = (sp.diags(fine.free.astype(np.float64)) @ P @ sp.diags(coarse.free.astype(np.float64))).tocsr()
    P.eliminate_zeros()
    return P


def leaf_vertex_sets(grid: AdaptiveGrid):
    """V_e for every leaf: the regular vertices its corners depend on."""
    cache = {}
    sets = []
    for li in range(len(grid.leaves)):
        vs = set()
        for a in range(4):
            k = int(grid.corner_keys[li, a])
            w = cache.get(k)
            if w is None:
                w = cache[k] = grid.weights(k)
            vs.update(w.keys())
        sets.append(vs)
    return sets


def mv_colouring(grid: AdaptiveGrid):
    """Greedy colouring in patch order, by vertex sets (so that it does not
    depend on which assembled entries happen to cancel): the row pattern of
    vertex v is the union of V_e over the leaves with v in V_e; the vertex set
    of patch i is the union of V_e over the leaves that have i as a corner
    (masked vertices included); patch i takes the smallest colour not used by
    an earlier patch whose vertex set meets the row pattern of one of patch
    i's vertices.  Returns the colour of every patch."""
    sets = leaf_vertex_sets(grid)
    nV = grid.nV
    rows = [set() for _ in range(nV)]
    for vs in sets:
        for v in vs:
            rows[v] |= vs
    pverts = [set() for _ in range(nV)]
    for li in range(len(grid.leaves)):
        for a in range(4):
            i = grid.reg_index.get(int(grid.corner_keys[li, a]))
            if i is not None:
                pverts[i] |= sets[li]
    holders = [[] for _ in range(nV)]
    for i in range(nV):
        for v in pverts[i]:
            holders[v].append(i)
    colour = -np.ones(nV, dtype=np.int64)
    for i in range(nV):
        reach = set()
        for v in pverts[i]:
            reach |= rows[v]
        banned = {int(colour[q]) for u in reach for q in holders[u] if q < i}
        c = 0
        while c in banned:
            c += 1
        colour[i] = c
    return colour


class AdaptiveLevel(mg.Level):
    def __init__(self, grid: AdaptiveGrid, smooth=True):
        self.grid = grid
        self.L = grid.assemble()
        self.free = grid.free
        self.kind = mg.VERTEX
        self.P = None
        if smooth:
            dofs, owned = grid.patches()

            class _PS:
                pass

            ps = _PS()
            ps.dofs, ps.owned, ps.count = dofs, owned, len(dofs)
            ps.colour = mv_colouring(grid)
            ps.order = np.lexsort((np.arange(ps.count), ps.colour))
            self.patches = ps
            self.lus = sm.factor(self.L, dofs)
            self._W = None
        else:
            self.patches = None


class AdaptiveHierarchy(mg.Hierarchy):
    """V-cycle over the grids of an adaptive hierarchy (grid 0 coarsest); the
    smoothing, V-cycle and solve of the uniform-grid oracle."""

    def __init__(self, leaves_list, M, beta, eta=1.0, My=None, dmask=0xF):
        self.dim = 2
        grids = [AdaptiveGrid(lv, M, beta, eta, My, dmask) for lv in leaves_list]
        self.levels = [AdaptiveLevel(g, smooth=l > 0) for l, g in enumerate(grids)]
        for l in range(1, len(grids)):
            self.levels[l].P = prolongation(grids[l], grids[l - 1])
        self._coarse_setup()
