"""Stabilized equal-order Q1-Q1 Stokes discretization and its multigrid (Sec. 2,
eqs. 5-8; Sec. 3, eq. 13).  Test infrastructure: plain, slow, fp64.

Both velocity components and the pressure are continuous tensor-product
linears on the same vertices.  The pair is not inf-sup stable, so the lower
right block of the saddle-point system (eq. 6) is the stabilization matrix of
eq. (8): minus beta times, on every element, the square of the element's
diameter times the element integral of the product of the gradients of two
pressure basis functions.  The printed gradients in eq. (8) are those of the
velocity pair; this oracle reads them as the pressure pair (the block couples
pressure test and trial functions).  beta is a constant chosen by the caller;
the paper only asks for it to be large enough.  The element diameter of a
d-cube of side h is sqrt(d) h.

L = [[A, B], [B^T, C]]:
* A = (eta grad v, grad u) on each velocity component (no cross-component block),
* B = -(div v, q),
* C = -beta sum_e diam_e^2 (grad q, grad p)_e.
Element integrals use the tensor 2-point Gauss rule, which integrates every
constant-coefficient integrand of this pair exactly; with a viscosity that
varies between Gauss points (inclusions, eta_in inside the closed disc/ball)
the rule defines the discrete form.  Right-hand sides use the same rule.

Numbering: vertex v in [0, N]^d has lexicographic index sum_d v_d (N+1)^d
(x fastest); the global vector is [u_1; ...; u_d; p] with component c of the
velocity at index c*nV + v and the pressure at d*nV + v, nV = (N+1)^d.
Velocity on a Dirichlet side (bit 2d is x_d = 0, 2d+1 is x_d = 1) is masked:
x = 0 there and its rows and columns are dropped.

Vanka patches (Sec. 3): the patch of vertex k holds the pressure at k and every
free velocity DoF at the vertices of the elements that contain k, i.e. the
vertex block [k-1, k+1]^d clipped to the grid; local order component-major,
vertices lexicographic, the pressure last (2D interior: 2*9 + 1 = 19).  The
RAV owned set is the patch's pressure and the velocity at the same vertex,
which partitions the DoFs.  AV (eq. 12) and MV (eq. 11, colour order below)
use the same patches with every row of the local inverse.

Transfer: bilinear/trilinear interpolation of every field (nested spaces),
restriction its transpose; masked rows and columns zero.  Every level is
rediscretised (its own h in A, B and C).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from . import mg
from . import mms
from . import smoothers as sm
from .fem import q1_1d
from .transfer import _kron_dims, interp_1d_q1

GAUSS2_T = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
GAUSS2_W = np.array([0.5, 0.5])


def dq1_1d(t):
    t = np.asarray(t, dtype=np.float64)
    return np.stack([-np.ones_like(t), np.ones_like(t)])


class GridQ1:
    """Vertex numbering of the equal-order pair on [0,1]^d with N^d cells."""

    def __init__(self, dim: int, n_cells: int, dmask: int):
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        self.dim = dim
        self.N = n_cells
        self.dmask = dmask
        self.h = 1.0 / n_cells
        self.np1 = n_cells + 1
        self.nV = self.np1 ** dim
        self.nP = self.nV
        self.n = (dim + 1) * self.nV
        self.all_dirichlet = all((dmask >> b) & 1 for b in range(2 * dim))
        self.vnode = np.stack(np.unravel_index(np.arange(self.nV), (self.np1,) * dim)[::-1], axis=1)
        dir_node = np.zeros(self.nV, dtype=bool)
        for d in range(dim):
            if (dmask >> (2 * d)) & 1:
                dir_node |= self.vnode[:, d] == 0
            if (dmask >> (2 * d + 1)) & 1:
                dir_node |= self.vnode[:, d] == n_cells
        self.dirichlet_node = dir_node
        self.free = np.ones(self.n, dtype=bool)
        for c in range(dim):
            self.free[c * self.nV:(c + 1) * self.nV] = ~dir_node

    def vidx(self, v):
        v = np.asarray(v)
        idx = np.zeros(v.shape[:-1], dtype=np.int64)
        stride = 1
        for d in range(self.dim):
            idx = idx + v[..., d] * stride
            stride *= self.np1
        return idx

    def vel(self, c, v):
        return c * self.nV + self.vidx(v)

    def pres(self, v):
        return self.dim * self.nV + self.vidx(v)

    def elements(self):
        return np.stack(np.unravel_index(np.arange(self.N ** self.dim), (self.N,) * self.dim)[::-1], axis=1)

    def pressure_slice(self):
        return slice(self.dim * self.nV, self.n)


class RefQ1:
    """Q1 basis values and gradients at the 2^d Gauss points of [0,1]^d."""

    def __init__(self, dim: int):
        self.dim = dim
        pts, wts = [], []
        for idx in itertools.product(range(2), repeat=dim):
            idx = idx[::-1]
            pts.append([GAUSS2_T[i] for i in idx])
            wts.append(np.prod([GAUSS2_W[i] for i in idx]))
        self.qp, self.qw = np.asarray(pts), np.asarray(wts)
        self.nodes = np.asarray([i[::-1] for i in itertools.product(range(2), repeat=dim)], dtype=np.int64)
        nq, nb = len(self.qw), len(self.nodes)
        v1 = [q1_1d(self.qp[:, d]) for d in range(dim)]
        g1 = [dq1_1d(self.qp[:, d]) for d in range(dim)]
        self.phi = np.ones((nb, nq))
        self.grad = np.ones((dim, nb, nq))
        for a, idx in enumerate(self.nodes):
            for d in range(dim):
                self.phi[a] *= v1[d][idx[d]]
                for c in range(dim):
                    self.grad[c, a] *= (g1[d][idx[d]] if c == d else v1[d][idx[d]])
        self.G = np.einsum("cak,cbk->kab", self.grad, self.grad)   # (nq, nb, nb)

    def stiffness(self, h, eta_q):
        """(eta grad phi_a, grad phi_b) over a cube of side h; eta_q (..., nq)."""
        return h ** (self.dim - 2) * np.einsum("...k,kab->...ab", np.asarray(eta_q) * self.qw, self.G)

    def divergence(self, h):
        """B_e[c, a, k] = -(d phi_a / dx_c, psi_k) over a cube of side h."""
        return -h ** (self.dim - 1) * np.einsum("k,qk,cak->caq", self.qw, self.phi, self.grad)

    def stabilization(self, h, beta):
        """C_e[k, l] = -beta diam^2 (grad psi_k, grad psi_l), diam = sqrt(d) h (eq. 8)."""
        diam2 = self.dim * h * h
        return -beta * diam2 * h ** (self.dim - 2) * np.einsum("k,kab->ab", self.qw, self.G)

    def load(self, h, f_q):
        return h ** self.dim * np.einsum("...ck,k,ak->...ca", f_q, self.qw, self.phi)


def quad_positions(grid: GridQ1, ref: RefQ1, elems):
    e = np.asarray(elems, dtype=np.float64)
    return (e[:, None, :] + ref.qp[None, :, :]) * grid.h


def viscosity(grid: GridQ1, ref: RefQ1, elems, eta_out=1.0, eta_in=1.0, incl=None):
    """Viscosity at the 2^d Gauss points of each element (closed disc/ball rule)."""
    x = quad_positions(grid, ref, elems)
    eta = np.full(x.shape[:2], float(eta_out))
    if incl is not None and len(incl):
        inside = np.zeros(x.shape[:2], dtype=bool)
        for row in np.asarray(incl, dtype=np.float64):
            d2 = sum((x[..., d] - row[d]) ** 2 for d in range(grid.dim))
            inside |= d2 <= row[grid.dim] ** 2
        eta[inside] = float(eta_in)
    return eta


def element_dofs(grid: GridQ1, ref: RefQ1, elems):
    verts = np.asarray(elems)[:, None, :] + ref.nodes[None, :, :]
    vd = np.stack([grid.vel(c, verts) for c in range(grid.dim)], axis=1)   # (ne, d, 2^d)
    return vd, grid.pres(verts)


def assemble_matrix(grid: GridQ1, beta, eta_out=1.0, eta_in=1.0, incl=None, keep_masked=False):
    """Global L (CSR); masked rows/columns empty unless ``keep_masked``."""
    ref = RefQ1(grid.dim)
    elems = grid.elements()
    eta = viscosity(grid, ref, elems, eta_out, eta_in, incl)
    Ae = ref.stiffness(grid.h, eta)
    Be = ref.divergence(grid.h)
    Ce = ref.stabilization(grid.h, beta)
    vd, pd = element_dofs(grid, ref, elems)
    nb = Ae.shape[1]
    rows, cols, vals = [], [], []

    def add(r, c, v):
        rows.append(r.ravel()); cols.append(c.ravel()); vals.append(np.broadcast_to(v, r.shape).ravel())

    for c in range(grid.dim):
        add(np.repeat(vd[:, c, :, None], nb, 2), np.repeat(vd[:, c, None, :], nb, 1), Ae)
        rb = np.repeat(vd[:, c, :, None], nb, 2)
        cb = np.repeat(pd[:, None, :], nb, 1)
        add(rb, cb, Be[c][None])
        add(cb, rb, Be[c][None])
    add(np.repeat(pd[:, :, None], nb, 2), np.repeat(pd[:, None, :], nb, 1), Ce[None])
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    keep = np.ones(len(rows), bool) if keep_masked else grid.free[rows] & grid.free[cols]
    L = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(grid.n, grid.n)).tocsr()
    L.sum_duplicates()
    return L


def assemble_rhs(grid: GridQ1, params):
    """b = [(f, phi); 0] with the 2^d-point rule; masked rows zero."""
    ref = RefQ1(grid.dim)
    elems = grid.elements()
    f = mms.forcing(params, quad_positions(grid, ref, elems))          # (ne, nq, d)
    be = ref.load(grid.h, np.moveaxis(f, 2, 1))                        # (ne, d, 2^d)
    vd, _ = element_dofs(grid, ref, elems)
    b = np.zeros(grid.n)
    np.add.at(b, vd.ravel(), be.ravel())
    b[~grid.free] = 0.0
    return b


def lid_velocity(grid: GridQ1, U=1.0):
    """Driven-cavity data (Sec. 4.1): u_x = U on the top side's vertices strictly
    between the corners (the corners belong to the no-slip walls)."""
    assert grid.dim == 2
    u = np.zeros(grid.n)
    v = grid.vnode
    top = (v[:, 1] == grid.N) & (v[:, 0] > 0) & (v[:, 0] < grid.N)
    u[: grid.nV][top] = U
    u[grid.free] = 0.0
    return u


def dirichlet_lifting(grid: GridQ1, uD, beta, eta_out=1.0, eta_in=1.0, incl=None):
    """b = -L_all[free, masked] uD on free rows (L_all keeps the masked columns)."""
    L_all = assemble_matrix(grid, beta, eta_out, eta_in, incl, keep_masked=True)
    b = -(L_all @ np.where(grid.free, 0.0, uD))
    b[~grid.free] = 0.0
    return b


def prolongation(fine: GridQ1, coarse: GridQ1) -> sp.csr_matrix:
    """Interpolation of all d+1 fields from the coarse to the fine vertices."""
    assert fine.dim == coarse.dim and fine.N == 2 * coarse.N
    P1 = _kron_dims(interp_1d_q1(coarse.N), fine.dim)
    P = sp.block_diag([P1] * (fine.dim + 1), format="csr")
    P = (sp.diags(fine.free.astype(np.float64)) @ P @ sp.diags(coarse.free.astype(np.float64))).tocsr()
    P.eliminate_zeros()
    return P


class PatchSetQ1:
    """Vertex patches with the literal owned set (pressure + co-located velocity)."""

    def __init__(self, grid: GridQ1):
        self.grid = grid
        d = grid.dim
        self.count = grid.nV
        self.owner = np.concatenate([np.arange(grid.nV)] * (d + 1))
        self.owner[~grid.free] = -1
        self.dofs, self.owned = [], []
        for k in range(grid.nV):
            v = grid.vnode[k]
            lo, hi = np.maximum(v - 1, 0), np.minimum(v + 1, grid.N)
            ranges = [range(lo[i], hi[i] + 1) for i in range(d)]
            verts = np.asarray([p[::-1] for p in itertools.product(*ranges[::-1])], dtype=np.int64)
            parts = []
            for c in range(d):
                g = grid.vel(c, verts)
                parts.append(g[grid.free[g]])
            parts.append(np.array([grid.pres(v)]))
            I = np.concatenate(parts)
            self.dofs.append(I)
            self.owned.append(np.nonzero(self.owner[I] == k)[0])
        # MV order (eq. 11): ascending colour sum_d (k_d mod 4) 4^d, lexicographic
        # within a colour.  A patch writes x within one vertex of k and its residual
        # rows read x within two vertices of k, so patches of one colour (4 or
        # more vertices apart in some direction) never see each other's updates:
        # the sequential product in this order equals the colour-parallel form.
        colour = sum((grid.vnode[:, d] % 4) * 4 ** d for d in range(d))
        self.order = np.lexsort((np.arange(self.count), colour))
        self.colour = colour


class LevelQ1(mg.Level):
    def __init__(self, grid: GridQ1, beta, eta_out, eta_in, incl, smooth=True, L=None):
        self.grid = grid
        self.L = assemble_matrix(grid, beta, eta_out, eta_in, incl) if L is None else L
        self.free = grid.free
        self.kind = mg.VERTEX
        self.P = None
        if smooth:
            self.patches = PatchSetQ1(grid)
            self.lus = sm.factor(self.L, self.patches.dofs)
            self._W = None
        else:
            self.patches = None


class HierarchyQ1(mg.Hierarchy):
    """V-cycle hierarchy of the stabilized pair; smoothing, V-cycle and solve are
    those of the Taylor-Hood oracle (same eqs. 10-13 on a different L).
    coarse='rediscretised' assembles every level with its own h (Sec. 4);
    coarse='galerkin' takes L_{l-1} = P_l^T L_l P_l from the finest level down
    (a literal sparse triple product)."""

    def __init__(self, dim, n_cells, n_levels, dmask, beta, eta_out=1.0, eta_in=1.0, incl=None,
                 coarse="rediscretised"):
        if n_cells % (2 ** (n_levels - 1)):
            raise ValueError("n_cells must be divisible by 2^(n_levels-1)")
        if coarse not in ("rediscretised", "galerkin"):
            raise ValueError(coarse)
        self.dim = dim
        self.beta = beta
        Ns = [n_cells // 2 ** (n_levels - 1 - l) for l in range(n_levels)]
        grids = [GridQ1(dim, N, dmask) for N in Ns]
        Ps = [None] + [prolongation(grids[l], grids[l - 1]) for l in range(1, n_levels)]
        Ls = [None] * n_levels
        if coarse == "galerkin":
            Ls[-1] = assemble_matrix(grids[-1], beta, eta_out, eta_in, incl)
            for l in range(n_levels - 1, 0, -1):
                Ls[l - 1] = (Ps[l].T @ Ls[l] @ Ps[l]).tocsr()
        self.levels = [LevelQ1(grids[l], beta, eta_out, eta_in, incl, smooth=l > 0, L=Ls[l])
                       for l in range(n_levels)]
        for l in range(1, n_levels):
            self.levels[l].P = Ps[l]
        self._coarse_setup()


def nodal_error(grid: GridQ1, params, x):
    """Max velocity error at the vertices and the L2-like pressure error after
    mean removal, against the manufactured solution."""
    pts = grid.vnode * grid.h
    u = mms.velocity(params, pts)                  # (nV, d)
    p = mms.pressure(params, pts)
    d = grid.dim
    eu = max(np.abs(x[c * grid.nV:(c + 1) * grid.nV] - u[:, c]).max() for c in range(d))
    ph = x[d * grid.nV:]
    ep = np.sqrt(np.mean(((ph - ph.mean()) - (p - p.mean())) ** 2))
    return eu, ep


def matrix_row(grid: GridQ1, row: int, beta, eta_out=1.0, eta_in=1.0, incl=None):
    """One row of L as {column: value}, from the (at most 2^d) elements that
    touch the row's vertex; for single rows of grids too large to assemble."""
    if not grid.free[row]:
        return {}
    d = grid.dim
    f, vi = divmod(row, grid.nV)
    v = grid.vnode[vi]
    lo, hi = np.maximum(v - 1, 0), np.minimum(v, grid.N - 1)
    ranges = [np.arange(lo[i], hi[i] + 1) for i in range(d)]
    elems = np.stack([m.ravel() for m in np.meshgrid(*ranges, indexing="ij")], axis=1)
    ref = RefQ1(d)
    Ae = ref.stiffness(grid.h, viscosity(grid, ref, elems, eta_out, eta_in, incl))
    Be = ref.divergence(grid.h)
    Ce = ref.stabilization(grid.h, beta)
    vd, pd = element_dofs(grid, ref, elems)
    out = {}

    def add(col, val):
        if grid.free[col]:
            out[col] = out.get(col, 0.0) + val

    for ie in range(len(elems)):
        (loc,) = np.nonzero(pd[ie] == grid.pres(v))
        a = loc[0]
        for b in range(pd.shape[1]):
            if f < d:
                add(vd[ie, f, b], Ae[ie, a, b])
                add(pd[ie, b], Be[f, a, b])
            else:
                for c in range(d):
                    add(vd[ie, c, b], Be[c, b, a])
                add(pd[ie, b], Ce[a, b])
    return out
