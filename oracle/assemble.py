"""Global Stokes block system and right-hand side (Sec. 2, eqs. 5-8).

L = [[A, B], [B^T, C]] with A = (eta grad v, grad u) applied to each velocity
component (no cross-component block), B = -(div v, p) and C = 0, the choice
the paper states for an inf-sup stable conforming pair such as Q2/Q1.
Rows and columns of masked (Dirichlet) velocity DoFs are dropped: they stay in
the full-length numbering as all-zero rows/columns.

Viscosity is evaluated at each Gauss point: ``eta_in`` inside any inclusion
(closed disc/ball (x-c).(x-c) <= r^2) and ``eta_out`` elsewhere.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import mms
from .fem import RefElement
from .grid import Grid


def quad_positions(grid: Grid, ref: RefElement, elems):
    """Physical Gauss-point coordinates (ne, nq, d): x = (e + t_q) * h."""
    e = np.asarray(elems, dtype=np.float64)
    return (e[:, None, :] + ref.qp[None, :, :]) * grid.h


def viscosity(grid: Grid, ref: RefElement, elems, eta_out=1.0, eta_in=1.0, incl=None):
    """Viscosity at the Gauss points of the given elements, shape (ne, nq)."""
    x = quad_positions(grid, ref, elems)
    eta = np.full(x.shape[:2], float(eta_out))
    if incl is not None and len(incl):
        inside = np.zeros(x.shape[:2], dtype=bool)
        for row in np.asarray(incl, dtype=np.float64):
            d2 = np.zeros(x.shape[:2])
            for d in range(grid.dim):
                dd = x[..., d] - row[d]
                d2 = d2 + dd * dd
            rad = row[grid.dim]
            inside |= d2 <= rad * rad
        eta[inside] = float(eta_in)
    return eta


def element_dofs(grid: Grid, ref: RefElement, elems):
    """Global velocity DoFs (ne, d, 3^d) and pressure DoFs (ne, 2^d) of each element."""
    elems = np.asarray(elems)
    vnode = 2 * elems[:, None, :] + ref.vnodes[None, :, :]
    vdofs = np.stack([grid.vel(c, vnode) for c in range(grid.dim)], axis=1)
    pnode = elems[:, None, :] + ref.pnodes[None, :, :]
    return vdofs, grid.pres(pnode)


def assemble_matrix(grid: Grid, eta_out=1.0, eta_in=1.0, incl=None):
    """Global L (CSR, n x n) on the free DoFs, masked rows/columns empty."""
    ref = RefElement(grid.dim)
    elems = grid.elements()
    eta = viscosity(grid, ref, elems, eta_out, eta_in, incl)
    Ae = ref.stiffness(grid.h, eta)                 # (ne, nv, nv)
    Be = ref.divergence(grid.h)                     # (d, nv, np)
    vd, pd = element_dofs(grid, ref, elems)          # (ne, d, nv), (ne, np)
    rows, cols, vals = [], [], []
    nv = Ae.shape[1]
    for c in range(grid.dim):
        r = np.repeat(vd[:, c, :, None], nv, axis=2)
        cc = np.repeat(vd[:, c, None, :], nv, axis=1)
        rows.append(r.ravel()); cols.append(cc.ravel()); vals.append(Ae.ravel())
        npn = pd.shape[1]
        rb = np.repeat(vd[:, c, :, None], npn, axis=2)
        cb = np.repeat(pd[:, None, :], nv, axis=1)
        vb = np.broadcast_to(Be[c][None], rb.shape)
        rows.append(rb.ravel()); cols.append(cb.ravel()); vals.append(vb.ravel())
        rows.append(cb.ravel()); cols.append(rb.ravel()); vals.append(vb.ravel())
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    keep = grid.free[rows] & grid.free[cols]
    L = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(grid.n, grid.n)).tocsr()
    L.sum_duplicates()
    return L


def assemble_rhs(grid: Grid, params):
    """b = [(f, phi); 0] with 3^d Gauss on every element; masked rows zero."""
    ref = RefElement(grid.dim)
    elems = grid.elements()
    x = quad_positions(grid, ref, elems)             # (ne, nq, d)
    f = mms.forcing(params, x)                       # (ne, nq, d)
    be = ref.load(grid.h, np.moveaxis(f, 2, 1))      # (ne, d, nv)
    vd, _ = element_dofs(grid, ref, elems)
    b = np.zeros(grid.n)
    np.add.at(b, vd.ravel(), be.ravel())
    b[~grid.free] = 0.0
    return b


def matrix_row(grid: Grid, row: int, eta_out=1.0, eta_in=1.0, incl=None):
    """One row of L as a dict {column: value}, assembled from the elements that
    touch the row's node.  Used to check single outputs of large grids."""
    ref = RefElement(grid.dim)
    d = grid.dim
    out = {}
    if not grid.free[row]:
        return out
    if row < d * grid.nV:
        c = row // grid.nV
        a = grid.vnode[row % grid.nV]
        lo = np.maximum((a - 1) // 2, 0)
        hi = np.minimum(a // 2, grid.N - 1)
    else:
        k = grid.pnode[row - d * grid.nV]
        lo = np.maximum(k - 1, 0)
        hi = np.minimum(k, grid.N - 1)
    ranges = [np.arange(lo[i], hi[i] + 1) for i in range(d)]
    mesh = np.meshgrid(*ranges, indexing="ij")
    elems = np.stack([m.ravel() for m in mesh], axis=1)
    eta = viscosity(grid, ref, elems, eta_out, eta_in, incl)
    Ae = ref.stiffness(grid.h, eta)
    Be = ref.divergence(grid.h)
    vd, pd = element_dofs(grid, ref, elems)
    for ie in range(len(elems)):
        if row < d * grid.nV:
            (loc,) = np.nonzero(vd[ie, c] == row)
            if len(loc) == 0:
                continue
            la = loc[0]
            for lb in range(vd.shape[2]):
                col = vd[ie, c, lb]
                if grid.free[col]:
                    out[col] = out.get(col, 0.0) + Ae[ie, la, lb]
            for lk in range(pd.shape[1]):
                col = pd[ie, lk]
                out[col] = out.get(col, 0.0) + Be[c, la, lk]
        else:
            (loc,) = np.nonzero(pd[ie] == row)
            if len(loc) == 0:
                continue
            lk = loc[0]
            for cc in range(d):
                for la in range(vd.shape[2]):
                    col = vd[ie, cc, la]
                    if grid.free[col]:
                        out[col] = out.get(col, 0.0) + Be[cc, la, lk]
    return out


def lid_velocity(grid: Grid, U=1.0):
    """Dirichlet data of the driven cavity (Sec. 4.1): horizontal velocity U on
    the top side's nodes strictly between the corners, zero elsewhere (the
    corners belong to the no-slip walls, so the data has no normal flux).
    Full-length vector, nonzero only on masked DoFs."""
    assert grid.dim == 2
    u = np.zeros(grid.n)
    a = grid.vnode
    top = (a[:, 1] == 2 * grid.N) & (a[:, 0] > 0) & (a[:, 0] < 2 * grid.N)
    u[: grid.nV][top] = U
    u[grid.free] = 0.0   # only masked (Dirichlet) entries carry data
    return u


def dirichlet_lifting(grid: Grid, uD, eta_out=1.0, eta_in=1.0, incl=None):
    """Right-hand side contribution of nonhomogeneous Dirichlet data uD (values
    on masked DoFs): b = -L_all[free, masked] uD on free rows, zero on masked
    rows, where L_all is the operator assembled with no DoF masked (eq. 6 with
    the Dirichlet columns kept)."""
    open_grid = Grid(grid.dim, grid.N, 0)
    L_all = assemble_matrix(open_grid, eta_out, eta_in, incl)
    ud = np.where(grid.free, 0.0, uD)
    b = -(L_all @ ud)
    b[~grid.free] = 0.0
    return b
