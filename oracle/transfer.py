"""Nested-space interpolation between uniform levels (Sec. 2, Fig. 1).

The coarse grid of size N/2 and the fine grid of size N give nested Q2/Q1
spaces.  P maps coarse nodal values to the fine nodal values of the same
finite-element function, so each column of P is a coarse basis function
evaluated at the fine nodes.  It is built per dimension by evaluating the 1D
coarse Lagrange bases at the fine node positions and tensorised; restriction
is P^T (variational).  Rows of masked fine DoFs and columns of masked coarse
DoFs are zero.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import q1_1d, q2_1d
from .grid import Grid


def interp_1d_q2(n_coarse: int) -> np.ndarray:
    """(2*nf+1, 2*nc+1) values of the coarse 1D Q2 basis at fine half-grid nodes."""
    nf = 2 * n_coarse
    P = np.zeros((2 * nf + 1, 2 * n_coarse + 1))
    for E in range(n_coarse):
        fine = np.arange(4 * E, 4 * E + 5)          # fine nodes inside coarse element E
        t = (fine - 4 * E) / 4.0
        vals = q2_1d(t)                              # (3, 5)
        for i in range(3):
            P[fine, 2 * E + i] = vals[i]
    return P


def interp_1d_q1(n_coarse: int) -> np.ndarray:
    """(nf+1, nc+1) values of the coarse 1D Q1 basis at fine vertices."""
    nf = 2 * n_coarse
    P = np.zeros((nf + 1, n_coarse + 1))
    for E in range(n_coarse):
        fine = np.arange(2 * E, 2 * E + 3)
        t = (fine - 2 * E) / 2.0
        vals = q1_1d(t)
        for i in range(2):
            P[fine, E + i] = vals[i]
    return P


def _kron_dims(P1, dim):
    """Tensor product for lexicographic (x fastest) numbering."""
    out = sp.csr_matrix(P1)
    for _ in range(dim - 1):
        out = sp.kron(sp.csr_matrix(P1), out, format="csr")
    return out


def prolongation(fine: Grid, coarse: Grid) -> sp.csr_matrix:
    """P (fine.n x coarse.n)."""
    assert fine.dim == coarse.dim and fine.N == 2 * coarse.N
    d = fine.dim
    Pv = _kron_dims(interp_1d_q2(coarse.N), d)
    Pp = _kron_dims(interp_1d_q1(coarse.N), d)
    P = sp.block_diag([Pv] * d + [Pp], format="csr")
    P.eliminate_zeros()
    Dr = sp.diags(fine.free.astype(np.float64))
    Dc = sp.diags(coarse.free.astype(np.float64))
    P = (Dr @ P @ Dc).tocsr()
    P.eliminate_zeros()
    return P
