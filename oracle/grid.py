"""Uniform-grid DoF numbering for Taylor-Hood Q2/Q1 on [0,1]^d (eq. 6 ordering).

The global vector is [u_1; ...; u_d; p] as in eq. (6):
* velocity component c at half-grid node a in [0, 2N]^d has index
  c*nV + sum_d a_d (2N+1)^d  (x fastest), nV = (2N+1)^d;
* pressure at vertex k in [0, N]^d has index d*nV + sum_d k_d (N+1)^d.

Velocity nodes on a Dirichlet side (eq. 2, Gamma_D) are masked: they carry
x = 0 and a residual of 0.  Side bit 2*d is x_d = 0, bit 2*d+1 is x_d = 1.
"""
from __future__ import annotations

import numpy as np


class Grid:
    def __init__(self, dim: int, n_cells: int, dmask: int):
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        self.dim = dim
        self.N = n_cells
        self.dmask = dmask
        self.h = 1.0 / n_cells
        self.nn = 2 * n_cells + 1
        self.np1 = n_cells + 1
        self.nV = self.nn ** dim
        self.nP = self.np1 ** dim
        self.n = dim * self.nV + self.nP
        self.all_dirichlet = all((dmask >> b) & 1 for b in range(2 * dim))
        # Velocity node coordinates (nV, d), x fastest.
        self.vnode = np.stack(np.unravel_index(np.arange(self.nV), (self.nn,) * dim)[::-1], axis=1)
        self.pnode = np.stack(np.unravel_index(np.arange(self.nP), (self.np1,) * dim)[::-1], axis=1)
        dir_node = np.zeros(self.nV, dtype=bool)
        for d in range(dim):
            if (dmask >> (2 * d)) & 1:
                dir_node |= self.vnode[:, d] == 0
            if (dmask >> (2 * d + 1)) & 1:
                dir_node |= self.vnode[:, d] == 2 * n_cells
        self.dirichlet_node = dir_node
        self.free = np.ones(self.n, dtype=bool)
        for c in range(dim):
            self.free[c * self.nV:(c + 1) * self.nV] = ~dir_node

    def vel(self, c, a):
        """Global index of velocity component c at node(s) a (..., d)."""
        a = np.asarray(a)
        idx = np.zeros(a.shape[:-1], dtype=np.int64)
        stride = 1
        for d in range(self.dim):
            idx = idx + a[..., d] * stride
            stride *= self.nn
        return c * self.nV + idx

    def pres(self, k):
        """Global index of the pressure at vertex/vertices k (..., d)."""
        k = np.asarray(k)
        idx = np.zeros(k.shape[:-1], dtype=np.int64)
        stride = 1
        for d in range(self.dim):
            idx = idx + k[..., d] * stride
            stride *= self.np1
        return self.dim * self.nV + idx

    def elements(self):
        """Element multi-indices (N^d, d), lexicographic with x fastest."""
        return np.stack(np.unravel_index(np.arange(self.N ** self.dim), (self.N,) * self.dim)[::-1], axis=1)

    def pressure_slice(self):
        return slice(self.dim * self.nV, self.n)
