"""Taylor-Hood Q2/Q1 reference-element quantities (Sec. 2, eqs. 5-7).

Velocity uses the tensor-product Lagrange quadratics (Q2), pressure the
tensor-product Lagrange linears (Q1).  Integrals use the tensor 3-point
Gauss-Legendre rule, which integrates every polynomial element integrand of
the Stokes bilinear forms exactly; with a viscosity that varies between
quadrature points the same rule *defines* the discrete form.

Local node numbering is lexicographic with x fastest: a = ix + 3*iy + 9*iz
for velocity, k = kx + 2*ky + 4*kz for pressure.
"""
from __future__ import annotations

import itertools

import numpy as np

GAUSS_T = np.array([0.5 - 0.5 * np.sqrt(0.6), 0.5, 0.5 + 0.5 * np.sqrt(0.6)])
GAUSS_W = np.array([5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0])


def q2_1d(t):
    """1D quadratic Lagrange basis on [0,1] with nodes 0, 1/2, 1; shape (3, len(t))."""
    t = np.asarray(t, dtype=np.float64)
    return np.stack([(1 - t) * (1 - 2 * t), 4 * t * (1 - t), t * (2 * t - 1)])


def dq2_1d(t):
    """Derivatives of :func:`q2_1d`."""
    t = np.asarray(t, dtype=np.float64)
    return np.stack([4 * t - 3, 4 - 8 * t, 4 * t - 1])


def q1_1d(t):
    """1D linear Lagrange basis on [0,1]; shape (2, len(t))."""
    t = np.asarray(t, dtype=np.float64)
    return np.stack([1 - t, t])


def quad_points(dim):
    """Tensor Gauss points (nq, dim) in lexicographic order (x fastest) and weights (nq,)."""
    pts, wts = [], []
    for idx in itertools.product(range(3), repeat=dim):
        idx = idx[::-1]  # idx[0] is x, the fastest index
        pts.append([GAUSS_T[i] for i in idx])
        wts.append(np.prod([GAUSS_W[i] for i in idx]))
    return np.asarray(pts), np.asarray(wts)


def local_nodes(dim, per_dim):
    """Local multi-indices (n, dim) in lexicographic order, x fastest."""
    out = []
    for idx in itertools.product(range(per_dim), repeat=dim):
        out.append(idx[::-1])
    return np.asarray(out, dtype=np.int64)


class RefElement:
    """Basis values and gradients at the Gauss points of [0,1]^dim."""

    def __init__(self, dim: int):
        self.dim = dim
        self.qp, self.qw = quad_points(dim)
        self.vnodes = local_nodes(dim, 3)   # (3^d, d)
        self.pnodes = local_nodes(dim, 2)   # (2^d, d)
        nq = len(self.qw)
        nv = len(self.vnodes)
        npn = len(self.pnodes)
        v1 = [q2_1d(self.qp[:, d]) for d in range(dim)]   # each (3, nq)
        g1 = [dq2_1d(self.qp[:, d]) for d in range(dim)]
        p1 = [q1_1d(self.qp[:, d]) for d in range(dim)]
        self.phi = np.ones((nv, nq))
        self.grad = np.ones((dim, nv, nq))
        for a, idx in enumerate(self.vnodes):
            for d in range(dim):
                self.phi[a] *= v1[d][idx[d]]
                for c in range(dim):
                    self.grad[c, a] *= (g1[d][idx[d]] if c == d else v1[d][idx[d]])
        self.psi = np.ones((npn, nq))
        for k, idx in enumerate(self.pnodes):
            for d in range(dim):
                self.psi[k] *= p1[d][idx[d]]
        # G[q, a, b] = grad phi_a(q) . grad phi_b(q)
        self.G = np.einsum("cak,cbk->kab", self.grad, self.grad)

    def stiffness(self, h, eta_q):
        """A_e[a, b] = int eta grad phi_a . grad phi_b over a cube of side h (eq. 7).

        ``eta_q`` has shape (..., nq): viscosity at each Gauss point.
        Returns (..., 3^d, 3^d).
        """
        wq = np.asarray(eta_q) * self.qw
        return h ** (self.dim - 2) * np.einsum("...k,kab->...ab", wq, self.G)

    def divergence(self, h):
        """B_e[c, a, k] = -int psi_k d(phi_a)/dx_c over a cube of side h (eq. 7)."""
        return -h ** (self.dim - 1) * np.einsum("k,qk,cak->caq", self.qw, self.psi, self.grad)

    def load(self, h, f_q):
        """b_e[c, a] = int f_c phi_a with ``f_q`` of shape (..., dim, nq)."""
        return h ** self.dim * np.einsum("...ck,k,ak->...ca", f_q, self.qw, self.phi)
