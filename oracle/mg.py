"""Geometric multigrid V-cycle with Vanka smoothing (Sec. 2, Fig. 1; Sec. 4).

Levels 0 (coarsest) .. L-1 (finest), N_l = N / 2^(L-1-l).  Every level is
rediscretised (Sec. 4 assembles the system anew on every grid).
V(nu, nu): nu smoothing sweeps, restrict the residual with P^T, recurse from a
zero coarse iterate, add the prolongated correction, nu smoothing sweeps.
The coarsest level is solved directly by LU (Sec. 2).

With Dirichlet velocity on the whole boundary the pressure is determined only
up to a constant: L has the null vector (0, 1_p).  The coarse solve then uses
the bordered system [[L_0, e], [e^T, 0]] with e = (0, 1_p), which returns the
zero-mean-pressure solution of a consistent system.  Masked rows are identity
rows in the coarse matrix.

The solve starts from x_0 = 0 and stops when ||r_k||_2 <= rtol ||r_0||_2
(Sec. 4: reduction of the initial residual by 10^8); the average reduction
factor is (||r_k|| / ||r_0||)^(1/k).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import smoothers as sm
from .assemble import assemble_matrix
from .grid import Grid
from .patches import PatchSet, VERTEX
from .transfer import prolongation

RAV, AV, MV = "rav", "av", "mv"


class Level:
    def __init__(self, dim, N, dmask, kind, eta_out, eta_in, incl, smooth=True, L=None):
        self.grid = Grid(dim, N, dmask)
        self.L = assemble_matrix(self.grid, eta_out, eta_in, incl) if L is None else L
        self.free = self.grid.free
        self.kind = kind
        self.P = None
        if smooth:
            self.patches = PatchSet(self.grid, kind)
            self.lus = sm.factor(self.L, self.patches.dofs)
            self._W = None
        else:
            self.patches = None

    def W(self):
        """Owned rows of every local inverse (computed on first use)."""
        if self._W is None:
            self._W = [sm.owned_rows(lu, own, len(I))
                       for lu, own, I in zip(self.lus, self.patches.owned, self.patches.dofs)]
        return self._W


class Hierarchy:
    """coarse='rediscretised' assembles every level (Sec. 4); coarse='galerkin'
    takes L_{l-1} = P_l^T L_l P_l from the finest level down (the variational
    coarse operator, here only as a literal sparse triple product)."""

    def __init__(self, dim, n_cells, n_levels, dmask, kind=VERTEX,
                 eta_out=1.0, eta_in=1.0, incl=None, coarse="rediscretised"):
        if n_cells % (2 ** (n_levels - 1)):
            raise ValueError("n_cells must be divisible by 2^(n_levels-1)")
        if coarse not in ("rediscretised", "galerkin"):
            raise ValueError(coarse)
        self.dim = dim
        Ns = [n_cells // 2 ** (n_levels - 1 - l) for l in range(n_levels)]
        grids = [Grid(dim, N, dmask) for N in Ns]
        Ps = [None] + [prolongation(grids[l], grids[l - 1]) for l in range(1, n_levels)]
        Ls = [None] * n_levels
        if coarse == "galerkin":
            Ls[-1] = assemble_matrix(grids[-1], eta_out, eta_in, incl)
            for l in range(n_levels - 1, 0, -1):
                Ls[l - 1] = (Ps[l].T @ Ls[l] @ Ps[l]).tocsr()
        self.levels = []
        for l in range(n_levels):
            self.levels.append(Level(dim, Ns[l], dmask, kind, eta_out, eta_in, incl, smooth=l > 0, L=Ls[l]))
        for l in range(1, n_levels):
            self.levels[l].P = Ps[l]
        self._coarse_setup()

    @property
    def finest(self):
        return self.levels[-1]

    def _coarse_setup(self):
        lv = self.levels[0]
        g = lv.grid
        M = lv.L.toarray()
        M[~g.free, ~g.free] = 1.0
        self.bordered = g.all_dirichlet
        if self.bordered:
            e = np.zeros(g.n)
            e[g.pressure_slice()] = 1.0
            M = np.block([[M, e[:, None]], [e[None, :], np.zeros((1, 1))]])
        self.coarse_lu = sla.lu_factor(M)

    def coarse_solve(self, b):
        g = self.levels[0].grid
        rhs = b.copy()
        rhs[~g.free] = 0.0
        if self.bordered:
            rhs = np.concatenate([rhs, [0.0]])
        x = sla.lu_solve(self.coarse_lu, rhs)
        return x[:g.n]

    # --- smoothing ---------------------------------------------------------
    def smooth(self, l, x, b, smoother, omega, sweeps, precision="fp64"):
        lv = self.levels[l]
        ps = lv.patches
        for _ in range(sweeps):
            if smoother == RAV:
                if precision == "fp64":
                    x = sm.rav_sweep(lv.L, lv.free, ps.dofs, ps.owned, lv.lus, omega, x, b)
                else:
                    Wl = [sm.round_storage(W, precision) for W in lv.W()]
                    x = sm.rav_sweep_rows_lowp(lv.L, lv.free, ps.dofs, ps.owned, Wl, omega, x, b)
            elif smoother == AV:
                x = sm.av_sweep(lv.L, lv.free, ps.dofs, lv.lus, omega, x, b)
            elif smoother == MV:
                x = sm.mv_sweep(lv.L, lv.free, ps.dofs, lv.lus, omega, ps.order, x, b)
            else:
                raise ValueError(smoother)
        return x

    def vcycle(self, x, b, smoother=RAV, omega=0.66, nu=2, l=None, precision="fp64"):
        """One V(nu, nu) cycle on level l (default finest); returns the new x."""
        if l is None:
            l = len(self.levels) - 1
        if l == 0:
            return self.coarse_solve(b)
        lv = self.levels[l]
        om = omega[l] if isinstance(omega, dict) else omega
        x = self.smooth(l, x, b, smoother, om, nu, precision)
        r = sm.residual(lv.L, x, b, lv.free)
        bc = lv.P.T @ r
        xc = np.zeros(self.levels[l - 1].grid.n)
        xc = self.vcycle(xc, bc, smoother, omega, nu, l - 1, precision)
        x = x + lv.P @ xc
        x = self.smooth(l, x, b, smoother, om, nu, precision)
        return x

    def solve(self, b, rtol=1e-8, maxit=200, smoother=RAV, omega=0.66, nu=2,
              x0=None, precision="fp64", diverge=1e3):
        """V-cycles from x0 (default 0) until ||r|| <= rtol ||r_0||.

        Returns (x, iterations, history of ||r_k||, status) with status one of
        'converged', 'maxit', 'diverged'."""
        lv = self.finest
        x = np.zeros(lv.grid.n) if x0 is None else x0.copy()
        r0 = np.linalg.norm(sm.residual(lv.L, x, b, lv.free))
        hist = [r0]
        if r0 == 0.0:
            return x, 0, hist, "converged"
        for k in range(1, maxit + 1):
            x = self.vcycle(x, b, smoother, omega, nu, precision=precision)
            rk = np.linalg.norm(sm.residual(lv.L, x, b, lv.free))
            hist.append(rk)
            if not np.isfinite(rk) or rk > diverge * r0:
                return x, k, hist, "diverged"
            if rk <= rtol * r0:
                return x, k, hist, "converged"
        return x, maxit, hist, "maxit"


def avg_reduction(hist):
    """Average reduction factor (||r_k|| / ||r_0||)^(1/k)."""
    k = len(hist) - 1
    return (hist[-1] / hist[0]) ** (1.0 / k) if k > 0 else 0.0


def zero_mean_pressure(grid, x):
    """Subtract the arithmetic mean of the pressure DoFs (comparison normal form)."""
    y = x.copy()
    s = grid.pressure_slice()
    y[s] -= y[s].mean()
    return y


def rel_l2(grid, a, b):
    """Relative L2 difference over free DoFs after pressure normalisation."""
    a = zero_mean_pressure(grid, a)[grid.free]
    b = zero_mean_pressure(grid, b)[grid.free]
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def dense_smoother_operator(L, free, dofs_list, owned_list, lus, omega, smoother, order=None):
    """Brute-force dense error propagation M with x_new = M x for b = 0
    (RAV: I - S_RAV L with S_RAV = sum_i Rt_i^T w L_i^{-1} R_i, eq. 13;
    AV: the same with R_i, eq. 12; MV: prod_i (I - R_i^T w L_i^{-1} R_i L), eq. 11).
    Only for tiny grids."""
    n = L.shape[0]
    Ld = L.toarray()
    I_n = np.eye(n)
    if smoother in (RAV, AV):
        S = np.zeros((n, n))
        for i, (I, lu) in enumerate(zip(dofs_list, lus)):
            Li_inv = np.linalg.inv(Ld[np.ix_(I, I)])
            w = float(omega[i]) if np.ndim(omega) else float(omega)
            rows = I[owned_list[i]] if smoother == RAV else I
            lrows = owned_list[i] if smoother == RAV else np.arange(len(I))
            S[np.ix_(rows, I)] += w * Li_inv[lrows, :]
        M = I_n - S @ Ld
    else:
        M = I_n.copy()
        for i in order:
            I = dofs_list[i]
            Li_inv = np.linalg.inv(Ld[np.ix_(I, I)])
            w = float(omega[i]) if np.ndim(omega) else float(omega)
            Ei = I_n.copy()
            Ei[np.ix_(I, np.arange(n))] -= w * Li_inv @ Ld[I, :]
            M = Ei @ M
    M[~free, :] = 0.0
    M[:, ~free] = 0.0
    return M
