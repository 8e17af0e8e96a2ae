"""Learned per-patch damping (extension of the diagonal weighting omega_i of
eq. 11, restricted to one scalar per patch; the network itself is not in the
paper).

Features of vertex patch k on a grid of N cells (h = 1/N), 16 per patch:
  f_0..f_8   log10(eta / eta_out) / 4 at the points (k + (a, b)/2) h,
             a, b in {-1, 0, 1} (b slow), clamped to [0, 1]^2;
  f_9, f_10, f_11  min, max, mean of f_0..f_8;
  f_12, f_13       1 if k_x (resp. k_y) lies on the boundary, else 0;
  f_14             log2(N) / 10;   f_15 = 1.
Network: z1 = W1 f + b1, h1 = relu(z1); z2 = W2 h1 + b2, h2 = relu(z2);
z3 = w3 . h2 + b3; omega = 0.2 + sigmoid(z3).  Parameters flat in the order
W1, b1, W2, b2, w3, b3 (``rav_inputs.MLP_SIZES``).

Training loss of one problem: the residual reduction of one exact two-grid
cycle from an initial error x0 (b = 0):
  nu RAV sweeps with the per-patch omega (eq. 13),
  x += P L_c^{-1} P^T (b - L x)       (exact coarse solve),
  nu RAV sweeps,
  loss = ||L x_out||^2 / ||L x0||^2.
Its gradient with respect to every omega_i is obtained by the reverse sweep
(adjoint) of these linear steps, and with respect to the parameters by
back-propagation through the network.  Parity: pinned against central
finite differences (tests/test_oracle_learned.py).
"""
from __future__ import annotations

import numpy as np

from . import smoothers as sm
from .assemble import viscosity  # noqa: F401  (same inclusion rule, used below)
from .grid import Grid
from .patches import VERTEX, patch_anchor

SIZES = ((64, 16), (64,), (64, 64), (64,), (64,), (1,))


def eta_at(points, eta_out, eta_in, incl):
    """Viscosity at arbitrary points (n, d): closed-disc inclusion rule."""
    eta = np.full(len(points), float(eta_out))
    if incl is not None and len(incl):
        inside = np.zeros(len(points), dtype=bool)
        d = points.shape[1]
        for row in np.asarray(incl, dtype=np.float64):
            d2 = np.zeros(len(points))
            for c in range(d):
                dd = points[:, c] - row[c]
                d2 = d2 + dd * dd
            inside |= d2 <= row[d] * row[d]
        eta[inside] = float(eta_in)
    return eta


def features(grid: Grid, eta_out=1.0, eta_in=1.0, incl=None):
    """(n_patches, 16) features of the 2D vertex patches of ``grid``."""
    assert grid.dim == 2
    N = grid.N
    h = grid.h
    npt = grid.nP
    F = np.zeros((npt, 16))
    for p in range(npt):
        k = patch_anchor(grid, VERTEX, p)
        pts = []
        for b in (-1, 0, 1):
            for a in (-1, 0, 1):
                x = min(max((k[0] + 0.5 * a) * h, 0.0), 1.0)
                y = min(max((k[1] + 0.5 * b) * h, 0.0), 1.0)
                pts.append((x, y))
        e = eta_at(np.asarray(pts), eta_out, eta_in, incl)
        f = np.log10(e / eta_out) / 4.0
        F[p, :9] = f
        F[p, 9], F[p, 10], F[p, 11] = f.min(), f.max(), f.mean()
        F[p, 12] = 1.0 if k[0] in (0, N) else 0.0
        F[p, 13] = 1.0 if k[1] in (0, N) else 0.0
        F[p, 14] = np.log2(N) / 10.0
        F[p, 15] = 1.0
    return F


def unpack(theta):
    out, off = [], 0
    theta = np.asarray(theta, dtype=np.float64)
    for s in SIZES:
        n = int(np.prod(s))
        out.append(theta[off:off + n].reshape(s))
        off += n
    return out


def mlp_forward(theta, F):
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    z1 = F @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ w3 + b3[0]
    sig = 1.0 / (1.0 + np.exp(-z3))
    omega = 0.2 + sig
    return omega, (F, z1, h1, z2, h2, sig)


def mlp_backward(theta, cache, g_omega):
    """Gradient of sum_i g_omega[i] * omega_i with respect to theta."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    F, z1, h1, z2, h2, sig = cache
    d3 = g_omega * sig * (1.0 - sig)
    gw3 = h2.T @ d3
    gb3 = np.array([d3.sum()])
    d2 = np.outer(d3, w3) * (z2 > 0)
    gW2 = d2.T @ h1
    gb2 = d2.sum(0)
    d1 = (d2 @ W2) * (z1 > 0)
    gW1 = d1.T @ F
    gb1 = d1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, gb3])


class TwoGrid:
    """Exact two-grid cycle of a 2-level ``mg.Hierarchy`` with per-patch omega."""

    def __init__(self, H, nu=2):
        assert len(H.levels) == 2
        self.H = H
        self.nu = nu
        self.lv = H.levels[1]
        self.W = self.lv.W()
        self.ps = self.lv.patches

    def _sweep(self, x, omega):
        lv, ps = self.lv, self.ps
        return sm.rav_sweep_rows(lv.L, lv.free, ps.dofs, ps.owned, self.W, omega, x, np.zeros_like(x))

    def _coarse(self, x):
        lv = self.lv
        r = sm.residual(lv.L, x, np.zeros_like(x), lv.free)
        return x + lv.P @ self.H.coarse_solve(lv.P.T @ r)

    def forward(self, omega, x0):
        """States before every sweep and after the coarse correction."""
        states = [x0.copy()]
        x = x0.copy()
        for _ in range(self.nu):
            x = self._sweep(x, omega)
            states.append(x.copy())
        x = self._coarse(x)
        states.append(x.copy())
        for _ in range(self.nu):
            x = self._sweep(x, omega)
            states.append(x.copy())
        return states

    def loss(self, omega, x0):
        lv = self.lv
        L, free = lv.L, lv.free
        xo = self.forward(omega, x0)[-1]
        num = np.sum(sm.residual(L, xo, np.zeros_like(xo), free) ** 2)
        den = np.sum(sm.residual(L, x0, np.zeros_like(x0), free) ** 2)
        return num / den

    def _sweep_adjoint(self, lam, x_pre, omega):
        """Adjoint of x' = x + S_w (-L x): returns (lam_pre, d loss / d omega)."""
        lv, ps = self.lv, self.ps
        L, free = lv.L, lv.free
        r = sm.residual(L, x_pre, np.zeros_like(x_pre), free)
        g = np.zeros(ps.count)
        z = np.zeros_like(lam)
        for i, (I, own, W) in enumerate(zip(ps.dofs, ps.owned, self.W)):
            lo = lam[I[own]]
            g[i] = lo @ (W @ r[I])
            w = float(omega[i]) if np.ndim(omega) else float(omega)
            z[I] += W.T @ (w * lo)
        z[~free] = 0.0
        lam_pre = lam - L @ z
        lam_pre[~free] = 0.0
        return lam_pre, g

    def _coarse_adjoint(self, lam):
        lv = self.lv
        L, free = lv.L, lv.free
        z = lv.P @ self.H.coarse_solve(lv.P.T @ lam)
        out = lam - L @ z
        out[~free] = 0.0
        return out

    def loss_and_grad(self, omega, x0):
        """Loss and its gradient with respect to the per-patch omega."""
        lv = self.lv
        L, free = lv.L, lv.free
        states = self.forward(omega, x0)
        xo = states[-1]
        den = np.sum(sm.residual(L, x0, np.zeros_like(x0), free) ** 2)
        Lx = L @ xo
        Lx[~free] = 0.0
        num = np.sum(Lx ** 2)
        lam = 2.0 * (L @ Lx) / den
        lam[~free] = 0.0
        g = np.zeros(self.ps.count)
        nu = self.nu
        for s in range(2 * nu + 1, nu + 1, -1):
            lam, gs = self._sweep_adjoint(lam, states[s - 1], omega)
            g += gs
        lam = self._coarse_adjoint(lam)
        for s in range(nu, 0, -1):
            lam, gs = self._sweep_adjoint(lam, states[s - 1], omega)
            g += gs
        return num / den, g
