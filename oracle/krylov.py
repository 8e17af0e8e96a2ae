"""Restarted flexible GMRES with right preconditioning (Krylov acceleration of
the multigrid cycle; Sec. 4 mentions multigrid as a Krylov preconditioner).

Plain Arnoldi with modified Gram-Schmidt and Givens rotations; the
preconditioner is any linear map (one V-cycle from a zero guess).  GMRES
minimises the residual over the Krylov space, so its iterates are unique:
pinned against scipy's GMRES in tests/test_oracle_krylov.py.
"""
from __future__ import annotations

import numpy as np


def fgmres(apply_L, apply_M, b, x0=None, rtol=1e-8, restart=30, maxit=300):
    """Returns (x, number of preconditioner applications, residual history)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_L(x)
    beta0 = np.linalg.norm(r)
    hist = [beta0]
    total = 0
    if beta0 == 0.0:
        return x, 0, hist
    while total < maxit:
        r = b - apply_L(x)
        beta = np.linalg.norm(r)
        if beta <= rtol * beta0:
            break
        m = restart
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        g = np.zeros(m + 1)
        g[0] = beta
        cs, sn = np.zeros(m), np.zeros(m)
        jend = 0
        for j in range(m):
            if total >= maxit:
                break
            z = apply_M(V[j])
            Z.append(z)
            w = apply_L(z)
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] != 0 else w)
            total += 1
            for i in range(j):
                a, c = H[i, j], H[i + 1, j]
                H[i, j], H[i + 1, j] = cs[i] * a + sn[i] * c, -sn[i] * a + cs[i] * c
            rr = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = (H[j, j] / rr, H[j + 1, j] / rr) if rr > 0 else (1.0, 0.0)
            H[j, j], H[j + 1, j] = rr, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            jend = j + 1
            hist.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= rtol * beta0:
                break
        y = np.zeros(jend)
        for i in range(jend - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:jend] @ y[i + 1:jend]) / H[i, i]
        for i in range(jend):
            x = x + y[i] * Z[i]
        if hist[-1] <= rtol * beta0 and np.linalg.norm(b - apply_L(x)) <= rtol * beta0:
            break
    return x, total, hist
