"""Vanka smoothers as fixed-point iterations x <- x + S (b - L x) (Sec. 3, eq. 10).

* MV  (eq. 11): patches one after another in the canonical order; the
  residual on the patch rows is recomputed before each local solve (eq. 15).
* AV  (eq. 12): every patch solves with the same residual; corrections of all
  patch rows are summed.
* RAV (eq. 13): as AV, but a patch only writes the rows it owns.

Local solves use scipy's LU with partial pivoting of L_i = L[I_i, I_i].
``omega`` is a scalar or one weight per patch (the diagonal weighting of
eq. 11 restricted to a per-patch scalar).  The ``*_rows`` variants apply the
precomputed owned rows W_i of L_i^{-1} instead (Sec. 4.3: only those rows
need to be stored), optionally rounded to float32/bfloat16 and accumulated
in float32.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def residual(L, x, b, free):
    """r = b - L x on free rows, 0 on masked rows (eq. 10)."""
    r = b - L @ x
    r[~free] = 0.0
    return r


def local_matrix(L, dofs):
    """L_i = R_i L R_i^T, the principal submatrix on the patch DoFs (Sec. 3)."""
    return L[dofs][:, dofs].toarray()


def factor(L, dofs_list):
    return [sla.lu_factor(local_matrix(L, I)) for I in dofs_list]


def owned_rows(lu, owned, n):
    """W_i = rows ``owned`` of L_i^{-1}, from L_i^T Z = E_owned (Sec. 4.3)."""
    E = np.zeros((n, len(owned)))
    E[owned, np.arange(len(owned))] = 1.0
    Z = sla.lu_solve(lu, E, trans=1)
    return Z.T.copy()


def full_inverse(lu, n):
    return sla.lu_solve(lu, np.eye(n))


def _omega(omega, i):
    return float(omega[i]) if np.ndim(omega) else float(omega)


def rav_sweep(L, free, dofs_list, owned_list, lus, omega, x, b):
    """One RAV sweep (eq. 13): all patch solves from one residual, owned rows updated."""
    r = residual(L, x, b, free)
    dx = np.zeros_like(x)
    for i, (I, own, lu) in enumerate(zip(dofs_list, owned_list, lus)):
        y = sla.lu_solve(lu, r[I])
        dx[I[own]] += _omega(omega, i) * y[own]
    return x + dx


def av_sweep(L, free, dofs_list, lus, omega, x, b):
    """One AV sweep (eq. 12): all patch corrections summed over all patch rows."""
    r = residual(L, x, b, free)
    dx = np.zeros_like(x)
    for i, (I, lu) in enumerate(zip(dofs_list, lus)):
        y = sla.lu_solve(lu, r[I])
        dx[I] += _omega(omega, i) * y
    return x + dx


def mv_sweep(L, free, dofs_list, lus, omega, order, x, b):
    """One MV sweep (eqs. 11, 15): sequential patch updates in ``order``."""
    x = x.copy()
    Lcsr = L.tocsr()
    for i in order:
        I = dofs_list[i]
        ri = b[I] - Lcsr[I] @ x
        x[I] += _omega(omega, i) * sla.lu_solve(lus[i], ri)
    return x


def rav_sweep_rows(L, free, dofs_list, owned_list, W_list, omega, x, b):
    """RAV sweep with the stored owned rows W_i (FP64)."""
    r = residual(L, x, b, free)
    dx = np.zeros_like(x)
    for i, (I, own, W) in enumerate(zip(dofs_list, owned_list, W_list)):
        dx[I[own]] += _omega(omega, i) * (W @ r[I])
    return x + dx


def round_bf16(a):
    """Round float64 -> float32 (RNE) -> bfloat16 (RNE on the float32 bits);
    returned as float32 values holding the bfloat16 numbers."""
    f = np.asarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) >> 16 << 16
    return bits.astype(np.uint32).view(np.float32)


def round_storage(W, precision):
    """W in the storage precision: 'fp64', 'fp32' or 'bf16' (as float32 values)."""
    if precision == "fp64":
        return np.asarray(W, dtype=np.float64)
    if precision == "fp32":
        return np.asarray(W, dtype=np.float32)
    if precision == "bf16":
        return round_bf16(W)
    raise ValueError(precision)


def rav_sweep_rows_lowp(L, free, dofs_list, owned_list, Wlp_list, omega, x, b):
    """RAV sweep with W_i stored in float32/bfloat16: r_i rounded to float32,
    products and sums in float32, the correction added to the FP64 iterate."""
    r = residual(L, x, b, free)
    dx = np.zeros_like(x)
    for i, (I, own, W) in enumerate(zip(dofs_list, owned_list, Wlp_list)):
        y = (W @ r[I].astype(np.float32)).astype(np.float32)
        dx[I[own]] += _omega(omega, i) * y.astype(np.float64)
    return x + dx
