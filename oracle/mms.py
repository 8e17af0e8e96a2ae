"""Manufactured Stokes solutions on [0,1]^d and their forcing (eq. 1).

2D: a stream function psi = sum_k a_k S(x; m_k) S(y; n_k) with S(t; m) = sin^2(m pi t)
gives u = (d psi/dy, -d psi/dx), which is divergence free and vanishes on the
boundary together with psi's first derivatives.
3D: u = curl Psi with every component Psi_c a sum of the same sin^2 products.
Pressure: p = sum_k c_k prod_d cos(r_{k,d} pi x_d), which has zero mean.
Forcing: f = -eta Laplace(u) + grad p, eta taken from the parameter array.

The parameter layout is that of ``rav_inputs.mms_params``.
"""
from __future__ import annotations

import numpy as np

N_MODES = 4


def _S(t, m, order):
    """order-th derivative of sin^2(m pi t)."""
    w = m * np.pi
    if order == 0:
        return np.sin(w * t) ** 2
    if order == 1:
        return w * np.sin(2 * w * t)
    if order == 2:
        return 2 * w * w * np.cos(2 * w * t)
    if order == 3:
        return -4 * w ** 3 * np.sin(2 * w * t)
    raise ValueError(order)


def unpack(params, dim):
    p = np.asarray(params, dtype=np.float64)
    eta = p[0]
    if dim == 2:
        if len(p) != 1 + 6 * N_MODES:
            raise ValueError("2D MMS parameter array must have 25 entries")
        a, m, n, c, r, s = (p[1 + i * N_MODES:1 + (i + 1) * N_MODES] for i in range(6))
        return eta, dict(a=a, m=m, n=n), dict(c=c, w=np.stack([r, s], 1))
    if len(p) != 1 + 16 * N_MODES:
        raise ValueError("3D MMS parameter array must have 65 entries")
    comps = []
    off = 1
    for _ in range(3):
        a, m, n, l = (p[off + i * N_MODES:off + (i + 1) * N_MODES] for i in range(4))
        comps.append(dict(a=a, w=np.stack([m, n, l], 1)))
        off += 4 * N_MODES
    c, r, s, t = (p[off + i * N_MODES:off + (i + 1) * N_MODES] for i in range(4))
    return eta, comps, dict(c=c, w=np.stack([r, s, t], 1))


def _prod_term(x, w, orders):
    """prod_d S^(orders[d])(x_d; w_d) for points x (..., d)."""
    out = np.ones(x.shape[:-1])
    for d, o in enumerate(orders):
        out = out * _S(x[..., d], w[d], o)
    return out


def velocity(params, x):
    """Exact velocity at points x (..., d) -> (..., d)."""
    dim = x.shape[-1]
    eta, vel, pres = unpack(params, dim)
    u = np.zeros(x.shape)
    if dim == 2:
        for k in range(N_MODES):
            w = (vel["m"][k], vel["n"][k])
            u[..., 0] += vel["a"][k] * _prod_term(x, w, (0, 1))
            u[..., 1] -= vel["a"][k] * _prod_term(x, w, (1, 0))
        return u
    # u = curl Psi: u_i = d_j Psi_k - d_k Psi_j for (i, j, k) cyclic
    for i in range(3):
        j, kk = (i + 1) % 3, (i + 2) % 3
        for m in range(N_MODES):
            oj = [0, 0, 0]; oj[j] = 1
            ok = [0, 0, 0]; ok[kk] = 1
            u[..., i] += vel[kk]["a"][m] * _prod_term(x, vel[kk]["w"][m], oj)
            u[..., i] -= vel[j]["a"][m] * _prod_term(x, vel[j]["w"][m], ok)
    return u


def pressure(params, x):
    dim = x.shape[-1]
    _, _, pres = unpack(params, dim)
    p = np.zeros(x.shape[:-1])
    for k in range(N_MODES):
        term = np.full(x.shape[:-1], pres["c"][k])
        for d in range(dim):
            term = term * np.cos(pres["w"][k][d] * np.pi * x[..., d])
        p += term
    return p


def grad_pressure(params, x):
    dim = x.shape[-1]
    _, _, pres = unpack(params, dim)
    g = np.zeros(x.shape)
    for k in range(N_MODES):
        for c in range(dim):
            term = np.full(x.shape[:-1], pres["c"][k])
            for d in range(dim):
                wd = pres["w"][k][d] * np.pi
                term = term * (-wd * np.sin(wd * x[..., d]) if d == c else np.cos(wd * x[..., d]))
            g[..., c] += term
    return g


def _laplace_prod(x, w, orders):
    """Laplacian of prod_d S^(orders[d])(x_d; w_d)."""
    out = np.zeros(x.shape[:-1])
    for d in range(len(orders)):
        o = list(orders)
        o[d] += 2
        out += _prod_term(x, w, o)
    return out


def laplace_velocity(params, x):
    dim = x.shape[-1]
    _, vel, _ = unpack(params, dim)
    lu = np.zeros(x.shape)
    if dim == 2:
        for k in range(N_MODES):
            w = (vel["m"][k], vel["n"][k])
            lu[..., 0] += vel["a"][k] * _laplace_prod(x, w, (0, 1))
            lu[..., 1] -= vel["a"][k] * _laplace_prod(x, w, (1, 0))
        return lu
    for i in range(3):
        j, kk = (i + 1) % 3, (i + 2) % 3
        for m in range(N_MODES):
            oj = [0, 0, 0]; oj[j] = 1
            ok = [0, 0, 0]; ok[kk] = 1
            lu[..., i] += vel[kk]["a"][m] * _laplace_prod(x, vel[kk]["w"][m], oj)
            lu[..., i] -= vel[j]["a"][m] * _laplace_prod(x, vel[j]["w"][m], ok)
    return lu


def forcing(params, x):
    """f = -eta Laplace(u) + grad p at points x (..., d) -> (..., d)."""
    eta = float(np.asarray(params)[0])
    return -eta * laplace_velocity(params, x) + grad_pressure(params, x)
