"""Pins of the oracle's element integrals and manufactured solution.

Closed forms are derived by hand from the 1D Lagrange bases (exact rationals);
the oracle evaluates the same integrals by 3-point Gauss quadrature.
"""
import numpy as np
import pytest

import rav_inputs as ri
from oracle import fem, mms

# 1D Q2 stiffness and mass on an interval of length h (nodes 0, h/2, h).
K1 = np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 3.0
M1 = np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) / 30.0
# G[k, a] = int_0^1 psi_k phi_a', H[k, a] = int_0^1 psi_k phi_a (psi: Q1, phi: Q2).
G1 = np.array([[-5 / 6, 2 / 3, 1 / 6], [-1 / 6, -2 / 3, 5 / 6]])
H1 = np.array([[1 / 6, 1 / 3, 0.0], [0.0, 1 / 3, 1 / 6]])


def kron_lex(*mats):
    """Tensor product for x-fastest lexicographic numbering; mats given as (x, y, z)."""
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(m, out)
    return out


@pytest.mark.parametrize("h", [1.0, 0.125])
def test_stiffness_2d_closed_form(h):
    ref = fem.RefElement(2)
    A = ref.stiffness(h, np.ones(9))
    K, M = K1 / h, M1 * h
    expect = kron_lex(K, M) + kron_lex(M, K)
    np.testing.assert_allclose(A, expect, rtol=0, atol=1e-14)


def test_stiffness_3d_closed_form():
    h = 0.25
    ref = fem.RefElement(3)
    A = ref.stiffness(h, np.ones(27))
    K, M = K1 / h, M1 * h
    expect = kron_lex(K, M, M) + kron_lex(M, K, M) + kron_lex(M, M, K)
    np.testing.assert_allclose(A, expect, rtol=0, atol=1e-14)


def test_viscosity_scales_stiffness_per_point():
    ref = fem.RefElement(2)
    eta = np.arange(1.0, 10.0)
    A = ref.stiffness(0.5, eta)
    # A is linear in the Gauss-point viscosities: compare against unit impulses.
    acc = sum(eta[q] * ref.stiffness(0.5, np.eye(9)[q]) for q in range(9))
    np.testing.assert_allclose(A, acc, atol=1e-13)
    assert np.all(np.linalg.eigvalsh(A)[1:] > 0)     # SPD up to the constant mode
    assert abs(np.linalg.eigvalsh(A)[0]) < 1e-12


@pytest.mark.parametrize("h", [1.0, 0.25])
def test_divergence_2d_closed_form(h):
    ref = fem.RefElement(2)
    B = ref.divergence(h)                       # (2, 9, 4)
    expect0 = -h * np.einsum("ka,lb->balk", G1, H1).reshape(9, 4)
    expect1 = -h * np.einsum("ka,lb->balk", H1, G1).reshape(9, 4)
    np.testing.assert_allclose(B[0], expect0, atol=1e-15)
    np.testing.assert_allclose(B[1], expect1, atol=1e-15)


def test_divergence_3d_closed_form():
    h = 0.5
    ref = fem.RefElement(3)
    B = ref.divergence(h)                       # (3, 27, 8)
    mats = [(G1, H1, H1), (H1, G1, H1), (H1, H1, G1)]
    for c, (X, Y, Z) in enumerate(mats):
        # node a = ix + 3 iy + 9 iz, pressure k = kx + 2 ky + 4 kz
        e = np.einsum("pa,qb,rc->cbarqp", X, Y, Z).reshape(27, 8)
        np.testing.assert_allclose(B[c], -h * h * e, atol=1e-15)


def test_load_of_constant():
    ref = fem.RefElement(2)
    h = 0.5
    f = np.ones((2, 9))
    b = ref.load(h, f)
    w1 = np.array([1 / 6, 2 / 3, 1 / 6])
    np.testing.assert_allclose(b[0], h * h * np.kron(w1, w1), atol=1e-15)


# ---- manufactured solution: invariants fixed by the construction (eq. 1) ----

def _fd_grad(fun, x, eps=1e-5):
    out = []
    for d in range(x.shape[-1]):
        e = np.zeros(x.shape[-1]); e[d] = eps
        out.append((fun(x + e) - fun(x - e)) / (2 * eps))
    return np.stack(out, axis=-1)


@pytest.mark.parametrize("dim,seed", [(2, 1001), (3, 1003)])
def test_mms_divergence_free_and_boundary(dim, seed):
    p = ri.mms_params(dim, seed)
    rng = np.random.default_rng(0)
    x = rng.uniform(0.05, 0.95, (50, dim))
    J = _fd_grad(lambda y: mms.velocity(p, y), x)       # (50, d, d): J[..., c, d]
    div = np.einsum("ncc->n", J)
    scale = np.abs(J).max()
    assert np.abs(div).max() < 1e-7 * scale
    xb = rng.uniform(0, 1, (50, dim))
    for d in range(dim):
        for side in (0.0, 1.0):
            y = xb.copy(); y[:, d] = side
            assert np.abs(mms.velocity(p, y)).max() < 1e-12


@pytest.mark.parametrize("dim,seed", [(2, 1001), (3, 1003)])
def test_mms_forcing_matches_finite_differences(dim, seed):
    p = ri.mms_params(dim, seed, eta=1.7)
    rng = np.random.default_rng(1)
    x = rng.uniform(0.1, 0.9, (20, dim))
    eps = 1e-3
    lap = np.zeros((20, dim))
    u0 = mms.velocity(p, x)
    for d in range(dim):
        e = np.zeros(dim); e[d] = eps
        lap += (mms.velocity(p, x + e) - 2 * u0 + mms.velocity(p, x - e)) / eps ** 2
    gp = _fd_grad(lambda y: mms.pressure(p, y), x)
    f_fd = -1.7 * lap + gp
    f = mms.forcing(p, x)
    assert np.abs(f - f_fd).max() < 1e-4 * np.abs(f).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_mms_pressure_zero_mean(dim):
    p = ri.mms_params(dim, 7)
    pts, wts = np.polynomial.legendre.leggauss(12)
    t = 0.5 * (pts + 1); w = 0.5 * wts
    grids = np.meshgrid(*([t] * dim), indexing="ij")
    W = np.ones_like(grids[0])
    for gw in np.meshgrid(*([w] * dim), indexing="ij"):
        W = W * gw
    x = np.stack([g.ravel() for g in grids], axis=1)
    assert abs(np.sum(W.ravel() * mms.pressure(p, x))) < 1e-12
