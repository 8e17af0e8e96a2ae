"""Pins of the oracle's global system (eqs. 6-7): sizes, invariants, and the
textbook Taylor-Hood convergence orders of the manufactured solution."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import rav_inputs as ri
from oracle import assemble as A
from oracle import fem, mms
from oracle.grid import Grid


@pytest.mark.parametrize("dim,N,n", [(2, 32, 9539), (2, 512, 2364419), (3, 64, 6714692),
                                     (2, 1024, 9447427), (2, 8, 659), (3, 4, 2312)])
def test_dof_counts(dim, N, n):
    g = Grid(dim, N, ri.ALL_DIRICHLET_2D if dim == 2 else ri.ALL_DIRICHLET_3D)
    assert g.n == n


@pytest.mark.parametrize("dim,N,nnz", [(2, 8, 11526), (2, 16, 52038), (2, 32, 220614), (3, 4, 65979)])
def test_nnz_all_dirichlet(dim, N, nnz):
    g = Grid(dim, N, ri.ALL_DIRICHLET_2D if dim == 2 else ri.ALL_DIRICHLET_3D)
    L = A.assemble_matrix(g)
    assert L.nnz == nnz          # structural pattern: every coupled (row, col) pair


@pytest.mark.parametrize("dim,N", [(2, 8), (3, 4)])
def test_symmetry_nullspace_spd(dim, N):
    dm = ri.ALL_DIRICHLET_2D if dim == 2 else ri.ALL_DIRICHLET_3D
    g = Grid(dim, N, dm)
    incl = np.array([[0.4, 0.5, 0.2]]) if dim == 2 else np.array([[0.4, 0.5, 0.5, 0.3]])
    L = A.assemble_matrix(g, 1.0, 50.0, incl)
    assert abs(L - L.T).max() < 1e-14 * abs(L).max()
    e = np.zeros(g.n); e[g.pressure_slice()] = 1.0
    assert np.abs(L @ e).max() < 1e-13 * abs(L).max()      # B 1_p = 0 on free rows
    nv = dim * g.nV
    fv = np.nonzero(g.free[:nv])[0]
    Af = L[fv][:, fv].toarray()
    assert np.linalg.eigvalsh(Af).min() > 0
    assert not np.any(L[~g.free].toarray())                  # masked rows empty


def test_outflow_nonsingular():
    g = Grid(2, 4, ri.OUTFLOW_2D)
    L = A.assemble_matrix(g)
    f = np.nonzero(g.free)[0]
    Lf = L[f][:, f].toarray()
    s = np.linalg.svd(Lf, compute_uv=False)
    assert s.min() > 1e-8 * s.max()


@pytest.mark.parametrize("dim,N", [(2, 8), (3, 4)])
def test_matrix_row_matches_global(dim, N):
    dm = ri.ALL_DIRICHLET_2D if dim == 2 else ri.OUTFLOW_3D
    g = Grid(dim, N, dm)
    incl = np.array([[0.3, 0.6, 0.25]]) if dim == 2 else np.array([[0.3, 0.6, 0.5, 0.3]])
    L = A.assemble_matrix(g, 1.0, 1e3, incl)
    rng = np.random.default_rng(3)
    for row in rng.choice(g.n, 40, replace=False):
        d = A.matrix_row(g, row, 1.0, 1e3, incl)
        dense = np.zeros(g.n)
        for c, v in d.items():
            dense[c] = v
        np.testing.assert_allclose(dense, L[row].toarray().ravel(), atol=1e-12 * abs(L).max())


# ---- manufactured-solution convergence (textbook Q2/Q1 orders) -------------

def _solve_direct(g, L, b):
    Lm = L.tolil()
    for i in np.nonzero(~g.free)[0]:
        Lm[i, i] = 1.0
    e = np.zeros(g.n); e[g.pressure_slice()] = 1.0
    M = sp.bmat([[Lm.tocsr(), sp.csr_matrix(e[:, None])], [sp.csr_matrix(e[None, :]), None]]).tocsc()
    return spla.spsolve(M, np.concatenate([b, [0.0]]))[:g.n]


def _errors(g, params, x):
    """L2 errors of velocity and (mean-free) pressure with a 5-point Gauss rule."""
    d = g.dim
    t, w = np.polynomial.legendre.leggauss(5)
    t = 0.5 * (t + 1); w = 0.5 * w
    import itertools
    qp = np.array([p[::-1] for p in itertools.product(t, repeat=d)])
    qw = np.array([np.prod(p) for p in itertools.product(w, repeat=d)])
    ref = fem.RefElement(d)
    v1 = [fem.q2_1d(qp[:, k]) for k in range(d)]
    p1 = [fem.q1_1d(qp[:, k]) for k in range(d)]
    phi = np.ones((len(ref.vnodes), len(qw)))
    for a, idx in enumerate(ref.vnodes):
        for k in range(d):
            phi[a] *= v1[k][idx[k]]
    psi = np.ones((len(ref.pnodes), len(qw)))
    for a, idx in enumerate(ref.pnodes):
        for k in range(d):
            psi[a] *= p1[k][idx[k]]
    elems = g.elements()
    xq = (elems[:, None, :] + qp[None]) * g.h
    vd, pd = A.element_dofs(g, ref, elems)
    uh = np.einsum("ecn,nq->eqc", x[vd], phi)
    ph = np.einsum("en,nq->eq", x[pd], psi)
    ue = mms.velocity(params, xq)
    pe = mms.pressure(params, xq)
    W = qw[None, :] * g.h ** d
    eu = np.sqrt(np.sum(W[..., None] * (uh - ue) ** 2))
    dp = ph - pe
    dp = dp - np.sum(W * dp) / np.sum(W)
    ep = np.sqrt(np.sum(W * dp ** 2))
    return eu, ep


def _low_frequency(params, dim):
    """Same amplitudes, every wave number set to 1 (reaches the asymptotic
    range on the coarse 3D grids a direct solve can afford)."""
    p = params.copy()
    nm = 4
    if dim == 3:
        for comp in range(3):
            off = 1 + comp * 16
            p[off + nm:off + 4 * nm] = 1.0
        p[1 + 48 + nm:] = 1.0
    return p


@pytest.mark.parametrize("dim,Ns,seed", [(2, (8, 16, 32), 1001), (3, (2, 4, 8), 1003)])
def test_mms_convergence_orders(dim, Ns, seed):
    params = ri.mms_params(dim, seed)
    if dim == 3:
        params = _low_frequency(params, dim)
    dm = ri.ALL_DIRICHLET_2D if dim == 2 else ri.ALL_DIRICHLET_3D
    eus, eps_ = [], []
    for N in Ns:
        g = Grid(dim, N, dm)
        L = A.assemble_matrix(g)
        b = A.assemble_rhs(g, params)
        x = _solve_direct(g, L, b)
        eu, ep = _errors(g, params, x)
        eus.append(eu); eps_.append(ep)
    ou = np.log2(eus[-2] / eus[-1])
    op = np.log2(eps_[-2] / eps_[-1])
    assert ou >= 2.8, (eus, ou)
    assert op >= 1.9, (eps_, op)
