"""Pins of the adaptive-grid oracle (Sec. 2, Fig. 2; Sec. 4.1, Table 1): on a
uniformly refined grid it is the uniform Q1-Q1 oracle (operator and patches),
bilinear functions pass through hanging nodes and the transfer exactly, the
shear flow u = (y, 0) is the discrete solution on a grid with hanging nodes,
the MV colouring makes the colour-parallel sweep equal the sequential one,
and the V-cycle over the first four Table 1 grids converges."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import rav_inputs as ri
from oracle import adaptive as ad
from oracle import adaptive_mg as am
from oracle import mg
from oracle import q1q1 as q
from oracle import smoothers as sm

BETA = 0.05


def _uniform_leaves(N, M):
    s = M // N
    return np.array([[i * s, j * s, s] for j in range(N) for i in range(N)])


def test_uniform_grid_equals_the_uniform_oracle():
    g = am.AdaptiveGrid(_uniform_leaves(8, 32), 32, BETA)
    gq = q.GridQ1(2, 8, ri.ALL_DIRICHLET_2D)
    assert abs(g.assemble() - q.assemble_matrix(gq, BETA)).max() == 0.0
    ps = q.PatchSetQ1(gq)
    dofs, owned = g.patches()
    assert all(np.array_equal(a, b) for a, b in zip(dofs, ps.dofs))
    assert all(np.array_equal(a, b) for a, b in zip(owned, ps.owned))


def _bilinear(g):
    x, y = g.rx / g.M, g.ry / g.M
    f = 1.0 + 2.0 * x - 3.0 * y + 5.0 * x * y
    return np.concatenate([f, 2 * f, -f])


def _hierarchy(kind, n=3):
    """Grids of Table 1, or a randomly refined balanced hierarchy whose hanging
    nodes include constrained endpoints (chains of constraints)."""
    if kind == "table1":
        return ad.cavity_grids(n), ad.lattice(n)
    return ri.random_quadtree_grids(n, base=8, frac=0.35, seed=2)


@pytest.mark.parametrize("kind", ["table1", "random"])
def test_bilinear_functions_through_hanging_nodes_and_transfer(kind):
    """Grids 2 and 3 (Table 1: 16 and 56 hanging nodes; the random hierarchy:
    more, some constrained by hanging nodes): interpolating a bilinear
    function to the fine regular vertices with P (its pressure block, which no
    boundary condition masks) equals its values there; every hanging node's
    constraint weights reproduce it too."""
    grids, M = _hierarchy(kind)
    gs = [am.AdaptiveGrid(lv, M, BETA) for lv in grids]
    for gc, gf in zip(gs[1:], gs[2:]):
        assert len(gf.hang_ends) > 0
        P = am.prolongation(gf, gc)
        ps, pc = gf.pressure_slice(), gc.pressure_slice()   # no masking in the pressure field
        np.testing.assert_allclose(P[ps, pc] @ _bilinear(gc)[pc], _bilinear(gf)[ps], rtol=0, atol=1e-13)
        f = _bilinear(gf)[: gf.nV]
        for key in gf.hang_ends:
            x, y = divmod(key, M + 1)
            val = sum(w * f[j] for j, w in gf.weights(key).items())
            exact = 1.0 + 2.0 * x / M - 3.0 * y / M + 5.0 * x * y / M / M
            assert abs(val - exact) <= 1e-13


@pytest.mark.parametrize("kind", ["table1", "random"])
def test_shear_flow_is_exact_with_hanging_nodes(kind):
    """Dirichlet data u = (y, 0) on the boundary of grid 3: the conforming
    bilinear space holds the Stokes solution exactly (p = const), hanging
    nodes included."""
    grids, M = _hierarchy(kind)
    g = am.AdaptiveGrid(grids[2], M, BETA)
    uD = np.zeros(g.n)
    uD[: g.nV] = g.ry / M
    b = g.lifting(uD)
    L = g.assemble()
    f = g.free
    e = np.zeros(g.n)
    e[g.pressure_slice()] = 1.0
    K = sp.bmat([[L[f][:, f], sp.csc_matrix(e[f][:, None])], [sp.csc_matrix(e[f][None, :]), None]]).tocsc()
    y = spl.spsolve(K, np.concatenate([b[f], [0.0]]))
    x = np.zeros(g.n)
    x[f] = y[:-1]
    fr = f[: g.nV]
    assert np.abs(x[: g.nV][fr] - (g.ry / M)[fr]).max() <= 1e-12
    assert np.abs(x[g.nV: 2 * g.nV][fr]).max() <= 1e-12
    assert np.abs(x[g.pressure_slice()]).max() <= 1e-9   # p = 0 up to the direct solve's rounding


@pytest.mark.parametrize("kind", ["table1", "random"])
def test_mv_colouring_gives_the_colour_parallel_sweep(kind):
    """MV in colour order equals adding all same-colour patch corrections
    computed from one x, colour after colour, on grid 3."""
    grids, M = _hierarchy(kind)
    H = am.AdaptiveHierarchy(grids, M, BETA)
    lv = H.finest
    ps = lv.patches
    g = lv.grid
    x = ri.random_vector(g.n, 31) * g.free
    b = ri.random_vector(g.n, 32) * g.free
    seq = sm.mv_sweep(lv.L, lv.free, ps.dofs, lv.lus, 0.7, ps.order, x.copy(), b)
    par = x.copy()
    L = lv.L.tocsr()
    for c in np.unique(ps.colour):
        dx = np.zeros_like(par)
        for i in np.nonzero(ps.colour == c)[0]:
            I = ps.dofs[i]
            dx[I] += 0.7 * sla.lu_solve(lv.lus[i], b[I] - L[I] @ par)
        par = par + dx
    np.testing.assert_allclose(seq, par, rtol=0, atol=1e-13)


def test_vcycle_over_table1_grids_converges():
    """Grids 1-4 of Table 1 (7,059 DoFs on the finest), driven cavity, V(3,3):
    RAV (omega 0.66) and MV (0.66) converge to 1e-8 in at most 10 cycles, AV
    (0.1) in at most 30."""
    H = am.AdaptiveHierarchy(ad.cavity_grids(4), ad.lattice(4), BETA)
    b = H.finest.grid.lid_rhs()
    for smoother, om, cap in (("rav", 0.66, 10), ("mv", 0.66, 10), ("av", 0.1, 30)):
        _, k, _, st = H.solve(b, 1e-8, 100, smoother, om, 3)
        assert st == "converged" and k <= cap, (smoother, k)
