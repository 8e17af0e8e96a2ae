"""Pins of the adaptive-grid oracle (Sec. 2, Fig. 2; Sec. 4.1, Table 1): on a
uniformly refined grid it is the uniform Q1-Q1 oracle (operator and patches),
bilinear functions pass through hanging nodes and the transfer exactly, the
shear flow u = (y, 0) is the discrete solution on a grid with hanging nodes,
the MV colouring makes the colour-parallel sweep equal the sequential one,
and the V-cycle over the first four Table 1 grids converges.  On the channel
with an obstacle and an open outflow side (Sec. 4.2): the vertex and
Dirichlet counts of the coarse grid by hand and Euler's formula, and the linear
flow u = (y, 0), p = 0 is the discrete solution and a fixed point of the
V-cycle (natural outflow condition, no pressure constraint)."""
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

# ---- channel with an obstacle and an open outflow side (Sec. 4.2) -------------
SMALL_CHANNEL = dict(bands=(ri.UNIFORM, 1, 1), cells=(16, 3))


def test_channel_coarse_grid_counts():
    """The coarse channel: 64 x 12 cells minus the six whose centres lie in the
    cylinder (cells (4,5), (5,4), (5,5), (5,6), (6,5), (6,6)), so 762 cells;
    65 x 13 lattice vertices minus the one inside the hole (6,6): 844.
    Dirichlet velocity: the rectangle's 2 x 65 + 2 x 11 boundary vertices
    minus the 11 inside the open side x = 64, plus the 12 vertices around the
    hole: 153.  Two uniform refinements of a mesh with one hole give the next
    vertex counts by Euler's formula.  The small test channel (16 x 3 cells, a
    one-cell hole): 68 vertices, 2 x 17 wall, 2 inflow and 4 hole vertices
    Dirichlet."""
    G, Mx, My = ri.channel_grids(3)
    g = am.AdaptiveGrid(G[0], Mx, BETA, My=My, dmask=ri.OUTFLOW_2D)
    assert (len(G[0]), g.nV, int(g.dirichlet_node.sum())) == (762, 844, 153)
    assert not g.all_dirichlet
    steps = ad.uniform_refinement_counts(844, 762, holes=1, steps=2)
    assert [(len(lv), ad.vertex_counts(lv)[2]) for lv in G[1:3]] == steps
    Gs, Mxs, Mys = ri.channel_grids(2, **SMALL_CHANNEL)
    gs = am.AdaptiveGrid(Gs[0], Mxs, BETA, My=Mys, dmask=ri.OUTFLOW_2D)
    assert (gs.nV, int(gs.dirichlet_node.sum())) == (68, 2 * 17 + 2 + 4)


@pytest.mark.parametrize("level", [0, 3])
def test_linear_flow_is_exact_in_the_channel(level):
    """With u_D = (y, 0) on every Dirichlet vertex (walls, inflow side and the
    obstacle) and the outflow side open, u = (y, 0), p = 0 solves the
    continuous problem (the natural condition grad(u) n - p n = 0 holds on
    x = const) and lies in the discrete space, so it is the discrete solution,
    on the coarse grid and on a grid with hanging nodes."""
    G, Mx, My = ri.channel_grids(4, **SMALL_CHANNEL)
    g = am.AdaptiveGrid(G[level], Mx, BETA, My=My, dmask=ri.OUTFLOW_2D)
    if level:
        assert ad.vertex_counts(G[level])[1] > 0
    outflow = (g.rx == Mx) & (g.ry > 0) & (g.ry < My)
    assert outflow.any() and g.free[: g.nV][outflow].all()
    u = np.zeros(g.n)
    u[: g.nV] = g.ry / My
    b = g.lifting(np.where(g.free, 0.0, u))
    fr = g.free
    x = np.zeros(g.n)
    x[fr] = spl.spsolve(g.assemble().tocsc()[fr][:, fr], b[fr])
    ex = np.where(fr, u, 0.0)
    assert np.abs(x[: 2 * g.nV] - ex[: 2 * g.nV]).max() <= 1e-12
    assert np.abs(x[2 * g.nV:]).max() <= 1e-9


def test_linear_flow_is_a_fixed_point_of_the_channel_vcycle():
    G, Mx, My = ri.channel_grids(4, **SMALL_CHANNEL)
    H = am.AdaptiveHierarchy(G, Mx, BETA, My=My, dmask=ri.OUTFLOW_2D)
    assert not H.bordered
    g = H.finest.grid
    u = np.zeros(g.n)
    u[: g.nV] = g.ry / My
    b = g.lifting(np.where(g.free, 0.0, u))
    ex = np.where(g.free, u, 0.0)
    for smoother in (mg.RAV, mg.MV):
        x = H.vcycle(ex.copy(), b, smoother, 0.66, 2)
        assert np.abs(x - ex).max() <= 1e-11, smoother
