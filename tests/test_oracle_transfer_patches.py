"""Pins of the oracle's grid transfer (nested interpolation) and Vanka patches."""
import itertools

import numpy as np
import pytest

import rav_inputs as ri
from oracle import patches as pt
from oracle import transfer
from oracle.grid import Grid


def test_q2_interp_weights_1d():
    P = transfer.interp_1d_q2(2)
    # Column of a coarse vertex node (A = 2): values at fine nodes 1..7.
    np.testing.assert_allclose(P[1:8, 2], [-1 / 8, 0, 3 / 8, 1, 3 / 8, 0, -1 / 8], atol=1e-16)
    # Column of a coarse mid node (A = 1): values at fine nodes 0..4.
    np.testing.assert_allclose(P[0:5, 1], [0, 3 / 4, 1, 3 / 4, 0], atol=1e-16)
    Pp = transfer.interp_1d_q1(2)
    np.testing.assert_allclose(Pp[1:4, 1], [1 / 2, 1, 1 / 2], atol=1e-16)


@pytest.mark.parametrize("dim", [2, 3])
def test_prolongation_reproduces_coarse_polynomials(dim):
    Nc = 2 if dim == 3 else 4
    fine, coarse = Grid(dim, 2 * Nc, 0), Grid(dim, Nc, 0)
    P = transfer.prolongation(fine, coarse)
    rng = np.random.default_rng(5)
    cq = rng.standard_normal((dim, 3 ** dim))     # per-component tensor quadratic coefficients

    def quad_fun(c, x):
        out = np.zeros(len(x))
        for j, e in enumerate(itertools.product(range(3), repeat=dim)):
            out += cq[c, j] * np.prod([x[:, d] ** e[d] for d in range(dim)], axis=0)
        return out

    def lin_fun(x):
        return 1.0 + x @ np.arange(1, dim + 1) + 0.5 * np.prod(x, axis=1)

    def nodal(g):
        xv = g.vnode * (g.h / 2)
        xp = g.pnode * g.h
        return np.concatenate([quad_fun(c, xv) for c in range(dim)] + [lin_fun(xp)])

    np.testing.assert_allclose(P @ nodal(coarse), nodal(fine), atol=1e-12)


def test_prolongation_keeps_constant_pressure_and_masks():
    fine, coarse = Grid(2, 8, ri.ALL_DIRICHLET_2D), Grid(2, 4, ri.ALL_DIRICHLET_2D)
    P = transfer.prolongation(fine, coarse)
    e = np.zeros(coarse.n); e[coarse.pressure_slice()] = 1.0
    ef = np.zeros(fine.n); ef[fine.pressure_slice()] = 1.0
    np.testing.assert_array_equal(P @ e, ef)
    assert not np.any(P[~fine.free].toarray())
    assert not np.any(P[:, ~coarse.free].toarray())


# ---- patches ---------------------------------------------------------------

@pytest.mark.parametrize("dim,N,kind,dm", [(2, 8, pt.VERTEX, ri.ALL_DIRICHLET_2D),
                                           (2, 6, pt.VERTEX, ri.OUTFLOW_2D),
                                           (3, 4, pt.ELEMENT, ri.ALL_DIRICHLET_3D),
                                           (3, 3, pt.ELEMENT, ri.OUTFLOW_3D),
                                           (2, 5, pt.ELEMENT, ri.ALL_DIRICHLET_2D)])
def test_owned_sets_partition_free_dofs(dim, N, kind, dm):
    g = Grid(dim, N, dm)
    ps = pt.PatchSet(g, kind)
    count = np.zeros(g.n, dtype=int)
    for I, own in zip(ps.dofs, ps.owned):
        assert len(np.unique(I)) == len(I)
        assert g.free[I].all()
        count[I[own]] += 1
    np.testing.assert_array_equal(count, g.free.astype(int))   # sum_i G_i = I on free DoFs


def _bucket_histogram_2d_vertex(N):
    """(n_i, owned_i) histogram of all-Dirichlet 2D vertex patches, counted per
    dimension: free nodes of [2k-2, 2k+2] and of {2k, 2k+1} in each direction."""
    k = np.arange(N + 1)
    lo = np.maximum(2 * k - 2, 1); hi = np.minimum(2 * k + 2, 2 * N - 1)
    span = hi - lo + 1
    own = np.minimum(2 * k + 1, 2 * N - 1) - np.maximum(2 * k, 1) + 1
    own = np.maximum(own, 0)
    hist = {}
    for i in range(N + 1):
        for j in range(N + 1):
            key = (2 * span[i] * span[j] + 1, 2 * own[i] * own[j] + 1)
            hist[key] = hist.get(key, 0) + 1
    return hist


def test_bucket_histogram_512():
    # Bucket table of the 512x512 hierarchy's finest level.
    expect = {(51, 9): 259081, (41, 9): 2036, (21, 5): 1018, (21, 1): 1018, (33, 9): 4,
              (17, 5): 4, (17, 1): 4, (9, 1): 3, (9, 3): 1}
    assert _bucket_histogram_2d_vertex(512) == expect


def test_patchset_matches_histogram_counting():
    g = Grid(2, 16, ri.ALL_DIRICHLET_2D)
    ps = pt.PatchSet(g, pt.VERTEX)
    hist = {}
    for I, own in zip(ps.dofs, ps.owned):
        key = (len(I), len(own))
        hist[key] = hist.get(key, 0) + 1
    assert hist == _bucket_histogram_2d_vertex(16)


def test_interior_patch_is_bt_row():
    """An interior vertex patch holds exactly the nonzero columns of row k of B^T
    plus p_k (Sec. 3)."""
    from oracle import assemble as A
    g = Grid(2, 8, ri.ALL_DIRICHLET_2D)
    L = A.assemble_matrix(g)
    ps = pt.PatchSet(g, pt.VERTEX)
    k = 4 + 9 * 4
    prow = g.pres(np.array([4, 4]))
    cols = L[prow].indices
    vel_cols = np.sort(cols[cols < 2 * g.nV])
    I = ps.dofs[k]
    np.testing.assert_array_equal(np.sort(I[:-1]), vel_cols)
    assert I[-1] == prow and len(I) == 51 and len(ps.owned[k]) == 9


def test_mv_colours_are_independent():
    """Two patches of one colour never write into each other's residual rows."""
    from oracle import assemble as A
    for dim, N, kind, dm in [(2, 9, pt.VERTEX, ri.ALL_DIRICHLET_2D), (3, 4, pt.ELEMENT, ri.OUTFLOW_3D)]:
        g = Grid(dim, N, dm)
        L = A.assemble_matrix(g).tocsr()
        ps = pt.PatchSet(g, kind)
        reach = [np.unique(L[I].indices) for I in ps.dofs]
        cols = np.array([pt.colour(g, kind, i) for i in range(ps.count)])
        for c in np.unique(cols):
            members = np.nonzero(cols == c)[0]
            for a, b in itertools.combinations(members, 2):
                assert not np.intersect1d(ps.dofs[a], reach[b]).size
                assert not np.intersect1d(ps.dofs[b], reach[a]).size
