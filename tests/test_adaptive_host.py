"""Host-side set-up of the adaptive grids (rav_adaptive_host_export, no device)
against the oracle (Sec. 2, Fig. 2; Sec. 4.1, Table 1): conforming operator
with hanging-node constraints, lid lifting, grid transfer and the MV colouring
on the first grids of the cavity hierarchy, on a randomly refined one and on a
channel with an obstacle and an open outflow side (Sec. 4.2: the vertices and
their Dirichlet flags too), the DoF counts of Table 1, and the rejection of
grids that break the rules (not covering the region, not 2:1 balanced, not
nested)."""
import os

import numpy as np
import pytest

import rav_inputs as ri
from oracle import adaptive_mg as am
from paper_2103_10127_amd import capi

BETA, ETA = 0.05, 1.0
N_GRIDS = 4


@pytest.fixture(scope="module", params=["cavity", "random", "channel"])
def hierarchy(request):
    """(grids, lattice_x, lattice_y, Dirichlet mask)."""
    if request.param == "cavity":
        M = ri.lattice(N_GRIDS)
        return ri.cavity_grids(N_GRIDS), M, M, ri.ALL_DIRICHLET_2D
    if request.param == "random":
        G, M = ri.random_quadtree_grids(N_GRIDS, base=8, frac=0.35, seed=1)
        return G, M, M, ri.ALL_DIRICHLET_2D
    G, Mx, My = ri.channel_grids(N_GRIDS, bands=(ri.UNIFORM, 1, 1), cells=(16, 3))
    return G, Mx, My, ri.OUTFLOW_2D


def _export(hierarchy, level, what):
    G, Mx, My, dm = hierarchy
    return capi.adaptive_host_export(G, Mx, level, what, BETA, ETA, lattice_y=My, dmask=dm)


def _grid(hierarchy, level):
    G, Mx, My, dm = hierarchy
    return am.AdaptiveGrid(G[level], Mx, BETA, ETA, My=My, dmask=dm)


@pytest.mark.parametrize("level", range(N_GRIDS))
def test_operator_vertices_and_lid_match_oracle(hierarchy, level):
    g = _grid(hierarchy, level)
    L = g.assemble().toarray()
    Lh = _export(hierarchy, level, "operator")
    assert Lh.shape == L.shape
    np.testing.assert_allclose(Lh, L, rtol=0, atol=1e-13 * np.abs(L).max())
    np.testing.assert_allclose(_export(hierarchy, level, "lid"), g.lid_rhs(), rtol=0, atol=1e-14)
    V = _export(hierarchy, level, "vertices")
    np.testing.assert_array_equal(V[:, 0], g.rx)
    np.testing.assert_array_equal(V[:, 1], g.ry)
    np.testing.assert_array_equal(V[:, 2].astype(bool), g.dirichlet_node)


@pytest.mark.parametrize("level", range(1, N_GRIDS))
def test_transfer_and_colouring_match_oracle(hierarchy, level):
    g, gc = _grid(hierarchy, level), _grid(hierarchy, level - 1)
    P = am.prolongation(g, gc).toarray()
    np.testing.assert_allclose(_export(hierarchy, level, "prolong"), P, rtol=0, atol=1e-15)
    col = _export(hierarchy, level, "colours")
    np.testing.assert_array_equal(col.astype(np.int64), am.mv_colouring(g))


def test_table1_dof_counts_from_the_library():
    """Every grid of Table 1 up to Omega^8 built by the library: 3 unknowns
    per regular vertex give the printed n_DoF."""
    rows = [tuple(int(v) for v in line.split())
            for line in open(os.path.join(os.path.dirname(__file__), "golden", "table1_grids.txt"))
            if line.strip() and not line.startswith("#")]
    n = 8
    G, M = ri.cavity_grids(n), ri.lattice(n)
    for (k, n_e, n_dof) in rows[1:n]:
        lv = k - 1
        sub = G[: lv + 1]
        colours = capi.adaptive_host_export(sub, M, lv, "colours", BETA, ETA)
        assert len(sub[-1]) == n_e
        assert 3 * len(colours) == n_dof, k


def _expect_einval(grids, M):
    with pytest.raises(capi.RavError) as e:
        capi.adaptive_host_export(grids, M, 1, "prolong", BETA, ETA)
    assert e.value.status == -1
    return str(e.value)


def test_invalid_grids_are_rejected():
    M = 16
    coarse = np.array([(x, y, 8) for y in (0, 8) for x in (0, 8)], dtype=np.int32)
    fine = np.array([(x, y, 4) for y in range(0, 16, 4) for x in range(0, 16, 4)], dtype=np.int32)
    capi.adaptive_host_export([coarse, fine], M, 1, "prolong", BETA, ETA)   # valid
    assert "cover" in _expect_einval([coarse, fine[:-1]], M)
    # one 8-cell next to 2-cells: not 2:1 balanced
    unbal = [(0, 0, 8), (8, 8, 8), (0, 8, 8)] + [(8 + x, y, 2) for y in range(0, 8, 2) for x in range(0, 8, 2)]
    assert "balanced" in _expect_einval([coarse, np.array(unbal, dtype=np.int32)], M)
    # the coarse grid is finer than the fine one somewhere: not nested
    assert "nested" in _expect_einval([fine, coarse], M)
    odd = np.concatenate([fine[:-1], [(12, 12, 3)]]).astype(np.int32)   # size 3: not a power of two
    assert "aligned" in _expect_einval([coarse, odd], M)
    with pytest.raises(capi.RavError) as e:
        capi.adaptive_host_export([coarse, fine], 12, 1, "prolong", BETA, ETA)   # leaves beyond a 12-unit lattice
    assert "inside the rectangle" in str(e.value)


def test_open_sides_and_holes():
    """Dirichlet flags by side and around holes, from the library's set-up:
    with every side open and no hole nothing is Dirichlet; opening the top
    frees its inner vertices and leaves no lid (the lid export is refused);
    a hole's rim is Dirichlet whatever the mask."""
    M = 16
    full = np.array([(x, y, 4) for y in range(0, 16, 4) for x in range(0, 16, 4)], dtype=np.int32)
    coarse = np.array([(x, y, 8) for y in (0, 8) for x in (0, 8)], dtype=np.int32)
    V = capi.adaptive_host_export([coarse, full], M, 1, "vertices", BETA, ETA, dmask=0)
    assert V.shape == (25, 3) and not V[:, 2].any()
    V = capi.adaptive_host_export([coarse, full], M, 1, "vertices", BETA, ETA, dmask=0b0111)
    top_inner = (V[:, 1] == M) & (V[:, 0] > 0) & (V[:, 0] < M)
    assert not V[top_inner, 2].any() and V[~top_inner & ((V[:, 0] == 0) | (V[:, 1] == 0)), 2].all()
    with pytest.raises(capi.RavError) as e:
        capi.adaptive_host_export([coarse, full], M, 1, "lid", BETA, ETA, dmask=0b0111)
    assert "top side" in str(e.value)
    # a hole: the coarse cell (8, 8, 8) left out of both grids
    c2 = coarse[:3]
    f2 = full[~((full[:, 0] >= 8) & (full[:, 1] >= 8))]
    V = capi.adaptive_host_export([c2, f2], M, 1, "vertices", BETA, ETA, dmask=0)
    rim = ((V[:, 0] >= 8) & (V[:, 1] >= 8))
    assert rim.sum() == 5 and V[rim, 2].all() and not V[~rim, 2].any()
