"""Host-side set-up of the adaptive grids (rav_adaptive_host_export, no device)
against the oracle (Sec. 2, Fig. 2; Sec. 4.1, Table 1): conforming operator
with hanging-node constraints, lid lifting, grid transfer and the MV colouring
on the first grids of the cavity hierarchy and on a randomly refined one, the DoF counts of Table 1, and the
rejection of grids that break the rules (not tiling, not 2:1 balanced, not
nested)."""
import os

import numpy as np
import pytest

import rav_inputs as ri
from oracle import adaptive_mg as am
from paper_2103_10127_amd import capi

BETA, ETA = 0.05, 1.0
N_GRIDS = 4


@pytest.fixture(scope="module", params=["cavity", "random"])
def hierarchy(request):
    if request.param == "cavity":
        return ri.cavity_grids(N_GRIDS), ri.lattice(N_GRIDS)
    return ri.random_quadtree_grids(N_GRIDS, base=8, frac=0.35, seed=1)


@pytest.mark.parametrize("level", range(N_GRIDS))
def test_operator_and_lid_match_oracle(hierarchy, level):
    G, M = hierarchy
    g = am.AdaptiveGrid(G[level], M, BETA, ETA)
    L = g.assemble().toarray()
    Lh = capi.adaptive_host_export(G, M, level, "operator", BETA, ETA)
    assert Lh.shape == L.shape
    np.testing.assert_allclose(Lh, L, rtol=0, atol=1e-13 * np.abs(L).max())
    np.testing.assert_allclose(capi.adaptive_host_export(G, M, level, "lid", BETA, ETA), g.lid_rhs(),
                               rtol=0, atol=1e-14)


@pytest.mark.parametrize("level", range(1, N_GRIDS))
def test_transfer_and_colouring_match_oracle(hierarchy, level):
    G, M = hierarchy
    g = am.AdaptiveGrid(G[level], M, BETA, ETA)
    gc = am.AdaptiveGrid(G[level - 1], M, BETA, ETA)
    P = am.prolongation(g, gc).toarray()
    np.testing.assert_allclose(capi.adaptive_host_export(G, M, level, "prolong", BETA, ETA), P, rtol=0, atol=1e-15)
    col = capi.adaptive_host_export(G, M, level, "colours", BETA, ETA)
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
    assert "tile" in _expect_einval([coarse, fine[:-1]], M)
    # one 8-cell next to 2-cells: not 2:1 balanced
    unbal = [(0, 0, 8), (8, 8, 8), (0, 8, 8)] + [(8 + x, y, 2) for y in range(0, 8, 2) for x in range(0, 8, 2)]
    assert "balanced" in _expect_einval([coarse, np.array(unbal, dtype=np.int32)], M)
    # the coarse grid is finer than the fine one somewhere: not nested
    assert "nested" in _expect_einval([fine, coarse], M)
    odd = np.concatenate([fine[:-1], [(12, 12, 3)]]).astype(np.int32)   # size 3: not a power of two
    assert "aligned" in _expect_einval([coarse, odd], M)
    with pytest.raises(capi.RavError):
        capi.adaptive_host_export([coarse, fine], 12, 1, "prolong", BETA, ETA)   # lattice not a power of two
