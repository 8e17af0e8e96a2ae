"""One RAV sweep on a 3D grid whose top-edge buckets exceed 64 patches.

Element patches on a top edge of the box (two coordinates at N - 1) form
buckets of N - 1 patches.  Up to N = 65 they run in the row-parallel kernel;
on this 80^3 grid (79 patches per edge bucket) they take the column-group
variants of the edge classes, alone or in the merged launch with the edge
bodies compiled in.  Every owned row of sampled patches of each class is
checked against the oracle's LU solve of the patch system (eq. 13 restricted
to the owned DoFs), with the patch rows from the oracle's row-wise assembly.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import rav_inputs as ri
from oracle import assemble as A
from oracle import patches as pt
from oracle.grid import Grid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2103_10127_amd import Hierarchy  # noqa: E402

N, NL = 80, 5
DM = ri.ALL_DIRICHLET_3D
OMEGA = 0.5


def _elem(e0, e1, e2):
    return e0 + N * (e1 + N * e2)


def test_one_sweep_edge_classes_above_64_patches():
    print("[gpu] 3D 80^3 element-patch hierarchy (edge buckets of 79 patches)", flush=True)
    g = Grid(3, N, DM)
    H = Hierarchy(dim=3, n_cells=N, n_levels=NL, dmask=DM, kind="element", omega=OMEGA)
    try:
        H.factor()
        x = ri.random_vector(g.n, 91) * g.free
        b = ri.random_vector(g.n, 92) * g.free
        xd = torch.from_numpy(x).cuda()
        H.smooth(NL - 1, 1, xd, torch.from_numpy(b).cuda())
        xg = xd.cpu().numpy()
    finally:
        H.close()
    owner = pt.owner_of_dofs(g, pt.ELEMENT)
    rng = np.random.default_rng(93)
    k = rng.integers(1, N - 2, size=8)
    t = N - 1
    patches = [
        _elem(t, t, k[0]), _elem(t, t, k[1]),          # edge classes: two top coordinates
        _elem(t, k[2], t), _elem(t, k[3], t),
        _elem(k[4], t, t), _elem(k[5], t, t),
        _elem(t, t, t),                                # corner
        _elem(t, k[6], k[7]), _elem(k[6], t, k[7]), _elem(k[6], k[7], t),   # faces
        _elem(k[0], k[1], k[2]),                       # interior
    ]
    checked = 0
    for p in patches:
        I = pt.patch_dofs(g, pt.ELEMENT, int(p))
        rows = {i: A.matrix_row(g, int(i)) for i in I}
        Li = np.array([[rows[i].get(j, 0.0) for j in I] for i in I])
        r_i = np.array([b[i] - sum(v * x[c] for c, v in rows[i].items()) for i in I])
        y = sla.lu_solve(sla.lu_factor(Li), r_i)
        own = np.nonzero(owner[I] == p)[0]
        assert len(own) > 0, p
        for loc in own:
            d = I[loc]
            expect = x[d] + OMEGA * y[loc]
            assert abs(xg[d] - expect) <= 1e-10 * max(1.0, abs(y[loc])), (p, d)
            checked += 1
    assert checked > 100
    assert np.all(xg[~g.free] == 0.0)
