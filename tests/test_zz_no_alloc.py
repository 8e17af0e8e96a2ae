"""rav_solve_gmres_noalloc (the entry point for callers that cannot allocate
device memory) against rav_solve_gmres on the same problems: two calls in a
row, the second on a smaller problem, each bit-identical to the allocating
entry point (same kernels and order, only the workspace differs); requests
beyond the static workspace are refused."""
import numpy as np
import pytest

import rav_inputs as ri
from oracle import assemble as A
from oracle.grid import Grid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2103_10127_amd import Hierarchy  # noqa: E402
from paper_2103_10127_amd.capi import RavError  # noqa: E402


def _problem(N, nl, contrast, seed):
    incl = ri.inclusions(seed)
    g = Grid(2, N, ri.ALL_DIRICHLET_2D)
    b = A.assemble_rhs(g, ri.mms_params(2, 1004))
    print(f"[gpu] no-alloc GMRES N={N} levels={nl} contrast={contrast}", flush=True)
    G = Hierarchy(dim=2, n_cells=N, n_levels=nl, eta_in=contrast, inclusions=incl)
    G.factor()
    return G, torch.from_numpy(b).cuda()


def test_noalloc_gmres_equals_allocating_gmres_twice():
    for N, nl, contrast, restart in [(64, 4, 1e3, 30), (32, 3, 1e2, 20)]:
        G, b = _problem(N, nl, contrast, 2000 + N)
        xa = torch.zeros_like(b)
        sa, ia, ra = G.solve_gmres(xa, b, 1e-8, 300, restart)
        xn = torch.zeros_like(b)
        sn, in_, rn = G.solve_gmres_noalloc(xn, b, 1e-8, 300, restart)
        assert sa == 0 and ra <= 1e-8, (sa, ia, ra)
        assert (sn, in_, rn) == (sa, ia, ra)
        assert torch.equal(xn, xa)
        G.close()


def test_noalloc_gmres_refuses_oversized_requests():
    G, b = _problem(16, 2, 1.0, 2016)
    x = torch.zeros_like(b)
    with pytest.raises(RavError) as e:
        G.solve_gmres_noalloc(x, b, 1e-8, 10, 65)   # restart above the maximum
    assert e.value.status == -1
    G.close()
    G, b = _problem(128, 5, 1.0, 2128)
    x = torch.zeros_like(b)
    with pytest.raises(RavError) as e:
        G.solve_gmres_noalloc(x, b, 1e-8, 10, 64)   # 131 vectors of 148,739 entries: 156 MB
    assert e.value.status == -1 and "workspace" in str(e.value)
    # a restart that fits runs and matches the allocating solver
    st, it, rel = G.solve_gmres_noalloc(x, b, 1e-8, 100, 20)
    xa = torch.zeros_like(b)
    assert (st, it, rel) == G.solve_gmres(xa, b, 1e-8, 100, 20) and torch.equal(x, xa)
    G.close()
