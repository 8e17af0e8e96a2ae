"""V-cycle-preconditioned GMRES on the GPU against the oracle's FGMRES with the
same preconditioner (same iterates up to rounding)."""
import numpy as np
import pytest

import rav_inputs as ri
from oracle import assemble as A
from oracle import krylov
from oracle import mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2103_10127_amd import Hierarchy  # noqa: E402


@pytest.mark.parametrize("N,nl,contrast", [(32, 2, 1e3), (32, 3, 1.0), (40, 3, 1e2)])
def test_gmres_matches_oracle(N, nl, contrast):
    incl = ri.inclusions(3000)
    print(f"[gpu] gmres N={N} nl={nl} contrast={contrast}", flush=True)
    H = mg.Hierarchy(2, N, nl, ri.ALL_DIRICHLET_2D, 0, 1.0, contrast, incl)
    g = H.finest.grid
    b = A.assemble_rhs(g, ri.mms_params(2, 3000))
    Lf = H.finest.L

    def apply_L(v):
        y = Lf @ v
        y[~g.free] = 0.0
        return y

    xo, ko, hist = krylov.fgmres(apply_L, lambda r: H.vcycle(np.zeros(g.n), r, "rav", 0.66, 2), b,
                                 rtol=1e-8, restart=30, maxit=300)
    G = Hierarchy(dim=2, n_cells=N, n_levels=nl, eta_in=contrast, inclusions=incl)
    G.factor()
    x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    st, it, rel = G.solve_gmres(x, torch.from_numpy(b).cuda(), 1e-8, 300, 30)
    assert st == 0 and rel <= 1e-8, (st, it, rel)
    assert abs(it - ko) <= 1, (it, ko)
    assert mg.rel_l2(g, x.cpu().numpy(), xo) <= 1e-6
    G.close()
