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


def _oracle_fgmres(H, b, smoother, omega, nu, restart=30, maxit=300):
    lv = H.finest
    g = lv.grid

    def apply_L(v):
        y = lv.L @ v
        y[~g.free] = 0.0
        return y

    return krylov.fgmres(apply_L, lambda r: H.vcycle(np.zeros(g.n), r, smoother, omega, nu), b,
                         rtol=1e-8, restart=restart, maxit=maxit)


def _check_gmres(G, g, b, xo, ko):
    G.factor()
    x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    st, it, rel = G.solve_gmres(x, torch.from_numpy(b).cuda(), 1e-8, 300, 30)
    assert st == 0 and rel <= 1e-8, (st, it, rel)
    assert abs(it - ko) <= 1, (it, ko)
    assert mg.rel_l2(g, x.cpu().numpy(), xo) <= 1e-6
    x2 = torch.zeros_like(x)
    st2, it2, _ = G.solve_gmres_noalloc(x2, torch.from_numpy(b).cuda(), 1e-8, 300, 30)
    assert st2 == 0 and it2 == it and torch.equal(x2, x)
    G.close()


def test_gmres_q1q1_cavity():
    """FGMRES on the stabilized Q1-Q1 cavity (32^2, coarsest 8^2, RAV V(2,2))."""
    from oracle import q1q1 as q
    print("[gpu] gmres q1q1 cavity 32^2", flush=True)
    H = q.HierarchyQ1(2, 32, 3, ri.ALL_DIRICHLET_2D, 0.05)
    g = H.finest.grid
    b = q.dirichlet_lifting(g, q.lid_velocity(g), 0.05)
    xo, ko, _ = _oracle_fgmres(H, b, mg.RAV, 0.66, 2)
    _check_gmres(Hierarchy(dim=2, n_cells=32, n_levels=3, discretization="q1q1", beta=0.05), g, b, xo, ko)


@pytest.mark.parametrize("case", ["cavity", "channel"])
def test_gmres_adaptive(case):
    """FGMRES on the adaptive grids: the first four Table 1 grids with the lid,
    and a small channel with inflow and an open outflow side (RAV V(2,2))."""
    from oracle import adaptive_mg as am
    from paper_2103_10127_amd.capi import AdaptiveHierarchy
    print(f"[gpu] gmres adaptive {case}", flush=True)
    if case == "cavity":
        G_, Mx, My, dm = ri.cavity_grids(4), ri.lattice(4), ri.lattice(4), ri.ALL_DIRICHLET_2D
    else:
        G_, Mx, My = ri.channel_grids(4, bands=(ri.UNIFORM, 1, 1), cells=(16, 3))
        dm = ri.OUTFLOW_2D
    H = am.AdaptiveHierarchy(G_, Mx, 0.05, 1.0, My=My, dmask=dm)
    g = H.finest.grid
    b = g.lid_rhs() if case == "cavity" else g.lifting(g.inflow_velocity(0.3))
    xo, ko, _ = _oracle_fgmres(H, b, mg.RAV, 0.66, 2)
    _check_gmres(AdaptiveHierarchy(G_, Mx, smoother="rav", omega=0.66, nu_pre=2, nu_post=2, beta=0.05,
                                   lattice_y=My, dmask=dm), g, b, xo, ko)


def test_gmres_workspace_kept_and_replaced():
    """The context keeps FGMRES's work vectors between calls and replaces them
    when the restart length changes: restart 10, then 30, then 10 again on one
    context give the first call's iterate bit for bit, and the 30 result agrees
    with a fresh context's (to rounding: the set-up autotuner may pick other
    lane counts, so other summation orders, in another context)."""
    print("[gpu] gmres workspace reuse", flush=True)
    N, nl = 32, 3
    xs = {}
    G = Hierarchy(dim=2, n_cells=N, n_levels=nl)
    G.factor()
    g_n = G.dofs(nl - 1)[0]
    H = mg.Hierarchy(2, N, nl, ri.ALL_DIRICHLET_2D, 0, 1.0, 1.0, ri.inclusions(3000))
    b = torch.from_numpy(A.assemble_rhs(H.finest.grid, ri.mms_params(2, 3001))).cuda()
    assert b.numel() == g_n
    for tag, m in (("a", 10), ("b", 30), ("c", 10)):
        x = torch.zeros(g_n, dtype=torch.float64, device="cuda")
        st, it, rel = G.solve_gmres(x, b, 1e-8, 300, m)
        assert st == 0, (tag, st)
        xs[tag] = (x, it)
    assert torch.equal(xs["a"][0], xs["c"][0]) and xs["a"][1] == xs["c"][1]
    G.close()
    F = Hierarchy(dim=2, n_cells=N, n_levels=nl)
    F.factor()
    x = torch.zeros(g_n, dtype=torch.float64, device="cuda")
    st, it, rel = F.solve_gmres(x, b, 1e-8, 300, 30)
    assert st == 0 and it == xs["b"][1]
    assert float((x - xs["b"][0]).norm() / xs["b"][0].norm()) <= 1e-10
    F.close()
