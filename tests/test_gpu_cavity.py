"""Driven cavity (Sec. 4.1) on the GPU: the lifted right-hand side of the lid
data against the oracle's -L[free, masked] u_D (with and without an
inclusion), and the cavity solve with RAV, MV and AV against the oracle's
cycle counts and solutions."""
import numpy as np
import pytest

import rav_inputs as ri
from oracle import assemble as A
from oracle import mg
from oracle.grid import Grid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2103_10127_amd import Hierarchy  # noqa: E402


@pytest.mark.parametrize("N,incl,eta_in", [(16, None, 1.0), (48, np.array([[0.5, 0.93, 0.1]]), 50.0),
                                           (512, None, 1.0)])
def test_lid_rhs_matches_oracle(N, incl, eta_in):
    g = Grid(2, N, ri.ALL_DIRICHLET_2D)
    print(f"[gpu] cavity rhs N={N}", flush=True)
    nl = 2 if N <= 64 else 7   # the coarsest grid must fit the dense direct solve
    G = Hierarchy(dim=2, n_cells=N, n_levels=nl, eta_in=eta_in, inclusions=incl)
    b = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    G.assemble_rhs_lid(b, 1.5)
    bo = A.dirichlet_lifting(g, A.lid_velocity(g, 1.5), 1.0, eta_in, incl)
    assert np.abs(b.cpu().numpy() - bo).max() <= 1e-13 * np.abs(bo).max()
    G.close()


@pytest.mark.parametrize("smoother,omega", [("rav", 0.66), ("mv", 0.66), ("av", 0.1)])
def test_cavity_solve_matches_oracle(smoother, omega):
    N, nl = 32, 3
    H = mg.Hierarchy(2, N, nl, ri.ALL_DIRICHLET_2D)
    g = H.finest.grid
    bo = A.dirichlet_lifting(g, A.lid_velocity(g))
    xo, ko, _, sto = H.solve(bo, smoother=smoother, omega=omega, nu=3, maxit=300)
    print(f"[gpu] cavity solve {smoother}", flush=True)
    G = Hierarchy(dim=2, n_cells=N, n_levels=nl, smoother=smoother, omega=omega, nu_pre=3, nu_post=3)
    G.factor()
    b = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    G.assemble_rhs_lid(b)
    x = torch.zeros_like(b)
    st, it, rel = G.solve(x, b, 1e-8, 300)
    assert sto == "converged" and st == 0 and abs(it - ko) <= 1, (smoother, st, it, ko)
    assert mg.rel_l2(g, x.cpu().numpy(), xo) <= 1e-8
    G.close()
