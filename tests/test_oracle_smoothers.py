"""Pins of the oracle's Vanka smoothers and V-cycle (Sec. 3, eqs. 10-13, 15; Sec. 2).

Each check compares against something other than the oracle's own sweep code:
dense LU of the whole system, textbook Jacobi / Gauss-Seidel, brute-force
dense smoother operators, and the dense V-cycle error recursion.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import rav_inputs as ri
from oracle import assemble as A
from oracle import mg
from oracle import patches as pt
from oracle import smoothers as sm
from oracle.grid import Grid


def _setup(dim, N, dm, kind):
    g = Grid(dim, N, dm)
    L = A.assemble_matrix(g, 1.0, 20.0, np.array([[0.3, 0.4, 0.2]]) if dim == 2 else None)
    ps = pt.PatchSet(g, kind)
    lus = sm.factor(L, ps.dofs)
    return g, L, ps, lus


def test_one_patch_equals_dense_lu():
    """One patch covering every free DoF, omega = 1: RAV = AV = MV = L^{-1} b,
    bitwise equal to LAPACK's LU solve of the same matrix."""
    g = Grid(2, 4, ri.OUTFLOW_2D)
    L = A.assemble_matrix(g)
    b = A.assemble_rhs(g, ri.mms_params(2, 11))
    b[g.pressure_slice()] = ri.random_vector(g.nP, 3)
    I = np.nonzero(g.free)[0]
    lus = sm.factor(L, [I])
    own = [np.arange(len(I))]
    x0 = np.zeros(g.n)
    ref = np.zeros(g.n)
    ref[I] = sla.lu_solve(sla.lu_factor(L[I][:, I].toarray()), b[I])
    x_rav = sm.rav_sweep(L, g.free, [I], own, lus, 1.0, x0, b)
    x_av = sm.av_sweep(L, g.free, [I], lus, 1.0, x0, b)
    x_mv = sm.mv_sweep(L, g.free, [I], lus, 1.0, [0], x0, b)
    for x in (x_rav, x_av, x_mv):
        np.testing.assert_array_equal(x, ref)
    W = [sm.owned_rows(lus[0], own[0], len(I))]
    x_rows = sm.rav_sweep_rows(L, g.free, [I], own, W, 1.0, x0, b)
    np.testing.assert_allclose(x_rows, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_point_patches_are_jacobi_and_gauss_seidel():
    """Point patches on the SPD velocity block: AV and RAV are damped Jacobi,
    MV in lexicographic order is damped Gauss-Seidel."""
    g = Grid(2, 6, ri.ALL_DIRICHLET_2D)
    L = A.assemble_matrix(g)
    fv = np.nonzero(g.free[:2 * g.nV])[0]
    Av = L[fv][:, fv].tocsr()
    n = Av.shape[0]
    free = np.ones(n, bool)
    dofs = [np.array([i]) for i in range(n)]
    own = [np.array([0]) for _ in range(n)]
    lus = sm.factor(Av, dofs)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(n); b = rng.standard_normal(n)
    D = Av.diagonal()
    w = 0.7
    jac = x + w * (b - Av @ x) / D
    np.testing.assert_allclose(sm.av_sweep(Av, free, dofs, lus, w, x, b), jac, rtol=1e-13)
    np.testing.assert_allclose(sm.rav_sweep(Av, free, dofs, own, lus, w, x, b), jac, rtol=1e-13)
    # Damped GS: (D/w + L_low) x_new = b - (U + (1 - 1/w) D) x
    Low = sp.tril(Av, k=-1, format="csr")
    Up = sp.triu(Av, k=1, format="csr")
    M = (sp.diags(D / w) + Low).tocsr()
    rhs = b - Up @ x - (1 - 1 / w) * D * x
    gs = spla.spsolve_triangular(M, rhs, lower=True)
    np.testing.assert_allclose(sm.mv_sweep(Av, free, dofs, lus, w, np.arange(n), x, b), gs, rtol=1e-12)


def test_non_overlapping_patches_rav_equals_av():
    """Disjoint patches (velocity part of each owned set, SPD blocks): RAV = AV."""
    g = Grid(2, 4, ri.OUTFLOW_2D)
    L = A.assemble_matrix(g)
    ps = pt.PatchSet(g, pt.VERTEX)
    parts = [I[own][I[own] < 2 * g.nV] for I, own in zip(ps.dofs, ps.owned)]
    parts = [p for p in parts if len(p)]
    own = [np.arange(len(p)) for p in parts]
    lus = sm.factor(L, parts)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(g.n) * g.free; b = rng.standard_normal(g.n) * g.free
    a = sm.rav_sweep(L, g.free, parts, own, lus, 0.8, x, b)
    assert np.all(np.isfinite(a))
    np.testing.assert_allclose(a, sm.av_sweep(L, g.free, parts, lus, 0.8, x, b), rtol=1e-14)


@pytest.mark.parametrize("dim,N,kind,dm", [(2, 2, pt.VERTEX, ri.ALL_DIRICHLET_2D),
                                           (2, 4, pt.VERTEX, ri.ALL_DIRICHLET_2D),
                                           (2, 4, pt.VERTEX, ri.OUTFLOW_2D),
                                           (3, 2, pt.ELEMENT, ri.OUTFLOW_3D)])
@pytest.mark.parametrize("smoother", [mg.RAV, mg.AV, mg.MV])
def test_sweeps_match_dense_operators(dim, N, kind, dm, smoother):
    g, L, ps, lus = _setup(dim, N, dm, kind)
    rng = np.random.default_rng(6)
    omega = rng.uniform(0.4, 1.0, ps.count)
    M = mg.dense_smoother_operator(L, g.free, ps.dofs, ps.owned, lus, omega, smoother, ps.order)
    x = rng.standard_normal(g.n) * g.free
    b = np.zeros(g.n)
    if smoother == mg.RAV:
        y = sm.rav_sweep(L, g.free, ps.dofs, ps.owned, lus, omega, x, b)
    elif smoother == mg.AV:
        y = sm.av_sweep(L, g.free, ps.dofs, lus, omega, x, b)
    else:
        y = sm.mv_sweep(L, g.free, ps.dofs, lus, omega, ps.order, x, b)
    np.testing.assert_allclose(y, M @ x, rtol=0, atol=1e-13 * np.abs(x).max() * max(1, np.abs(M).max()))


def test_stored_rows_match_local_solves():
    g, L, ps, lus = _setup(2, 6, ri.ALL_DIRICHLET_2D, pt.VERTEX)
    W = [sm.owned_rows(lu, own, len(I)) for lu, own, I in zip(lus, ps.owned, ps.dofs)]
    rng = np.random.default_rng(8)
    x = rng.standard_normal(g.n) * g.free
    b = rng.standard_normal(g.n) * g.free
    a = sm.rav_sweep(L, g.free, ps.dofs, ps.owned, lus, 0.66, x, b)
    c = sm.rav_sweep_rows(L, g.free, ps.dofs, ps.owned, W, 0.66, x, b)
    np.testing.assert_allclose(c, a, rtol=0, atol=1e-13 * np.abs(a).max())


def test_bf16_rounding_is_round_to_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 3.0e-3], dtype=np.float64)
    out = sm.round_bf16(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa wins (1.0);
    # 1 + 3*2^-8 ties between 1+2^-7 and 1+2^-6: even is 1 + 2^-6.
    np.testing.assert_array_equal(out[:4], np.float32([1.0, 1.0, 1.0 + 2 ** -6, 1.0]))
    assert out[4] == np.float32(-2.5)
    assert abs(out[5] - 3.0e-3) <= 2 ** -8 * 3.0e-3


# ---- V-cycle ---------------------------------------------------------------

@pytest.mark.parametrize("N,nl,smoother", [(4, 2, mg.RAV), (8, 3, mg.RAV), (4, 2, mg.MV), (4, 2, mg.AV)])
def test_vcycle_matches_dense_recursion(N, nl, smoother):
    """Error propagation of V(nu,nu) built column by column equals
    E_l = M^nu (I - P (I - E_{l-1}) L_{l-1}^{-1} P^T L_l) M^nu with E_0 = 0."""
    dm = ri.OUTFLOW_2D
    H = mg.Hierarchy(2, N, nl, dm)
    nu, omega = 2, (0.66 if smoother != mg.AV else 0.3)
    fine = H.finest
    n = fine.grid.n
    free = np.nonzero(fine.grid.free)[0]
    EV = np.zeros((len(free), len(free)))
    b = np.zeros(n)
    for j, col in enumerate(free):
        x = np.zeros(n); x[col] = 1.0
        EV[:, j] = H.vcycle(x, b, smoother, omega, nu)[free]

    def Linv(lv):
        g = lv.grid
        M = lv.L.toarray(); M[~g.free, ~g.free] = 1.0
        return np.linalg.inv(M)

    E = None
    for l in range(1, nl):
        lv = H.levels[l]
        Msm = mg.dense_smoother_operator(lv.L, lv.grid.free, lv.patches.dofs, lv.patches.owned,
                                         lv.lus, omega, smoother, lv.patches.order)
        Mnu = np.linalg.matrix_power(Msm, nu)
        P = lv.P.toarray()
        inner = Linv(H.levels[l - 1]) if E is None else (np.eye(E.shape[0]) - E) @ Linv(H.levels[l - 1])
        C = np.eye(lv.grid.n) - P @ inner @ P.T @ lv.L.toarray()
        E = Mnu @ C @ Mnu
    np.testing.assert_allclose(EV, E[np.ix_(free, free)], rtol=0, atol=1e-12 * max(1, np.abs(E).max()))
    # The measured asymptotic rate matches the spectral radius of E_V.
    rho = np.abs(np.linalg.eigvals(EV)).max()
    x = ri.random_vector(n, 9) * fine.grid.free
    for _ in range(30):
        x = H.vcycle(x, b, smoother, omega, nu)
        x /= np.linalg.norm(x)
    y = H.vcycle(x, b, smoother, omega, nu)
    rate = np.linalg.norm(y) / np.linalg.norm(x)
    assert abs(rate - rho) <= 0.05 * rho + 1e-12


def test_variant_ordering_32():
    """Iterations to a 1e-8 reduction: MV <= RAV < AV(omega=0.1) (Sec. 4.1)."""
    cfg = ri.CONFIGS["2d-32"]
    H = mg.Hierarchy(2, 32, 3, cfg["dmask"])
    b = A.assemble_rhs(H.finest.grid, ri.mms_params(2, cfg["seed"]))
    its = {}
    for s, w in [(mg.RAV, 0.66), (mg.MV, 0.66), (mg.AV, 0.1)]:
        _, k, hist, st = H.solve(b, smoother=s, omega=w, maxit=300)
        assert st == "converged"
        its[s] = k
    assert its[mg.MV] <= its[mg.RAV] < its[mg.AV]


@pytest.mark.parametrize("prec,band", [("fp32", 0.10), ("bf16", 0.25)])
def test_mixed_precision_iterative_refinement(prec, band):
    H = mg.Hierarchy(2, 32, 3, ri.ALL_DIRICHLET_2D)
    g = H.finest.grid
    b = A.assemble_rhs(g, ri.mms_params(2, 1001))
    x64, k64, h64, st = H.solve(b)
    xr, _, _, _ = H.solve(b, rtol=1e-12)
    xl, kl, hl, st = H.solve(b, precision=prec)
    assert st == "converged"
    assert mg.avg_reduction(hl) <= (1 + band) * mg.avg_reduction(h64)
    assert mg.rel_l2(g, xl, xr) <= 1e-7
