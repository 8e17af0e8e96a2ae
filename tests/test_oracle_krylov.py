"""Pins of the oracle's flexible GMRES: it reproduces scipy's GMRES (the
minimal-residual iterate is unique) and one iteration with the exact inverse as
preconditioner solves the system."""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import rav_inputs as ri
from oracle import assemble as A
from oracle import krylov
from oracle import mg
from oracle.grid import Grid


def _system():
    g = Grid(2, 4, ri.OUTFLOW_2D)
    L = A.assemble_matrix(g)
    f = np.nonzero(g.free)[0]
    Lf = L[f][:, f].toarray()
    b = ri.random_vector(len(f), 3)
    return Lf, b


def test_matches_scipy_gmres_without_preconditioner():
    Lf, b = _system()
    x, it, hist = krylov.fgmres(lambda v: Lf @ v, lambda v: v, b, rtol=1e-10, restart=200, maxit=200)
    xs, info = spla.gmres(Lf, b, rtol=1e-10, atol=0.0, restart=200, maxiter=200)
    assert info == 0
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-7 * np.abs(xs).max())
    np.testing.assert_allclose(x, np.linalg.solve(Lf, b), rtol=0, atol=1e-7 * np.abs(xs).max())


def test_minimal_residual_property():
    """The k-th iterate has the smallest residual over span{b, Lb, ..., L^(k-1) b}."""
    Lf, b = _system()
    k = 8
    x, it, hist = krylov.fgmres(lambda v: Lf @ v, lambda v: v, b, rtol=1e-30, restart=k, maxit=k)
    K = np.stack([np.linalg.matrix_power(Lf, i) @ b for i in range(k)], axis=1)
    Q, _ = np.linalg.qr(K)
    c, *_ = np.linalg.lstsq(Lf @ Q, b, rcond=None)
    best = np.linalg.norm(b - Lf @ (Q @ c))
    assert abs(np.linalg.norm(b - Lf @ x) - best) <= 1e-8 * best


def test_exact_preconditioner_one_step():
    Lf, b = _system()
    lu = sla.lu_factor(Lf)
    x, it, hist = krylov.fgmres(lambda v: Lf @ v, lambda v: sla.lu_solve(lu, v), b, rtol=1e-12, restart=10, maxit=10)
    assert it == 1
    np.testing.assert_allclose(x, sla.lu_solve(lu, b), rtol=0, atol=1e-12 * np.abs(x).max())


def test_vcycle_preconditioned_converges_at_high_contrast():
    """Where the stand-alone RAV V-cycle diverges (contrast 1e3 inclusions),
    the V-cycle-preconditioned GMRES still reaches 1e-8."""
    incl = ri.inclusions(3000)
    H = mg.Hierarchy(2, 32, 2, ri.ALL_DIRICHLET_2D, 0, 1.0, 1e3, incl)
    g = H.finest.grid
    b = A.assemble_rhs(g, ri.mms_params(2, 3000))
    _, k, hist, st = H.solve(b, maxit=30)
    assert st == "diverged"
    Lf = H.finest.L

    def apply_L(v):
        y = Lf @ v
        y[~g.free] = 0.0
        return y

    x, it, hist = krylov.fgmres(apply_L, lambda r: H.vcycle(np.zeros(g.n), r, "rav", 0.66, 2), b,
                                rtol=1e-8, restart=30, maxit=200)
    assert np.linalg.norm(b - apply_L(x)) <= 1e-8 * np.linalg.norm(b)
    assert it < 200
