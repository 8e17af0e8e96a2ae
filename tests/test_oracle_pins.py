"""Pins of oracle pieces that the other CPU tests only compared with themselves:
the inclusion rule at Gauss points, the low-precision RAV sweep arithmetic,
the 3D element-patch bucket table of the 64^3 workload and mesh independence
of the RAV V-cycle up to 256^2 (Sec. 4: rates that do not degrade with
refinement).  Expected values are worked out by hand in each docstring."""
import numpy as np
import pytest
import scipy.sparse as sp

import rav_inputs as ri
from oracle import assemble as A
from oracle import mg
from oracle import patches as pt
from oracle import smoothers as sm
from oracle.fem import RefElement
from oracle.grid import Grid

# 3-point Gauss abscissae on [0,1] are 1/2 and 1/2 -+ sqrt(15)/10 (0.3873 from the middle).
OFF = np.sqrt(15.0) / 10.0


def test_viscosity_single_cell_radius_cases():
    """One cell (N = 1, h = 1), disc centred at the cell centre.  The nine
    Gauss points sit at the centre (distance 0), at the four edge-parallel
    offsets (distance sqrt(15)/10 = 0.387) and at the four diagonal offsets
    (distance sqrt(30)/10 = 0.548).  Radii 0.3 / 0.45 / 0.6 take 1 / 5 / 9 of
    them; point order is lexicographic, x fastest.  A 2D inclusion is the
    row (cx, cy, r)."""
    g = Grid(2, 1, ri.ALL_DIRICHLET_2D)
    ref = RefElement(2)
    elems = g.elements()
    centre_only = np.array([[1, 1, 1, 1, 5, 1, 1, 1, 1]], dtype=float)
    plus = np.array([[1, 5, 1, 5, 5, 5, 1, 5, 1]], dtype=float)
    for r, expect in [(0.3, centre_only), (0.45, plus), (0.6, np.full((1, 9), 5.0))]:
        eta = A.viscosity(g, ref, elems, 1.0, 5.0, [[0.5, 0.5, r]])
        np.testing.assert_array_equal(eta, expect)
    assert OFF < 0.45 < np.sqrt(2) * OFF


def test_viscosity_element_and_axis_order():
    """N = 2 (h = 1/2): a disc of radius 0.1 at (0.75, 0.25) holds only the
    middle Gauss point of the cell with x-index 1 and y-index 0, which is
    element 1 in x-fastest order (an x/y mix-up would hit element 2).  The
    next Gauss point is h * sqrt(15)/10 = 0.194 away."""
    g = Grid(2, 2, ri.ALL_DIRICHLET_2D)
    ref = RefElement(2)
    eta = A.viscosity(g, ref, g.elements(), 2.0, 7.0, [[0.75, 0.25, 0.1]])
    expect = np.full((4, 9), 2.0)
    expect[1, 4] = 7.0
    np.testing.assert_array_equal(eta, expect)


def test_viscosity_3d_closed_ball_and_overlap():
    """3D, N = 1: a ball of radius 0.45 at the cell centre holds the centre
    point and the six axis offsets (0.387) but no point two offsets away
    (0.548): 7 of the 27 points.  A second ball overlapping the first changes
    nothing (overlaps take eta_in).  Point (a, b, c) has index a + 3b + 9c."""
    g = Grid(3, 1, ri.ALL_DIRICHLET_3D)
    ref = RefElement(3)
    incl = [[0.5, 0.5, 0.5, 0.45], [0.5, 0.5, 0.5, 0.41]]
    eta = A.viscosity(g, ref, g.elements(), 1.0, 3.0, incl)
    inside = {13, 4, 22, 10, 16, 12, 14}
    expect = np.array([[3.0 if q in inside else 1.0 for q in range(27)]])
    np.testing.assert_array_equal(eta, expect)


def _identity_problem(n):
    L = sp.identity(n, format="csr")
    return L, np.ones(n, dtype=bool)


def test_lowp_sweep_rounds_residual_to_fp32():
    """L = I, x = 0, b = 1 + 2^-30: r = b, which rounds to 1.0 in FP32.  A
    one-DoF patch with W = [1] gives y = 1 exactly, so x becomes 1.0 (with an
    FP64 residual it would be 1 + 2^-30)."""
    L, free = _identity_problem(1)
    b = np.array([1.0 + 2.0 ** -30])
    x = sm.rav_sweep_rows_lowp(L, free, [np.array([0])], [np.array([0])],
                               [np.array([[1.0]], dtype=np.float32)], 1.0, np.zeros(1), b)
    assert x[0] == 1.0


def test_lowp_sweep_accumulates_in_fp32():
    """Two-DoF patch, owned row 0, W = [1, 1], r = (1, 2^-24): the FP32 sum
    1 + 2^-24 is a tie and rounds to even, 1.0, in either order; FP64
    accumulation would keep 1 + 2^-24.  omega = 0.5 then gives exactly 0.5."""
    L, free = _identity_problem(2)
    b = np.array([1.0, 2.0 ** -24])
    x = sm.rav_sweep_rows_lowp(L, free, [np.array([0, 1])], [np.array([0])],
                               [np.array([[1.0, 1.0]], dtype=np.float32)], 0.5, np.zeros(2), b)
    assert x[0] == 0.5 and x[1] == 0.0


def test_lowp_sweep_rounds_products_to_fp32():
    """One term w r with w = r = 1 + 2^-23 (both FP32 numbers): the exact
    product 1 + 2^-22 + 2^-46 rounds to 1 + 2^-22 in FP32."""
    L, free = _identity_problem(1)
    w = 1.0 + 2.0 ** -23
    x = sm.rav_sweep_rows_lowp(L, free, [np.array([0])], [np.array([0])],
                               [np.array([[w]], dtype=np.float32)], 1.0, np.zeros(1), np.array([w]))
    assert x[0] == 1.0 + 2.0 ** -22


def test_bf16_storage_ties_and_double_rounding():
    """RNE to bfloat16 (8 significant bits): 1 + 2^-8 is a tie between 1 and
    1 + 2^-7 and goes to 1; 1 + 3 * 2^-8 is a tie between 1 + 2^-7 and
    1 + 2^-6 and goes to 1 + 2^-6; 1 + 2^-8 + 2^-30 is first rounded to FP32
    (giving the tie 1 + 2^-8) and then to 1.  FP32 storage of 1 + 2^-30 is 1."""
    v = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -30, -(1 + 3 * 2.0 ** -8)])
    out = sm.round_storage(v, "bf16").astype(np.float64)
    np.testing.assert_array_equal(out, [1.0, 1 + 2.0 ** -6, 1.0, -(1 + 2.0 ** -6)])
    assert float(sm.round_storage(np.array([1 + 2.0 ** -30]), "fp32")[0]) == 1.0


def _element_buckets_3d(N):
    """(n_i, owned_i) histogram of all-Dirichlet 3D element patches by
    counting per axis: a cell at e has 3 - [e = 0] - [e = N-1] free velocity
    positions, owns 2 - [e = 0] of them (its nodes 2e, 2e+1, and 2e+2 when
    e = N-1, minus masked ones) and 1 + [e = N-1] pressure positions;
    n_i = 3 prod(c) + 8 and owned_i = 3 prod(o) + prod(p)."""
    hist = {}
    e = np.arange(N)
    c = 3 - (e == 0) - (e == N - 1)
    o = 2 - (e == 0)
    p = 1 + (e == N - 1)
    for i in range(N):
        for j in range(N):
            for k in range(N):
                key = (int(3 * c[i] * c[j] * c[k] + 8), int(3 * o[i] * o[j] * o[k] + p[i] * p[j] * p[k]))
                hist[key] = hist.get(key, 0) + 1
    return hist


def test_3d_element_bucket_histogram_64():
    """The 64^3 element-patch table: 62^3 interior (89, 25) patches, lower
    faces (62, 13), upper faces (62, 26), edges and corners; and the entry count
    sum_i owned_i n_i of the stored inverse rows, 558,683,224."""
    h = _element_buckets_3d(64)
    assert h[(89, 25)] == 238328 and h[(62, 13)] == 11532 and h[(62, 26)] == 11532
    assert h[(44, 14)] == 372 and h[(44, 7)] == 186 and h[(44, 28)] == 186
    assert sum(v for (n, _), v in h.items() if n == 32) == 8
    assert sum(h.values()) == 64 ** 3
    assert sum(n * o * v for (n, o), v in h.items()) == 558683224


@pytest.mark.parametrize("N", [4, 5])
def test_3d_patchset_matches_element_counting(N):
    g = Grid(3, N, ri.ALL_DIRICHLET_3D)
    ps = pt.PatchSet(g, pt.ELEMENT)
    hist = {}
    for I, own in zip(ps.dofs, ps.owned):
        key = (len(I), len(own))
        hist[key] = hist.get(key, 0) + 1
    assert hist == _element_buckets_3d(N)


def test_rav_mesh_independence_to_256():
    """RAV V(2,2), omega = 0.66, coarsest grid 8x8, N = 16 ... 256: the
    average reduction stays in a +-25 % band and the cycle count moves by at
    most 3 (about two minutes of CPU)."""
    rhos, its = [], []
    for N, nl in [(16, 2), (32, 3), (64, 4), (128, 5), (256, 6)]:
        H = mg.Hierarchy(2, N, nl, ri.ALL_DIRICHLET_2D)
        b = A.assemble_rhs(H.finest.grid, ri.mms_params(2, 1001))
        _, k, hist, st = H.solve(b)
        assert st == "converged"
        rhos.append(mg.avg_reduction(hist))
        its.append(k)
    mid = 0.5 * (max(rhos) + min(rhos))
    assert max(rhos) <= 1.25 * mid and min(rhos) >= 0.75 * mid, rhos
    assert max(its) - min(its) <= 3, its


def test_galerkin_equals_rediscretised_at_constant_viscosity():
    """For nested Q2/Q1 spaces and one viscosity the Galerkin triple product
    P^T L P reproduces the rediscretised coarse operator (exact quadrature on
    both grids)."""
    Hr = mg.Hierarchy(2, 16, 3, ri.ALL_DIRICHLET_2D)
    Hg = mg.Hierarchy(2, 16, 3, ri.ALL_DIRICHLET_2D, coarse="galerkin")
    for lr, lg in zip(Hr.levels, Hg.levels):
        assert abs(lr.L - lg.L).max() <= 1e-14 * abs(lr.L).max()


def _coarse_viscous_by_fine_quadrature(gc, R, eta_out, eta_in, incl):
    """Viscous block of a coarse grid integrated with the Gauss rules of the
    R x R fine cells inside each coarse cell, the coarse Q2 basis evaluated at
    those points (written here from the Lagrange basis, independently of the
    oracle's assembly)."""
    from oracle import fem
    n = gc.nn
    A = np.zeros((n * n, n * n))
    t = fem.GAUSS_T
    w = fem.GAUSS_W
    for ey in range(gc.N):
        for ex in range(gc.N):
            K = np.zeros((9, 9))
            for sy in range(R):
                for sx in range(R):
                    for qy in range(3):
                        for qx in range(3):
                            xi, yi = (sx + t[qx]) / R, (sy + t[qy]) / R
                            x = np.array([(ex + xi) * gc.h, (ey + yi) * gc.h])
                            eta = eta_out
                            for c in incl:
                                if (x[0] - c[0]) ** 2 + (x[1] - c[1]) ** 2 <= c[2] ** 2:
                                    eta = eta_in
                            vx, dx = fem.q2_1d([xi])[:, 0], fem.dq2_1d([xi])[:, 0]
                            vy, dy = fem.q2_1d([yi])[:, 0], fem.dq2_1d([yi])[:, 0]
                            gx = np.outer(vy, dx).ravel()   # local a = ax + 3 ay
                            gy = np.outer(dy, vx).ravel()
                            K += w[qx] * w[qy] / (R * R) * eta * (np.outer(gx, gx) + np.outer(gy, gy))
            nodes = [(2 * ey + ay) * n + (2 * ex + ax) for ay in range(3) for ax in range(3)]
            A[np.ix_(nodes, nodes)] += K
    return A


def test_galerkin_coarse_operator_is_fine_quadrature_form():
    """With an inclusion, P^T L P's viscous block on the 4x4 grid of an 8x8
    hierarchy (3 levels: the 2x2 grid too) equals the coarse form integrated
    by the Gauss points of the finest cells inside each coarse cell, on free
    DoFs: the identity the GPU assembly of Galerkin coarse levels uses."""
    incl = np.array([[0.4, 0.55, 0.23]])
    H = mg.Hierarchy(2, 8, 3, ri.OUTFLOW_2D, 0, 1.0, 30.0, incl, coarse="galerkin")
    for l, R in ((1, 2), (0, 4)):
        gc = H.levels[l].grid
        Ag = H.levels[l].L.toarray()[: gc.nV, : gc.nV]
        Aq = _coarse_viscous_by_fine_quadrature(gc, R, 1.0, 30.0, incl)
        fr = gc.free[: gc.nV]
        Aq = Aq[np.ix_(fr, fr)]
        assert np.abs(Ag[np.ix_(fr, fr)] - Aq).max() <= 1e-13 * np.abs(Aq).max(), l
        # and it differs from the rediscretised one (the inclusion is resolved differently)
        Ar = A.assemble_matrix(gc, 1.0, 30.0, incl).toarray()[: gc.nV, : gc.nV][np.ix_(fr, fr)]
        assert np.abs(Ar - Aq).max() > 1e-3 * np.abs(Aq).max()


def _twogrid_rho(N, contrast, incl, coarse, nu=2, omega=0.66, iters=30):
    """Asymptotic error reduction per RAV V(nu,nu) two-grid cycle (power
    iteration with b = 0, pressure constant removed)."""
    import scipy.linalg as sla
    H = mg.Hierarchy(2, N, 2, ri.ALL_DIRICHLET_2D, pt.VERTEX, 1.0, contrast, incl, coarse=coarse)
    g = H.finest.grid
    x = np.random.default_rng(0).standard_normal(g.n) * g.free
    s = g.pressure_slice()
    rs = []
    for _ in range(iters):
        x[s] -= x[s].mean()
        x /= np.linalg.norm(x)
        x = H.vcycle(x, np.zeros(g.n), "rav", omega, nu)
        x[s] -= x[s].mean()
        rs.append(np.linalg.norm(x))
    return float(np.exp(np.mean(np.log(rs[-8:]))))


def test_galerkin_cures_the_two_grid_divergence_at_contrast_1e3():
    """Finding behind the coarse-operator option: at viscosity contrast 1e3
    (the 1024^2 workload's inclusions on a 32x32 grid) the RAV two-grid cycle
    with the rediscretised coarse operator amplifies the error (about 10 per
    cycle), with the Galerkin operator it converges (about 0.65); at contrast 1
    both give the same rate."""
    incl = ri.inclusions(1005)
    r_re = _twogrid_rho(32, 1e3, incl, "rediscretised")
    r_ga = _twogrid_rho(32, 1e3, incl, "galerkin")
    assert r_re > 2.0 and r_ga < 0.8, (r_re, r_ga)
    r1 = _twogrid_rho(32, 1.0, incl, "rediscretised")
    r2 = _twogrid_rho(32, 1.0, incl, "galerkin")
    assert abs(r1 - r2) <= 1e-6 and r1 < 0.5


def test_dirichlet_lifting_reproduces_couette_flow():
    """Nonhomogeneous Dirichlet data through the lifting b = -L[free, masked] u_D:
    with u_D = (y, 0) on the whole boundary the Stokes solution is the linear
    shear flow u = (y, 0), p = const, which Q2 velocities represent exactly, so
    the discrete solution equals it at every free node (solved to 1e-12)."""
    N = 16
    H = mg.Hierarchy(2, N, 3, ri.ALL_DIRICHLET_2D)
    g = H.finest.grid
    uD = np.zeros(g.n)
    uD[: g.nV] = g.vnode[:, 1] / (2.0 * N)
    b = A.dirichlet_lifting(g, uD)
    assert abs(b[g.pressure_slice()].sum()) <= 1e-14   # no net flux through the boundary
    x, _, _, st = H.solve(b, rtol=1e-12)
    fr = g.free[: g.nV]
    assert st == "converged"
    assert np.abs(x[: g.nV][fr] - g.vnode[fr, 1] / (2.0 * N)).max() <= 1e-10
    assert np.abs(x[g.nV: 2 * g.nV][g.free[g.nV: 2 * g.nV]]).max() <= 1e-10
    assert np.ptp(x[g.pressure_slice()]) <= 1e-8


def test_lid_data_is_flux_free_and_only_on_the_lid():
    """Cavity data (Sec. 4.1): U on the top side's inner nodes, zero on the
    corners and the walls; its lifting has zero pressure sum (the lid moves
    tangentially) and touches only rows next to the top row of cells."""
    g = Grid(2, 8, ri.ALL_DIRICHLET_2D)
    u = A.lid_velocity(g, 2.5)
    vals = u[: g.nV].reshape(17, 17)
    assert np.all(vals[16, 1:16] == 2.5) and vals[16, 0] == 0.0 and vals[16, 16] == 0.0
    assert np.count_nonzero(u) == 15
    b = A.dirichlet_lifting(g, u)
    assert abs(b[g.pressure_slice()].sum()) <= 1e-14
    rows = np.nonzero(b)[0]
    vel = rows[rows < g.nV]
    assert np.all(g.vnode[vel, 1] >= 14)
    assert np.all(b[g.nV: 2 * g.nV] == 0.0)
