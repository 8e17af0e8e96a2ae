"""Stabilized Q1-Q1 on the adaptive cavity grids (Sec. 2, Fig. 2; Sec. 4.1,
Table 1) on the GPU against the oracle: on Omega^1..Omega^4 (7,059 DoFs), on
a randomly refined balanced hierarchy, and on a channel with an obstacle, an
inflow and an open outflow side (Sec. 4.2; no pressure constraint), the
residual of every grid, DoF counts, owner and patch maps, the stored local
inverses (RAV owned rows, AV/MV every row), transfers, the coarse solve,
RAV/AV/MV sweeps and V-cycles, the lid and Dirichlet-data right-hand sides,
and solves to 1e-8 with the oracle's cycle counts.  On the full hierarchy Omega^1..Omega^10
(3,063,075 DoFs, the paper's finest cavity grid) in the configuration the
benchmark times: the RAV V(3,3) solve reaches 1e-8, and the lid right-hand
side and the final residual agree on sampled rows with the oracle's rows,
each assembled from the leaves around its vertex."""
import numpy as np
import pytest

import rav_inputs as ri
from oracle import adaptive_mg as am
from oracle import mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2103_10127_amd.capi import AdaptiveHierarchy  # noqa: E402

BETA, ETA = 0.05, 1.0
N_GRIDS = 4
OMEGA = {"rav": 0.66, "mv": 0.66, "av": 0.1}
SM = {"rav": mg.RAV, "av": mg.AV, "mv": mg.MV}


@pytest.fixture(scope="module", params=["cavity", "random", "channel"])
def grids(request):
    """(grids, lattice_x, lattice_y, Dirichlet mask): the first four grids of
    Table 1, a randomly refined 2:1-balanced hierarchy (many hanging nodes,
    including constrained endpoints), and a small channel (16 x 3 coarse cells,
    a one-cell obstacle, refined towards the walls and the obstacle)."""
    if request.param == "cavity":
        M = ri.lattice(N_GRIDS)
        return ri.cavity_grids(N_GRIDS), M, M, ri.ALL_DIRICHLET_2D
    if request.param == "random":
        G, M = ri.random_quadtree_grids(N_GRIDS, base=8, frac=0.35, seed=1)
        return G, M, M, ri.ALL_DIRICHLET_2D
    G, Mx, My = ri.channel_grids(N_GRIDS, bands=(ri.UNIFORM, 1, 1), cells=(16, 3))
    return G, Mx, My, ri.OUTFLOW_2D


@pytest.fixture(scope="module")
def oracle(grids):
    G, Mx, My, dm = grids
    return am.AdaptiveHierarchy(G, Mx, BETA, ETA, My=My, dmask=dm)


def _gpu(grids, smoother="rav", nu=2):
    G, Mx, My, dm = grids
    print(f"[gpu] adaptive {len(G)} grids {Mx}x{My} mask {dm} {smoother} nu={nu}", flush=True)
    H = AdaptiveHierarchy(G, Mx, smoother=smoother, omega=OMEGA[smoother], nu_pre=nu, nu_post=nu, beta=BETA, eta=ETA,
                          lattice_y=My, dmask=dm)
    return H


def _rhs(g):
    """The benchmark's data: the driven cavity's lid, or the channel's
    parabolic inflow (eq. 14, mean velocity 0.3)."""
    return g.lid_rhs() if g.all_dirichlet else g.lifting(g.inflow_velocity(0.3))


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("table", ["lds", "global", "size-rule"])
def test_residual_dofs_and_owner_every_grid(grids, oracle, table, monkeypatch):
    if table != "size-rule":   # lds: the residual's table in LDS on every grid; global: nowhere
        monkeypatch.setenv("RAV_AD_TABLE_LDS", "1" if table == "lds" else "0")
    H = _gpu(grids)
    for l, lv in enumerate(oracle.levels):
        g = lv.grid
        n_total, n_free = H.dofs(l)
        assert (n_total, n_free) == (g.n, int(g.free.sum()))
        x = ri.random_vector(g.n, 140 + l) * g.free
        b = ri.random_vector(g.n, 150 + l) * g.free
        ro = b - lv.L @ x
        r = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        nrm = H.residual(l, _dev(x), _dev(b), r, norm=True)
        scale = np.abs(b) + abs(lv.L) @ np.abs(x)
        assert np.all(np.abs(r.cpu().numpy() - ro) <= 1e-13 * scale + 1e-300), l
        assert abs(nrm - np.linalg.norm(ro)) <= 1e-12 * np.linalg.norm(ro)
        own = H.owner(l).cpu().numpy()
        expect = np.concatenate([np.arange(g.nV)] * 3)
        expect[~g.free] = -1
        np.testing.assert_array_equal(own, expect)
    H.close()


@pytest.mark.parametrize("smoother", ["rav", "av", "mv"])
def test_patch_maps_and_inverses(grids, oracle, smoother):
    H = _gpu(grids, smoother)
    H.factor()
    for l in range(1, len(oracle.levels)):
        lv = oracle.levels[l]
        ps = lv.patches
        assert H.n_patches(l) == ps.count
        rng = np.random.default_rng(200 + l)
        sample = np.unique(np.concatenate([[0, ps.count - 1, ps.count // 2], rng.choice(ps.count, 40, replace=False)]))
        for k in sample:
            dofs, owned = H.patch_map(l, int(k))
            np.testing.assert_array_equal(dofs, ps.dofs[k])
            np.testing.assert_array_equal(np.nonzero(owned)[0], np.sort(ps.owned[k]))
            I = ps.dofs[k]
            Linv = np.linalg.inv(lv.L[I][:, I].toarray())
            W = H.patch_inverse(l, int(k))
            expect = Linv if smoother != "rav" else Linv[np.sort(ps.owned[k])]
            assert W.shape == expect.shape, (l, k)
            assert _rel(W, expect) <= 1e-12, (smoother, l, k, _rel(W, expect))
    H.close()


def test_transfers_and_coarse_solve(grids, oracle):
    H = _gpu(grids)
    for l in range(1, len(oracle.levels)):
        lv = oracle.levels[l]
        gf, gc = lv.grid, oracle.levels[l - 1].grid
        rf = ri.random_vector(gf.n, 161 + l) * gf.free
        bc = torch.zeros(gc.n, dtype=torch.float64, device="cuda")
        H.restrict(l, _dev(rf), bc)
        assert _rel(bc.cpu().numpy(), lv.P.T @ rf) <= 1e-14
        xc = ri.random_vector(gc.n, 162 + l) * gc.free
        xf = ri.random_vector(gf.n, 163 + l) * gf.free
        xfd = _dev(xf)
        H.prolong_add(l, _dev(xc), xfd)
        assert _rel(xfd.cpu().numpy(), xf + lv.P @ xc) <= 1e-14
    g0 = oracle.levels[0].grid
    b0 = ri.random_vector(g0.n, 164) * g0.free
    b0[g0.pressure_slice()] -= b0[g0.pressure_slice()].mean()
    x0 = torch.zeros(g0.n, dtype=torch.float64, device="cuda")
    H.coarse_solve(_dev(b0), x0)
    assert mg.rel_l2(g0, x0.cpu().numpy(), oracle.coarse_solve(b0)) <= 1e-11
    H.close()


def test_lid_rhs(grids, oracle):
    H = _gpu(grids)
    g = oracle.finest.grid
    b = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    H.assemble_rhs_lid(b, 1.5)
    bo = g.lid_rhs(1.5)
    assert np.abs(b.cpu().numpy() - bo).max() <= 1e-14 * np.abs(bo).max()
    H.close()


def test_dirichlet_rhs(grids, oracle):
    """rav_assemble_rhs_dirichlet against the oracle's lifting, for random
    data on the Dirichlet vertices (the library reads only those)."""
    H = _gpu(grids)
    g = oracle.finest.grid
    rng = np.random.default_rng(5)
    ud = rng.standard_normal((2, g.nV))
    u = np.zeros(g.n)
    u[: 2 * g.nV] = ud.reshape(-1)
    bo = g.lifting(np.where(g.free, 0.0, u))
    b = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    H.assemble_rhs_dirichlet(ud, b)
    assert np.abs(b.cpu().numpy() - bo).max() <= 1e-14 * np.abs(bo).max()
    with pytest.raises(ValueError):
        H.assemble_rhs_dirichlet(ud[:, :-1], b)
    H.close()


@pytest.mark.parametrize("smoother", ["rav", "av", "mv"])
def test_sweeps_and_vcycles(grids, oracle, smoother):
    H = _gpu(grids, smoother)
    H.factor()
    om = OMEGA[smoother]
    for l in range(1, len(oracle.levels)):
        g = oracle.levels[l].grid
        x = ri.random_vector(g.n, 171 + l) * g.free
        b = ri.random_vector(g.n, 172 + l) * g.free
        xd = _dev(x)
        H.smooth(l, 2, xd, _dev(b))
        xo = oracle.smooth(l, x, b, SM[smoother], om, 2)
        assert _rel(xd.cpu().numpy() - x, xo - x) <= 1e-12, (smoother, l)
    g = oracle.finest.grid
    bb = _rhs(g)
    bd = _dev(bb)
    xd = torch.zeros_like(bd)
    xo = np.zeros(g.n)
    for k in range(4):
        H.vcycle(xd, bd)
        xo = oracle.vcycle(xo, bb, SM[smoother], om, 2)
        e = mg.rel_l2(g, xd.cpu().numpy(), xo)
        assert e <= 1e-10, (smoother, k, e)
    H.close()


@pytest.mark.parametrize("table", ["lds", "global", "size-rule"])
@pytest.mark.parametrize("smoother", ["rav", "av", "mv"])
def test_solve_matches_oracle(grids, oracle, smoother, table, monkeypatch):
    """V(3,3) to 1e-8 (Sec. 4): the oracle's cycle count within 1 and the
    same solution within 1e-8, with the residual's value table in LDS, in
    global memory, and by the default size rule (global on these small grids,
    while MV keeps its table in LDS)."""
    if table != "size-rule":   # lds: the residual's table in LDS on every grid; global: nowhere
        monkeypatch.setenv("RAV_AD_TABLE_LDS", "1" if table == "lds" else "0")
    g = oracle.finest.grid
    b = _rhs(g)
    xo, ko, _, sto = oracle.solve(b, 1e-8, 200, SM[smoother], OMEGA[smoother], 3)
    H = _gpu(grids, smoother, nu=3)
    H.factor()
    bd = _dev(b)
    x = torch.zeros_like(bd)
    st, it, rel = H.solve(x, bd, 1e-8, 200)
    assert sto == "converged" and st == 0 and abs(it - ko) <= 1, (smoother, st, it, ko)
    assert mg.rel_l2(g, x.cpu().numpy(), xo) <= 1e-8
    H.close()


# ---- full hierarchies, sampled rows -------------------------------------------
def _regular_vertices(leaves, Mx):
    """Keys y (Mx + 1) + x of the regular vertices of a grid, sorted, which is
    the library's vertex order (y slowest): leaf corners that are not edge
    midpoints of another leaf."""
    x0, y0, s = (leaves[:, k].astype(np.int64) for k in range(3))
    h = s // 2
    key = lambda x, y: y * (Mx + 1) + x
    corners = np.unique(np.concatenate([key(x0 + a * s, y0 + b * s) for a in (0, 1) for b in (0, 1)]))
    mids = np.unique(np.concatenate([key(x0 + h, y0), key(x0 + h, y0 + s), key(x0, y0 + h), key(x0 + s, y0 + h)]))
    return np.setdiff1d(corners, mids, assume_unique=True)   # sorted: y slowest, x fastest


def _window(leaves, px, py, rings=3):
    """Leaves within `rings` rings of neighbours of the leaves at (px, py):
    enough for the rows of that vertex and the hanging nodes they involve."""
    x0, y0, s = leaves[:, 0], leaves[:, 1], leaves[:, 2]
    lx = hx = px
    ly = hy = py
    for _ in range(rings + 1):
        m = (x0 <= hx) & (x0 + s >= lx) & (y0 <= hy) & (y0 + s >= ly)
        lx, hx = x0[m].min(), (x0[m] + s[m]).max()
        ly, hy = y0[m].min(), (y0[m] + s[m]).max()
    return leaves[m]


def _nearest(xs_, ys, px, py):
    return int(np.argmin(np.abs(xs_ - px) + np.abs(ys - py)))


@pytest.mark.parametrize("case", ["cavity-omega10", "channel-omega7"])
def test_full_hierarchy_solve_sampled(case):
    """The configurations the benchmarks time: the cavity on Omega^1..Omega^10
    (3,063,075 DoFs) with its lid, and the channel on Omega^1..Omega^7
    (1,680,678 DoFs) with its parabolic inflow; RAV V(3,3) to 1e-8, then the
    right-hand side and the final residual on sampled vertices (random, and at
    the places where the data or the boundary change) against rows the oracle
    assembles from the leaves around each vertex."""
    if case.startswith("cavity"):
        n = 10
        G, Mx = ri.cavity_grids(n), ri.lattice(n)
        My, dm, n_expect = Mx, ri.ALL_DIRICHLET_2D, 3_063_075
    else:
        n = 7
        G, Mx, My = ri.channel_grids(n)
        dm, n_expect = ri.OUTFLOW_2D, 1_680_678
    print(f"[gpu] adaptive full hierarchy {case} ({n_expect} DoFs) RAV V(3,3)", flush=True)
    H = AdaptiveHierarchy(G, Mx, smoother="rav", omega=0.66, nu_pre=3, nu_post=3, beta=BETA, eta=ETA,
                          lattice_y=My, dmask=dm)
    H.factor()
    n_total, _ = H.dofs(n - 1)
    assert n_total == n_expect
    leaves = np.asarray(G[-1], dtype=np.int64)
    reg = _regular_vertices(leaves, Mx)
    nV = len(reg)
    assert 3 * nV == n_total
    ys, xs_ = reg // (Mx + 1), reg % (Mx + 1)
    b = torch.zeros(n_total, dtype=torch.float64, device="cuda")
    if case.startswith("cavity"):
        H.assemble_rhs_lid(b, 1.0)
    else:
        yy = ys / My
        ud = np.zeros((2, nV))
        ud[0] = np.where(xs_ == 0, 4.0 * 0.3 * yy * (1.0 - yy), 0.0)
        H.assemble_rhs_dirichlet(ud, b)
    x = torch.zeros_like(b)
    st, it, rel = H.solve(x, b, 1e-8, 100)
    print(f"[gpu]   {it} cycles, rel {rel:.2e}", flush=True)
    assert st == 0 and rel <= 1e-8, (st, it, rel)
    r = torch.zeros_like(b)
    rn = H.residual(n - 1, x, b, r, norm=True)
    b0, xs, rg = b.cpu().numpy(), x.cpu().numpy(), r.cpu().numpy()
    assert rn <= 1.01e-8 * np.linalg.norm(b0)
    rng = np.random.default_rng(97)
    if case.startswith("cavity"):
        special = [_nearest(xs_, ys, 1, My),              # next to the lid's left end
                   _nearest(xs_, ys, Mx // 2, My // 2),   # centre
                   _nearest(xs_, ys, Mx // 2, 1024)]      # a refinement transition
    else:
        s0 = Mx // 64                                     # coarse cell
        special = [_nearest(xs_, ys, 0, My // 2),         # inflow side
                   _nearest(xs_, ys, 1, My // 2),         # next to it
                   _nearest(xs_, ys, Mx, My // 2),        # outflow side (free velocity)
                   _nearest(xs_, ys, 4 * s0, 5 * s0),     # obstacle corner
                   _nearest(xs_, ys, 7 * s0, 6 * s0),     # obstacle corner
                   _nearest(xs_, ys, 5 * s0 + 1, 7 * s0)]  # obstacle top
    sample = np.unique(np.concatenate([rng.choice(nV, 40, replace=False), special]))
    for v in sample:
        px, py = int(xs_[v]), int(ys[v])
        g = am.AdaptiveGrid(_window(leaves, px, py), Mx, BETA, ETA, My=My, dmask=dm)
        i = g.reg_index[px * (My + 1) + py]
        Lw = g.assemble().tocsr()
        Law = g.assemble(keep_masked=True).tocsr()
        # window vertex -> library vertex
        wkey = g.ry * (Mx + 1) + g.rx
        gidx = np.minimum(np.searchsorted(reg, wkey), nV - 1)
        known = np.tile(reg[gidx] == wkey, 3)   # corners hanging in the full grid may look regular at the rim
        gcol = np.concatenate([gidx, nV + gidx, 2 * nV + gidx])
        uD = g.lid_velocity(1.0) if case.startswith("cavity") else g.inflow_velocity(0.3)
        for f in range(3):
            row, grow = f * g.nV + i, f * nV + v
            cols, vals = Lw.indices[Lw.indptr[row]:Lw.indptr[row + 1]], Lw.data[Lw.indptr[row]:Lw.indptr[row + 1]]
            assert known[cols].all(), (v, f)
            # right-hand side of this row: -L_all[row, masked] u_D
            ca, va = Law.indices[Law.indptr[row]:Law.indptr[row + 1]], Law.data[Law.indptr[row]:Law.indptr[row + 1]]
            bo = 0.0 if not g.free[row] else -np.sum(va * np.where(g.free[ca], 0.0, uD[ca]))
            assert abs(b0[grow] - bo) <= 1e-14 * max(1.0, abs(bo)), (v, f)
            ro = (b0[grow] - np.sum(vals * xs[gcol[cols]])) if g.free[row] else 0.0
            scale = abs(b0[grow]) + np.sum(np.abs(vals * xs[gcol[cols]]))
            assert abs(rg[grow] - ro) <= 1e-12 * scale + 1e-300, (v, f, rg[grow], ro)
    H.close()
