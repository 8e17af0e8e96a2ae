"""Full-size parity on the 3D workload (Q2/Q1 64x64x64, 5 levels, RAV element
patches, all-Dirichlet velocity): sampled outputs that the oracle computes one
by one from its row-wise assembly, its element load vectors and its 1D
interpolation matrices (the full 6.7M-DoF operator is not formed).  A second
64^3 grid with a natural boundary on x = 1 and spherical inclusions at
viscosity contrast 1e3 checks the residual rows that take the general path of
the tiled kernel (boundary nodes with missing cells, cut cells)."""
import numpy as np
import pytest
import scipy.linalg as sla

import rav_inputs as ri
from oracle import assemble as A
from oracle import mms
from oracle import patches as pt
from oracle import transfer
from oracle.fem import RefElement
from oracle.grid import Grid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2103_10127_amd import Hierarchy  # noqa: E402

N, NL = 64, 5
DM = ri.ALL_DIRICHLET_3D
OMEGA = 0.5


@pytest.fixture(scope="module")
def h3d():
    print("[gpu] full-size 3D 64^3 element-patch hierarchy", flush=True)
    G = Hierarchy(dim=3, n_cells=N, n_levels=NL, dmask=DM, kind="element", omega=OMEGA)
    G.factor()
    yield G
    G.close()


@pytest.fixture(scope="module")
def grid():
    return Grid(3, N, DM)


def _row_dot(row, x):
    return sum(v * x[c] for c, v in row.items())


def test_rhs_sampled_rows(h3d, grid):
    g = grid
    params = ri.mms_params(3, ri.CONFIGS["3d-64"]["seed"])
    b = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    h3d.assemble_rhs(params, b)
    bg = b.cpu().numpy()
    ref = RefElement(3)
    rng = np.random.default_rng(81)
    rows = rng.choice(3 * g.nV, 200, replace=False)
    scale = np.abs(bg).max()
    for row in rows:
        if not g.free[row]:
            assert bg[row] == 0.0
            continue
        c, a = row // g.nV, g.vnode[row % g.nV]
        lo, hi = np.maximum((a - 1) // 2, 0), np.minimum(a // 2, N - 1)
        mesh = np.meshgrid(*[np.arange(lo[i], hi[i] + 1) for i in range(3)], indexing="ij")
        elems = np.stack([m.ravel() for m in mesh], axis=1)
        f = mms.forcing(params, A.quad_positions(g, ref, elems))
        be = ref.load(g.h, np.moveaxis(f, 2, 1))
        vd, _ = A.element_dofs(g, ref, elems)
        expect = be[:, c][vd[:, c] == row].sum()
        assert abs(bg[row] - expect) <= 1e-12 * scale, row


def test_residual_sampled_rows(h3d, grid):
    g = grid
    x = ri.random_vector(g.n, 82) * g.free
    b = ri.random_vector(g.n, 83) * g.free
    r = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    h3d.residual(NL - 1, torch.from_numpy(x).cuda(), torch.from_numpy(b).cuda(), r)
    rg = r.cpu().numpy()
    rng = np.random.default_rng(84)
    for i in np.concatenate([rng.choice(g.n, 300, replace=False), _rows_on_planes(g, rng, 1000)]):
        row = A.matrix_row(g, int(i))
        ro = b[i] - _row_dot(row, x) if g.free[i] else 0.0
        amax = max(1.0, np.abs(list(row.values()) or [1]).max())
        assert abs(rg[i] - ro) <= 1e-12 * (1 + abs(ro)) * amax, i


def _rows_on_planes(g, rng, count):
    """Velocity and pressure rows on the x = 0 and x = 1 sides and on the
    seams between 8 x 8 x 4-cell tiles (cell index multiples of 8, 8, 4)."""
    out = []
    for _ in range(count):
        kind = rng.integers(0, 4)
        a = rng.integers(0, 2 * N + 1, 3)
        if kind == 0:
            a[0] = rng.choice([0, 1, 2, 2 * N - 2, 2 * N - 1, 2 * N])
        elif kind == 1:
            d = rng.integers(0, 3)
            step = 8 if d < 2 else 4
            a[d] = min(2 * N, 2 * step * rng.integers(0, N // step + 1) + rng.integers(-2, 3))
            a[d] = max(a[d], 0)
        if kind == 3:
            k = a // 2
            if rng.integers(0, 2):
                k[0] = rng.choice([0, N])
            out.append(g.pres(k))
        else:
            out.append(g.vel(int(rng.integers(0, 3)), a))
    return np.asarray(out)


@pytest.fixture(scope="module")
def h3d_incl():
    print("[gpu] 64^3 grid, outflow side, spherical inclusions at contrast 1e3", flush=True)
    G = Hierarchy(dim=3, n_cells=N, n_levels=NL, dmask=ri.OUTFLOW_3D, kind="element", omega=OMEGA,
                  eta_in=1e3, inclusions=ri.spheres(1004))
    yield G
    G.close()


def test_residual_rows_outflow_and_inclusions(h3d_incl):
    incl = ri.spheres(1004)
    g = Grid(3, N, ri.OUTFLOW_3D)
    eta = A.viscosity(g, RefElement(3), g.elements(), 1.0, 1e3, incl)
    cut = np.nonzero(eta.min(1) != eta.max(1))[0]
    assert len(cut) > 100
    x = ri.random_vector(g.n, 92) * g.free
    b = ri.random_vector(g.n, 93) * g.free
    r = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    h3d_incl.residual(NL - 1, torch.from_numpy(x).cuda(), torch.from_numpy(b).cuda(), r)
    rg = r.cpu().numpy()
    rng = np.random.default_rng(94)
    near = []
    for e in rng.choice(cut, 1000):
        ec = np.array([e % N, (e // N) % N, e // (N * N)])
        near.append(g.vel(int(rng.integers(0, 3)), 2 * ec + rng.integers(0, 3, 3)))
    rows = np.concatenate([rng.choice(g.n, 1000, replace=False), near, _rows_on_planes(g, rng, 1500)])
    for i in rows:
        row = A.matrix_row(g, int(i), 1.0, 1e3, incl)
        ro = b[i] - _row_dot(row, x) if g.free[i] else 0.0
        amax = max(1.0, np.abs(list(row.values()) or [1]).max())
        assert abs(rg[i] - ro) <= 1e-12 * (1 + abs(ro)) * amax, i


def _patch_system(g, p):
    I = pt.patch_dofs(g, pt.ELEMENT, int(p))
    rows = {i: A.matrix_row(g, int(i)) for i in I}
    Li = np.array([[rows[i].get(j, 0.0) for j in I] for i in I])
    return I, rows, Li


def _sample_patches(rng):
    # every class of element (interior, faces, edges and the corner at the top boundary)
    corners = [(0, 0, 0), (N - 1, 0, 0), (0, N - 1, 0), (0, 0, N - 1), (N - 1, N - 1, 0),
               (N - 1, 0, N - 1), (0, N - 1, N - 1), (N - 1, N - 1, N - 1), (31, 17, 40)]
    fixed = [e[0] + N * (e[1] + N * e[2]) for e in corners]
    return np.concatenate([fixed, rng.choice(N ** 3, 8, replace=False)])


def test_patch_inverse_rows_sampled(h3d, grid):
    g = grid
    owner = pt.owner_of_dofs(g, pt.ELEMENT)
    for p in _sample_patches(np.random.default_rng(85)):
        I, _, Li = _patch_system(g, p)
        own = np.nonzero(owner[I] == p)[0]
        Wo = np.linalg.inv(Li)[own]
        Wg = h3d.patch_inverse(NL - 1, int(p))
        assert Wg.shape == Wo.shape, p
        assert np.linalg.norm(Wg - Wo) <= 1e-11 * np.linalg.norm(Wo), p


def test_one_sweep_sampled(h3d, grid):
    g = grid
    owner = pt.owner_of_dofs(g, pt.ELEMENT)
    x = ri.random_vector(g.n, 86) * g.free
    b = ri.random_vector(g.n, 87) * g.free
    xd = torch.from_numpy(x).cuda()
    h3d.smooth(NL - 1, 1, xd, torch.from_numpy(b).cuda())
    xg = xd.cpu().numpy()
    rng = np.random.default_rng(88)
    free = np.nonzero(g.free)[0]
    for d in rng.choice(free, 20, replace=False):
        p = owner[d]
        I, rows, Li = _patch_system(g, p)
        r_i = np.array([b[i] - _row_dot(rows[i], x) for i in I])
        y = sla.lu_solve(sla.lu_factor(Li), r_i)
        loc = int(np.nonzero(I == d)[0][0])
        expect = x[d] + OMEGA * y[loc]
        assert abs(xg[d] - expect) <= 1e-10 * max(1.0, abs(y[loc])), d
    assert np.all(xg[~g.free] == 0.0)


def _p_entry_tables(gc):
    return transfer.interp_1d_q2(gc.N), transfer.interp_1d_q1(gc.N)


def test_transfers_sampled(h3d, grid):
    """Sampled entries of P^T r and P x_c, each a tensor product of the
    oracle's 1D interpolation matrices (P = kron over dimensions, masked)."""
    gf, gc = grid, Grid(3, N // 2, DM)
    Pq, Pl = _p_entry_tables(gc)
    rng = np.random.default_rng(89)
    rf = ri.random_vector(gf.n, 90) * gf.free
    bc = torch.zeros(gc.n, dtype=torch.float64, device="cuda")
    h3d.restrict(NL - 1, torch.from_numpy(rf).cuda(), bc)
    bcg = bc.cpu().numpy()
    for i in rng.choice(gc.n, 150, replace=False):
        if i < 3 * gc.nV:
            c, Anode = i // gc.nV, gc.vnode[i % gc.nV]
            cols = [np.nonzero(Pq[:, Anode[d]])[0] for d in range(3)]
            w = [Pq[cols[d], Anode[d]] for d in range(3)]
            fi = [gf.vel(c, np.array([ax, ay, az])) for az in cols[2] for ay in cols[1] for ax in cols[0]]
        else:
            K = gc.pnode[i - 3 * gc.nV]
            cols = [np.nonzero(Pl[:, K[d]])[0] for d in range(3)]
            w = [Pl[cols[d], K[d]] for d in range(3)]
            fi = [gf.pres(np.array([ax, ay, az])) for az in cols[2] for ay in cols[1] for ax in cols[0]]
        ww = np.einsum("i,j,k->kji", w[0], w[1], w[2]).ravel()
        expect = float(np.dot(ww, rf[np.array(fi)])) if gc.free[i] else 0.0
        assert abs(bcg[i] - expect) <= 1e-13 * 8 * np.abs(rf).max(), i
    xc = ri.random_vector(gc.n, 91) * gc.free
    xf = torch.zeros(gf.n, dtype=torch.float64, device="cuda")
    h3d.prolong_add(NL - 1, torch.from_numpy(xc).cuda(), xf)
    xfg = xf.cpu().numpy()
    for j in rng.choice(gf.n, 150, replace=False):
        if j < 3 * gf.nV:
            c, a = j // gf.nV, gf.vnode[j % gf.nV]
            rows = [np.nonzero(Pq[a[d]])[0] for d in range(3)]
            w = [Pq[a[d], rows[d]] for d in range(3)]
            ci = [gc.vel(c, np.array([ax, ay, az])) for az in rows[2] for ay in rows[1] for ax in rows[0]]
        else:
            k = gf.pnode[j - 3 * gf.nV]
            rows = [np.nonzero(Pl[k[d]])[0] for d in range(3)]
            w = [Pl[k[d], rows[d]] for d in range(3)]
            ci = [gc.pres(np.array([ax, ay, az])) for az in rows[2] for ay in rows[1] for ax in rows[0]]
        ww = np.einsum("i,j,k->kji", w[0], w[1], w[2]).ravel()
        expect = float(np.dot(ww, xc[np.array(ci)])) if gf.free[j] else 0.0
        assert abs(xfg[j] - expect) <= 1e-13 * 4 * np.abs(xc).max(), j
