"""GPU parity of the HIP path (through the C-ABI) against the FP64 CPU oracle.

Bars: integer maps bit-exact; FP64 kernels <= 1e-12 relative (single
operations) and <= 1e-10 relative L2 for V-cycle iterates (first cycles);
mixed-precision solutions <= 1e-7 relative L2 against the oracle solved to a
1e-12 reduction.  Sizes are chosen so the oracle finishes in seconds while the
launches still span several tiles with ragged tails.
"""
import numpy as np
import pytest

import rav_inputs as ri
from oracle import assemble as A
from oracle import mg
from oracle import patches as pt
from oracle import smoothers as sm
from oracle.grid import Grid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2103_10127_amd import Hierarchy  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


CASES = {
    "2d-vertex-dir": dict(dim=2, N=8, nl=2, kind="vertex", dm=ri.ALL_DIRICHLET_2D, incl=None, eta_in=1.0),
    "2d-vertex-out-incl": dict(dim=2, N=12, nl=2, kind="vertex", dm=ri.OUTFLOW_2D,
                               incl=np.array([[0.3, 0.6, 0.2]]), eta_in=1e3),
    "2d-vertex-40": dict(dim=2, N=40, nl=3, kind="vertex", dm=ri.ALL_DIRICHLET_2D, incl=None, eta_in=1.0),
    "3d-element-dir": dict(dim=3, N=4, nl=2, kind="element", dm=ri.ALL_DIRICHLET_3D, incl=None, eta_in=1.0),
    "3d-element-out-incl": dict(dim=3, N=4, nl=2, kind="element", dm=ri.OUTFLOW_3D,
                                incl=np.array([[0.4, 0.5, 0.5, 0.3]]), eta_in=50.0),
    "2d-element-dir": dict(dim=2, N=10, nl=2, kind="element", dm=ri.ALL_DIRICHLET_2D, incl=None, eta_in=1.0),
}
SMALL = ["2d-vertex-dir", "2d-vertex-out-incl", "3d-element-dir", "3d-element-out-incl", "2d-element-dir"]


def _okind(kind):
    return pt.VERTEX if kind == "vertex" else pt.ELEMENT


def _gpu(case, smoother="rav", precision="fp64", omega=0.66, nu=2):
    c = CASES[case]
    print(f"[gpu] create {case} smoother={smoother} prec={precision}", flush=True)
    return Hierarchy(dim=c["dim"], n_cells=c["N"], n_levels=c["nl"], dmask=c["dm"], kind=c["kind"],
                     smoother=smoother, omega=omega, nu_pre=nu, nu_post=nu, precision=precision,
                     eta_in=c["eta_in"], inclusions=c["incl"])


def _oracle(case):
    c = CASES[case]
    return mg.Hierarchy(c["dim"], c["N"], c["nl"], c["dm"], _okind(c["kind"]), 1.0, c["eta_in"], c["incl"])


@pytest.mark.parametrize("case", SMALL)
def test_operator_matches_oracle(case):
    c = CASES[case]
    gh = _gpu(case)
    for level in range(c["nl"]):
        N = c["N"] >> (c["nl"] - 1 - level)
        g = Grid(c["dim"], N, c["dm"])
        Lo = A.assemble_matrix(g, 1.0, c["eta_in"], c["incl"]).toarray()
        Lg = gh.export_matrix(level)
        assert np.abs(Lg - Lo).max() <= 1e-13 * np.abs(Lo).max(), (case, level)
    gh.close()


@pytest.mark.parametrize("dim,N,nl,seed", [(2, 24, 2, 1001), (3, 4, 2, 1003)])
def test_rhs_matches_oracle(dim, N, nl, seed):
    dm = ri.ALL_DIRICHLET_2D if dim == 2 else ri.ALL_DIRICHLET_3D
    params = ri.mms_params(dim, seed, eta=1.3)
    g = Grid(dim, N, dm)
    bo = A.assemble_rhs(g, params)
    gh = Hierarchy(dim=dim, n_cells=N, n_levels=nl, dmask=dm, kind="vertex" if dim == 2 else "element")
    bd = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    gh.assemble_rhs(params, bd)
    assert np.abs(host(bd) - bo).max() <= 1e-12 * np.abs(bo).max()
    gh.close()


@pytest.mark.parametrize("dm", [ri.ALL_DIRICHLET_2D, ri.OUTFLOW_2D])
def test_residual_large_2d_levels(dm):
    """Level N = 512 takes the LDS-tiled residual, N = 128 and 256 the node-type
    one: every row against the oracle, with inclusions at contrast 1e3 (cut
    cells in interior and last tiles), an open side, and x nonzero on masked
    nodes (masked columns must contribute nothing)."""
    incl = ri.inclusions(1234)
    print(f"[gpu] tiled residual dm={dm}", flush=True)
    gh = Hierarchy(dim=2, n_cells=512, n_levels=7, dmask=dm, eta_in=1e3, inclusions=incl)
    for level in (4, 5, 6):
        lv = mg.Level(2, 512 >> (6 - level), dm, pt.VERTEX, 1.0, 1e3, incl, smooth=False)
        g = lv.grid
        x = ri.random_vector(g.n, 40 + level)
        b = ri.random_vector(g.n, 50 + level) * g.free
        ro = sm.residual(lv.L, x, b, g.free)
        rd = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        nrm = gh.residual(level, dev(x), dev(b), rd, norm=True)
        assert rel(host(rd), ro) <= 1e-13, level
        assert abs(nrm - np.linalg.norm(ro)) <= 1e-12 * np.linalg.norm(ro), level
    gh.close()


@pytest.mark.parametrize("case", SMALL + ["2d-vertex-40"])
def test_residual_and_norm(case):
    c = CASES[case]
    H = _oracle(case)
    gh = _gpu(case)
    for level in range(c["nl"]):
        lv = H.levels[level]
        g = lv.grid
        x = ri.random_vector(g.n, 10 + level) * g.free
        b = ri.random_vector(g.n, 20 + level) * g.free
        ro = sm.residual(lv.L, x, b, g.free)
        rd = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        nrm = gh.residual(level, dev(x), dev(b), rd, norm=True)
        assert rel(host(rd), ro) <= 1e-13
        assert abs(nrm - np.linalg.norm(ro)) <= 1e-12 * np.linalg.norm(ro)
    gh.close()


@pytest.mark.parametrize("case", SMALL + ["2d-vertex-40"])
def test_device_owner_map_bit_exact(case):
    c = CASES[case]
    gh = _gpu(case)
    for level in range(c["nl"]):
        N = c["N"] >> (c["nl"] - 1 - level)
        g = Grid(c["dim"], N, c["dm"])
        own = gh.owner(level).cpu().numpy()
        np.testing.assert_array_equal(own, pt.owner_of_dofs(g, _okind(c["kind"])))
    gh.close()


@pytest.mark.parametrize("case", SMALL + ["2d-vertex-40"])
@pytest.mark.parametrize("smoother", ["rav", "av"])
def test_patch_inverses(case, smoother):
    c = CASES[case]
    H = _oracle(case)
    gh = _gpu(case, smoother=smoother)
    gh.factor()
    lv = H.levels[-1]
    ps = lv.patches
    rng = np.random.default_rng(0)
    sample = np.unique(np.concatenate([[0, ps.count - 1], rng.choice(ps.count, min(40, ps.count), replace=False)]))
    for i in sample:
        n = len(ps.dofs[i])
        if smoother == "rav":
            Wo = sm.owned_rows(lv.lus[i], ps.owned[i], n)
        else:
            Wo = sm.full_inverse(lv.lus[i], n)
        Wg = gh.patch_inverse(c["nl"] - 1, int(i))
        assert Wg.shape == Wo.shape, (i, Wg.shape, Wo.shape)
        assert rel(Wg, Wo) <= 1e-12, (case, i, rel(Wg, Wo))
    gh.close()


@pytest.mark.parametrize("case", SMALL + ["2d-vertex-40"])
@pytest.mark.parametrize("smoother", ["rav", "av", "mv"])
def test_one_sweep(case, smoother):
    c = CASES[case]
    H = _oracle(case)
    omega = 0.66 if smoother != "av" else 0.3
    gh = _gpu(case, smoother=smoother, omega=omega)
    gh.factor()
    level = c["nl"] - 1
    lv = H.levels[level]
    g = lv.grid
    x = ri.random_vector(g.n, 31) * g.free
    b = ri.random_vector(g.n, 32) * g.free
    xd = dev(x)
    gh.smooth(level, 1, xd, dev(b))
    xo = H.smooth(level, x, b, smoother, omega, 1)
    assert rel(host(xd) - x, xo - x) <= 1e-12, (case, smoother)
    gh.close()


@pytest.mark.parametrize("case", SMALL + ["2d-vertex-40"])
def test_transfers(case):
    c = CASES[case]
    H = _oracle(case)
    gh = _gpu(case)
    for level in range(1, c["nl"]):
        lf, lc = H.levels[level], H.levels[level - 1]
        rf = ri.random_vector(lf.grid.n, 41) * lf.grid.free
        bc = torch.zeros(lc.grid.n, dtype=torch.float64, device="cuda")
        gh.restrict(level, dev(rf), bc)
        assert rel(host(bc), lf.P.T @ rf) <= 1e-14
        xc = ri.random_vector(lc.grid.n, 42) * lc.grid.free
        xf = ri.random_vector(lf.grid.n, 43) * lf.grid.free
        xfd = dev(xf)
        gh.prolong_add(level, dev(xc), xfd)
        assert rel(host(xfd), xf + lf.P @ xc) <= 1e-14
    gh.close()


@pytest.mark.parametrize("case", SMALL)
def test_coarse_solve(case):
    H = _oracle(case)
    gh = _gpu(case)
    g = H.levels[0].grid
    b = ri.random_vector(g.n, 51) * g.free
    b[g.pressure_slice()] -= b[g.pressure_slice()].mean()
    xd = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    gh.coarse_solve(dev(b), xd)
    assert rel(host(xd), H.coarse_solve(b)) <= 1e-10
    gh.close()


@pytest.mark.parametrize("case", ["2d-vertex-dir", "2d-vertex-out-incl", "2d-vertex-40", "3d-element-dir",
                                  "3d-element-out-incl"])
@pytest.mark.parametrize("smoother", ["rav", "mv", "av"])
def test_vcycle_iterates(case, smoother):
    """First cycles of V(2,2) from x0 = 0 agree to <= 1e-10 relative L2."""
    c = CASES[case]
    H = _oracle(case)
    omega = 0.66 if smoother != "av" else 0.1
    gh = _gpu(case, smoother=smoother, omega=omega)
    gh.factor()
    g = H.finest.grid
    dim = c["dim"]
    params = ri.mms_params(dim, 1001 if dim == 2 else 1003)
    b = A.assemble_rhs(g, params)
    bd = dev(b)
    x = np.zeros(g.n)
    xd = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    ncyc = 10 if c["N"] <= 12 or dim == 3 else 6
    for k in range(ncyc):
        gh.vcycle(xd, bd)
        x = H.vcycle(x, b, smoother, omega, 2)
        e = mg.rel_l2(g, host(xd), x)
        assert e <= 1e-10, (case, smoother, k, e)
    gh.close()


def test_solve_32_all_smoothers():
    """2D 32x32, 3 levels: iteration counts equal the oracle's and the FP64
    solutions agree; ordering MV <= RAV < AV(0.1) holds on the GPU too."""
    cfg = ri.CONFIGS["2d-32"]
    H = mg.Hierarchy(2, 32, 3, cfg["dmask"])
    g = H.finest.grid
    params = ri.mms_params(2, cfg["seed"])
    b = A.assemble_rhs(g, params)
    bd = dev(b)
    its = {}
    for smoother, omega in [("rav", 0.66), ("mv", 0.66), ("av", 0.1)]:
        gh = Hierarchy(dim=2, n_cells=32, n_levels=3, dmask=cfg["dmask"], smoother=smoother, omega=omega)
        gh.factor()
        xd = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        st, it, rr = gh.solve(xd, bd, 1e-8, 300)
        xo, ko, hist, sto = H.solve(b, smoother=smoother, omega=omega, maxit=300)
        assert st == 0 and sto == "converged"
        assert abs(it - ko) <= 1, (smoother, it, ko)
        assert mg.rel_l2(g, host(xd), xo) <= 1e-8
        its[smoother] = it
        gh.close()
    assert its["mv"] <= its["rav"] < its["av"]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_precision_solution(prec):
    """FP32/BF16 inverse rows: the FP64 outer cycle still reaches 1e-8 and the
    solution matches the oracle solved to 1e-12 within 1e-7."""
    H = mg.Hierarchy(2, 40, 3, ri.ALL_DIRICHLET_2D)
    g = H.finest.grid
    b = A.assemble_rhs(g, ri.mms_params(2, 1002))
    xref, _, _, _ = H.solve(b, rtol=1e-12)
    gh = Hierarchy(dim=2, n_cells=40, n_levels=3, precision=prec)
    gh.factor()
    xd = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    st, it, rr = gh.solve(xd, dev(b), 1e-8, 200)
    assert st == 0 and rr <= 1e-8
    assert mg.rel_l2(g, host(xd), xref) <= 1e-7
    gh.close()


def _storage_ulp(W, prec):
    """Spacing of the storage format at |W_ij|: 2^(e - 23) for FP32, 2^(e - 7)
    for BF16, e = floor(log2 |W_ij|); 0 where W_ij = 0."""
    a = np.abs(np.asarray(W, dtype=np.float64))
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    ulp = np.exp2(e - (23 if prec == "fp32" else 7))
    return np.where(a > 0, ulp, 0.0)


def test_low_precision_rows_are_rounded_fp64_rows():
    """Stored FP32/BF16 rows equal the FP64 rows rounded once (RNE)."""
    H = _oracle("2d-vertex-dir")
    lv = H.levels[-1]
    ps = lv.patches
    for prec in ("fp32", "bf16"):
        gh = _gpu("2d-vertex-dir", precision=prec)
        gh.factor()
        for i in range(0, ps.count, 7):
            Wo = sm.owned_rows(lv.lus[i], ps.owned[i], len(ps.dofs[i]))
            Wg = gh.patch_inverse(1, i)
            # per entry: at most one storage ulp of |W_ij| (a rounding decision
            # may flip where the GPU's FP64 row differs from the oracle's in
            # the last bits), plus that FP64 difference for tiny entries
            expect = sm.round_storage(Wo, prec).astype(np.float64)
            ulp = _storage_ulp(Wo, prec)
            tol = ulp + 1e-12 * np.abs(Wo).max()
            assert np.all(np.abs(Wg - expect) <= tol), (prec, i, np.max(np.abs(Wg - expect) / tol))
        gh.close()
