"""Batched RAV solves: problems of different sizes, level counts and viscosity
fields share every launch; each problem must behave exactly as if solved alone
(against single-problem contexts) and match the FP64 oracle."""
import numpy as np
import pytest

import rav_inputs as ri
from oracle import assemble as A
from oracle import mg
from oracle.grid import Grid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2103_10127_amd import Hierarchy  # noqa: E402
from paper_2103_10127_amd.capi import Batch  # noqa: E402


def _problems(sizes, coarsest=8, contrast=10.0):
    probs = []
    for i, N in enumerate(sizes):
        incl = ri.inclusions(2000 + i)
        probs.append(dict(dim=2, n_cells=N, n_levels=ri.levels_to(N, coarsest), dmask=ri.ALL_DIRICHLET_2D,
                          eta_out=1.0, eta_in=contrast, inclusions=incl, omega=0.66 if i % 2 == 0 else 0.6))
    return probs


def _rhs(p, i):
    g_n = 2 * (2 * p["n_cells"] + 1) ** 2 + (p["n_cells"] + 1) ** 2
    return ri.mms_params(2, 2000 + i), g_n


def test_batch_vcycle_equals_single_problem_vcycles():
    probs = _problems([16, 32, 64, 32, 16, 64])
    print("[gpu] batch create", flush=True)
    B = Batch(probs)
    B.factor()
    xs, bs, singles = [], [], []
    for i, p in enumerate(probs):
        params, n = _rhs(p, i)
        b = torch.zeros(n, dtype=torch.float64, device="cuda")
        B.assemble_rhs(i, params, b)
        bs.append(b)
        xs.append(torch.zeros_like(b))
    for _ in range(2):
        B.vcycle(xs, bs)
    for i, p in enumerate(probs):
        H = Hierarchy(dim=2, n_cells=p["n_cells"], n_levels=p["n_levels"], dmask=p["dmask"], omega=p["omega"],
                      eta_in=p["eta_in"], inclusions=p["inclusions"])
        H.factor()
        x = torch.zeros_like(bs[i])
        for _ in range(2):
            H.vcycle(x, bs[i])
        torch.cuda.synchronize()
        d = (xs[i] - x).norm().item() / x.norm().item()
        assert d <= 1e-12, (i, d)
        H.close()
    B.close()


def test_batch_solve_matches_oracle():
    probs = _problems([16, 32, 16, 32])
    B = Batch(probs)
    B.factor()
    xs, bs, bo = [], [], []
    for i, p in enumerate(probs):
        params, n = _rhs(p, i)
        b = torch.zeros(n, dtype=torch.float64, device="cuda")
        B.assemble_rhs(i, params, b)
        bs.append(b)
        xs.append(torch.zeros_like(b))
    st, its, rel = B.solve(xs, bs, 1e-8, 200)
    assert st == 0, (st, its, rel)
    for i, p in enumerate(probs):
        H = mg.Hierarchy(2, p["n_cells"], p["n_levels"], p["dmask"], 0, 1.0, p["eta_in"], p["inclusions"])
        g = H.finest.grid
        b = A.assemble_rhs(g, _rhs(p, i)[0])
        assert np.abs(bs[i].cpu().numpy() - b).max() <= 1e-12 * np.abs(b).max()
        xo, ko, hist, sto = H.solve(b, omega=p["omega"])
        assert sto == "converged" and abs(its[i] - ko) <= 1, (i, its[i], ko)
        assert rel[i] <= 1e-8
        assert mg.rel_l2(g, xs[i].cpu().numpy(), xo) <= 1e-7
    B.close()


def test_batch_rejects_mismatched_coarsest():
    from paper_2103_10127_amd.capi import RavError
    probs = _problems([16, 32])
    probs[1]["n_levels"] = 2   # coarsest 16 instead of 8
    with pytest.raises(RavError):
        Batch(probs)


def test_full_batch_vcycle_sampled_against_oracle():
    """The 256-problem batch workload as bench.py builds it (fine grids
    64/128/256, coarsest 16x16, 1-8 inclusions each at contrast 1e3): one
    batched V(2,2) cycle from x = 0, and for sampled 64x64 and 128x128
    problems the right-hand side and the iterate against the oracle's V-cycle."""
    cfg = ri.CONFIGS["batch256"]
    sizes = ri.batch_sizes(cfg["n_problems"], cfg["seed"])
    probs = [dict(dim=2, n_cells=int(n), n_levels=ri.levels_to(int(n), cfg["coarsest"]), dmask=cfg["dmask"],
                  eta_out=cfg["eta_out"], eta_in=cfg["contrast"], inclusions=ri.inclusions(cfg["seed"] + i),
                  omega=0.66) for i, n in enumerate(sizes)]
    print("[gpu] 256-problem batch create", flush=True)
    B = Batch(probs)
    B.factor()
    xs, bs = [], []
    for i, p in enumerate(probs):
        n, _ = B.dofs(i)
        b = torch.zeros(n, dtype=torch.float64, device="cuda")
        B.assemble_rhs(i, ri.mms_params(2, cfg["seed"] + i), b)
        bs.append(b)
        xs.append(torch.zeros_like(b))
    B.vcycle(xs, bs)
    torch.cuda.synchronize()
    picks = [int(np.nonzero(sizes == 64)[0][0]), int(np.nonzero(sizes == 64)[0][-1]),
             int(np.nonzero(sizes == 128)[0][0])]
    for i in picks:
        p = probs[i]
        print(f"[gpu] oracle problem {i} N={p['n_cells']}", flush=True)
        H = mg.Hierarchy(2, p["n_cells"], p["n_levels"], p["dmask"], 0, 1.0, p["eta_in"], p["inclusions"])
        g = H.finest.grid
        bo = A.assemble_rhs(g, ri.mms_params(2, cfg["seed"] + i))
        assert np.abs(bs[i].cpu().numpy() - bo).max() <= 1e-12 * np.abs(bo).max(), i
        xo = H.vcycle(np.zeros(g.n), bo, "rav", 0.66, 2)
        xg = xs[i].cpu().numpy()
        assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo), i
    B.close()


def _make(probs, precision="fp64"):
    for p in probs:
        p["precision"] = precision
    B = Batch(probs)
    B.factor()
    xs, bs = [], []
    for i, p in enumerate(probs):
        params, n = _rhs(p, i)
        b = torch.zeros(n, dtype=torch.float64, device="cuda")
        B.assemble_rhs(i, params, b)
        bs.append(b)
        xs.append(torch.zeros_like(b))
    return B, xs, bs


def test_batch_solve_replays_equal_eager_cycles():
    """rav_batch_solve replays one captured batched cycle per iteration; its
    iterates equal, bit for bit, those of eager rav_batch_vcycle calls (with
    eager launches and synchronizations between the replays)."""
    probs = _problems([16, 32, 64, 32])
    print("[gpu] batch graph replay", flush=True)
    B, xs, bs = _make(probs)
    for k in (1, 2, 4):
        for x in xs:
            x.zero_()
        st, its, _ = B.solve(xs, bs, 1e-300, k)
        assert all(it == k for it in its), its
        xe = [torch.zeros_like(b) for b in bs]
        for _ in range(k):
            B.vcycle(xe, bs)
        torch.cuda.synchronize()
        for i in range(len(xs)):
            assert torch.equal(xs[i], xe[i]), (k, i)
    B.close()


def test_batch_gmres_matches_oracle_fgmres():
    """Batched FGMRES(30) with one RAV V(2,2) cycle as preconditioner at
    contrast 1e3 (where plain V-cycles stagnate): every problem's cycle count
    is the oracle FGMRES's +-1 and its solution agrees to 1e-6."""
    from oracle import krylov
    probs = _problems([16, 32, 16, 32], contrast=1e3)
    print("[gpu] batch gmres", flush=True)
    B, xs, bs = _make(probs)
    st, its, rel = B.solve_gmres(xs, bs, 1e-8, 300, 30)
    assert st == 0 and max(rel) <= 1e-8, (st, its, rel)
    for i, p in enumerate(probs):
        H = mg.Hierarchy(2, p["n_cells"], p["n_levels"], p["dmask"], 0, 1.0, p["eta_in"], p["inclusions"])
        g = H.finest.grid
        b = A.assemble_rhs(g, _rhs(p, i)[0])
        Lf = H.finest.L

        def apply_L(v, Lf=Lf, g=g):
            y = Lf @ v
            y[~g.free] = 0.0
            return y

        xo, ko, _ = krylov.fgmres(apply_L, lambda r, H=H, g=g, om=p["omega"]: H.vcycle(np.zeros(g.n), r, "rav", om, 2),
                                  b, rtol=1e-8, restart=30, maxit=300)
        assert abs(its[i] - ko) <= 1, (i, its[i], ko)
        assert mg.rel_l2(g, xs[i].cpu().numpy(), xo) <= 1e-6, i
    B.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_mixed_precision_solve(prec):
    """FP32/BF16 inverse rows in a batch (contrast 10): every problem reaches
    1e-8 and its solution is within 1e-7 of the oracle's FP64 solve to 1e-12."""
    probs = _problems([16, 32, 64], contrast=10.0)
    print(f"[gpu] batch {prec}", flush=True)
    B, xs, bs = _make(probs, prec)
    st, its, rel = B.solve(xs, bs, 1e-8, 200)
    assert st == 0 and max(rel) <= 1e-8, (st, its, rel)
    for i, p in enumerate(probs):
        H = mg.Hierarchy(2, p["n_cells"], p["n_levels"], p["dmask"], 0, 1.0, p["eta_in"], p["inclusions"])
        g = H.finest.grid
        b = A.assemble_rhs(g, _rhs(p, i)[0])
        xo, _, _, sto = H.solve(b, rtol=1e-12, omega=p["omega"])
        assert mg.rel_l2(g, xs[i].cpu().numpy(), xo) <= 1e-7, i
    B.close()


def test_full_batch_gmres_reaches_tolerance():
    """The 256-problem workload (contrast 1e3) solved by the batched FGMRES(30)
    with one RAV V(4,4) cycle as preconditioner: at least 253 problems reach
    1e-8 within 300 cycles (measured: 253; with V(2,2) 186, V(3,3) 228: at this
    contrast the cycle amplifies some error components, see the design notes).
    For sampled converged problems of every size the true residual of the
    returned solution, recomputed with the oracle's assembled operator, is
    <= 1.01e-8 of the initial one."""
    cfg = ri.CONFIGS["batch256"]
    sizes = ri.batch_sizes(cfg["n_problems"], cfg["seed"])
    probs = [dict(dim=2, n_cells=int(n), n_levels=ri.levels_to(int(n), cfg["coarsest"]), dmask=cfg["dmask"],
                  eta_out=cfg["eta_out"], eta_in=cfg["contrast"], inclusions=ri.inclusions(cfg["seed"] + i),
                  omega=0.66, nu_pre=4, nu_post=4) for i, n in enumerate(sizes)]
    print("[gpu] 256-problem batch gmres", flush=True)
    B = Batch(probs)
    B.factor()
    xs, bs = [], []
    for i, p in enumerate(probs):
        n, _ = B.dofs(i)
        b = torch.zeros(n, dtype=torch.float64, device="cuda")
        B.assemble_rhs(i, ri.mms_params(2, cfg["seed"] + i), b)
        bs.append(b)
        xs.append(torch.zeros_like(b))
    st, its, rel = B.solve_gmres(xs, bs, 1e-8, 300, 30)
    rel = np.array(rel)
    ok = rel <= 1e-8
    assert st in (0, 1) and ok.sum() >= 253, (st, int(ok.sum()))
    picks = [int(np.nonzero((sizes == s) & ok)[0][0]) for s in (64, 128, 256)]
    for i in picks:
        p = probs[i]
        g = Grid(2, p["n_cells"], p["dmask"])
        L = A.assemble_matrix(g, 1.0, p["eta_in"], p["inclusions"])
        bo = bs[i].cpu().numpy()
        r = bo - L @ xs[i].cpu().numpy()
        r[~g.free] = 0.0
        assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(bo), (i, np.linalg.norm(r) / np.linalg.norm(bo))
    B.close()


def test_batch_call_aliases_give_identical_results(monkeypatch):
    """rav_create_batch / rav_solve_batch are the same calls as rav_batch_create /
    rav_batch_solve: the solutions agree bit for bit and so do the counts (the
    launch variants fixed by the size rule, so both batches run the same kernels)."""
    import ctypes
    monkeypatch.setenv("RAV_AUTOTUNE", "0")
    probs = _problems([16, 32])
    outs = []
    for alias in (False, True):
        B = Batch(probs)
        if alias:   # rebuild the batch through the alias entry point
            B.close()
            h = ctypes.c_void_p()
            st = B.lib.rav_create_batch(B.descs, len(probs), B.stream, ctypes.byref(h))
            assert st == 0
            B.h = h
        B.factor()
        xs, bs = [], []
        for i, p in enumerate(probs):
            params, n = _rhs(p, i)
            b = torch.zeros(n, dtype=torch.float64, device="cuda")
            B.assemble_rhs(i, params, b)
            bs.append(b)
            xs.append(torch.zeros_like(b))
        its = (ctypes.c_int * len(probs))()
        rel = (ctypes.c_double * len(probs))()
        fn = B.lib.rav_solve_batch if alias else B.lib.rav_batch_solve
        st = fn(B.h, B._ptrs(xs), B._ptrs(bs), 1e-8, 200, its, rel)
        assert st == 0
        outs.append(([x.cpu().numpy() for x in xs], list(its)))
        B.close()
    for a, b in zip(outs[0][0], outs[1][0]):
        np.testing.assert_array_equal(a, b)
    assert outs[0][1] == outs[1][1]
