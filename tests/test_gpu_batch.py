"""Batched RAV solves: problems of different sizes, level counts and viscosity
fields share every launch; each problem must behave exactly as if solved alone
(against single-problem contexts) and match the FP64 oracle."""
import numpy as np
import pytest

import rav_inputs as ri
from oracle import assemble as A
from oracle import mg

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
