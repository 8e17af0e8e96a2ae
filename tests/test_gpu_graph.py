"""The solve loop replays one captured V-cycle per iteration (stream capture,
RAV_GRAPH=0 switches it off).  Its iterates must equal, bit for bit, those of
the eagerly launched V-cycle entry point on the same problem, with eager
launches and synchronizations between the replays; changing the cycle
parameters must drop the captured cycle."""
import numpy as np
import pytest

import rav_inputs as ri

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2103_10127_amd import Hierarchy  # noqa: E402


def _problem(dim, n, nl, dm, kind):
    H = Hierarchy(dim=dim, n_cells=n, n_levels=nl, dmask=dm, kind=kind, omega=0.66 if kind == "vertex" else 0.5)
    H.factor()
    nf = H.dofs(nl - 1)[0]
    b = torch.zeros(nf, dtype=torch.float64, device="cuda")
    H.assemble_rhs(ri.mms_params(dim, 77), b)
    return H, b


@pytest.mark.parametrize("dim,n,nl,dm,kind", [(2, 64, 4, ri.OUTFLOW_2D, "vertex"),
                                             (3, 16, 3, ri.ALL_DIRICHLET_3D, "element")])
def test_replayed_cycles_equal_eager_cycles(dim, n, nl, dm, kind):
    print(f"[gpu] graph replay vs eager, dim {dim} N {n}", flush=True)
    H, b = _problem(dim, n, nl, dm, kind)
    try:
        for k in (1, 2, 3, 5):
            xs = torch.zeros_like(b)
            st, it, _ = H.solve(xs, b, 1e-300, k)       # up to k replays of the captured cycle
            assert 1 <= it <= k                          # (a divergence stop ends early)
            xe = torch.zeros_like(b)
            for _ in range(it):
                H.vcycle(xe, b)                          # eager launches between the replays
            torch.cuda.synchronize()
            assert torch.equal(xs, xe), (k, (xs - xe).abs().max().item())
        # other smoothing counts: the captured cycle must be rebuilt
        H.set_params(0.66 if kind == "vertex" else 0.5, 1, 3)
        xs = torch.zeros_like(b)
        _, it, _ = H.solve(xs, b, 1e-300, 2)
        xe = torch.zeros_like(b)
        for _ in range(it):
            H.vcycle(xe, b)
        torch.cuda.synchronize()
        assert torch.equal(xs, xe)
    finally:
        H.close()
