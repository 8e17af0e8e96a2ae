"""Caller-supplied device allocator (rav_set_device_allocator): every buffer of
a hierarchy comes from it and goes back to it, the results are those of the
default hipMalloc path, and the allocator cannot change while a context
lives.  The argument checks need no device."""
import numpy as np
import pytest

import rav_inputs as ri
from paper_2103_10127_amd import capi


def test_allocator_arguments_checked_without_device():
    capi.set_device_allocator()                       # restore the default: always allowed here
    with pytest.raises(capi.RavError):
        capi.set_device_allocator(lambda n: 0, None)   # one function without the other


@pytest.mark.gpu
def test_torch_caching_allocator_serves_every_buffer(monkeypatch):
    torch = pytest.importorskip("torch")
    from paper_2103_10127_amd import Hierarchy
    from paper_2103_10127_amd.capi import AdaptiveHierarchy
    monkeypatch.setenv("RAV_AUTOTUNE", "0")           # identical launch choices in both runs
    live, n_alloc = {}, [0]

    def alloc(n):
        p = torch.cuda.caching_allocator_alloc(n)
        live[p] = n
        n_alloc[0] += 1
        return p

    def release(p):
        assert p in live, "released a pointer the allocator did not hand out"
        del live[p]
        torch.cuda.caching_allocator_delete(p)

    def solve_all():
        out = []
        cfg = dict(dim=2, n_cells=32, n_levels=3, dmask=ri.ALL_DIRICHLET_2D)
        for kw in ({}, {"inv_format": "factored"}, {"discretization": "q1q1", "beta": 0.05}):
            H = Hierarchy(**cfg, **kw)
            H.factor()
            n = H.dofs(2)[0]
            b = torch.zeros(n, dtype=torch.float64, device="cuda")
            H.assemble_rhs_lid(b, 1.0)
            x = torch.zeros_like(b)
            out.append((H.solve(x, b, 1e-8, 100), x.cpu().numpy()))
            xg = torch.zeros_like(b)
            out.append((H.solve_gmres(xg, b, 1e-8, 100, 10) if not kw.get("discretization") else (0, 0, 0.0),
                        xg.cpu().numpy()))
            H.close()
        H = AdaptiveHierarchy(ri.cavity_grids(3), ri.lattice(3), beta=0.05)
        H.factor()
        n = H.dofs(2)[0]
        b = torch.zeros(n, dtype=torch.float64, device="cuda")
        H.assemble_rhs_lid(b, 1.0)
        x = torch.zeros_like(b)
        out.append((H.solve(x, b, 1e-8, 100), x.cpu().numpy()))
        H.close()
        return out

    print("[gpu] allocator: default run", flush=True)
    ref = solve_all()
    print("[gpu] allocator: torch caching allocator run", flush=True)
    capi.set_device_allocator(alloc, release)
    try:
        got = solve_all()
        assert n_alloc[0] > 0 and not live, (n_alloc[0], len(live))
        H = Hierarchy(dim=2, n_cells=16, n_levels=2)
        with pytest.raises(capi.RavError):
            capi.set_device_allocator()             # refused while a context lives
        assert live
        H.close()
        assert not live
    finally:
        capi.set_device_allocator()
    for (sr, xr), (sg, xg) in zip(ref, got):
        assert sr == sg
        np.testing.assert_array_equal(xr, xg)
