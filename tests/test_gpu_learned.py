"""Learned per-patch damping on the GPU against the FP64 oracle: network
outputs, the exact two-grid loss, its gradient with respect to every patch
weight (reverse sweep) and with respect to the network parameters."""
import numpy as np
import pytest

import rav_inputs as ri
from oracle import learned as ln
from oracle import mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2103_10127_amd import Hierarchy  # noqa: E402
from paper_2103_10127_amd.capi import MLP  # noqa: E402


def _pair(N=16, contrast=50.0, seed=3001):
    incl = ri.inclusions(seed)
    print(f"[gpu] learned pair N={N} contrast={contrast}", flush=True)
    H = mg.Hierarchy(2, N, 2, ri.ALL_DIRICHLET_2D, 0, 1.0, contrast, incl)
    G = Hierarchy(dim=2, n_cells=N, n_levels=2, eta_in=contrast, inclusions=incl)
    G.factor()
    return H, G, incl


def test_network_output_matches_oracle():
    H, G, incl = _pair()
    theta = ri.mlp_init(11, out_scale=0.5)
    M = MLP(theta)
    g = H.finest.grid
    om = torch.zeros(g.nP, dtype=torch.float32, device="cuda")
    G.learn_patch_omega(M, 1, om)
    F = ln.features(g, 1.0, 50.0, incl)
    ref, _ = ln.mlp_forward(theta.astype(np.float64), F)
    np.testing.assert_allclose(om.cpu().numpy(), ref, rtol=0, atol=2e-6)
    assert ref.std() > 1e-3   # the inclusions make the weights vary
    M.close(); G.close()


def test_twogrid_loss_and_gradients_match_oracle():
    H, G, incl = _pair()
    theta = ri.mlp_init(12, out_scale=0.5)
    M = MLP(theta)
    g = H.finest.grid
    x0 = ri.random_vector(g.n, 13) * g.free
    gom = torch.zeros(g.nP, dtype=torch.float64, device="cuda")
    loss, gth = G.learn_twogrid(M, torch.from_numpy(x0).cuda(), nu=2, grad_omega=gom)
    om = torch.zeros(g.nP, dtype=torch.float32, device="cuda")
    G.learn_patch_omega(M, 1, om)
    omega = om.cpu().numpy().astype(np.float64)
    tg = ln.TwoGrid(H, nu=2)
    lref, gref = tg.loss_and_grad(omega, x0)
    assert abs(loss - lref) <= 1e-10 * lref, (loss, lref)
    gg = gom.cpu().numpy()
    assert np.linalg.norm(gg - gref) <= 1e-9 * np.linalg.norm(gref)
    F = ln.features(g, 1.0, 50.0, incl)
    _, cache = ln.mlp_forward(theta.astype(np.float64), F)
    gth_ref = ln.mlp_backward(theta.astype(np.float64), cache, gref)
    assert np.linalg.norm(gth - gth_ref) <= 1e-4 * np.linalg.norm(gth_ref)
    M.close(); G.close()


def test_training_steps_reduce_the_loss():
    H, G, incl = _pair(N=16, contrast=100.0, seed=3002)
    g = H.finest.grid
    M = MLP(ri.mlp_init(14))
    x0s = [torch.from_numpy(ri.random_vector(g.n, 100 + i) * g.free).cuda() for i in range(4)]

    def mean_loss():
        return np.mean([G.learn_twogrid(M, x, nu=2, want_theta=False)[0] for x in x0s])

    before = mean_loss()
    for it in range(40):
        G.learn_step(M, x0s[it % 4], nu=2, lr=3e-3)
    after = mean_loss()
    assert after < before, (before, after)
    M.close(); G.close()
