"""Pins of the learned-damping oracle: the two-grid forward equals the pinned
V-cycle for constant omega, and every analytic gradient equals central finite
differences in FP64."""
import numpy as np

import rav_inputs as ri
from oracle import learned as ln
from oracle import mg
from oracle.grid import Grid


def _setup(N=8, contrast=50.0, seed=3001):
    incl = ri.inclusions(seed)
    H = mg.Hierarchy(2, N, 2, ri.ALL_DIRICHLET_2D, 0, 1.0, contrast, incl)
    return H, incl


def test_features_hand_case():
    g = Grid(2, 4, ri.ALL_DIRICHLET_2D)
    incl = np.array([[0.5, 0.5, 0.1]])          # covers only the centre point (0.5, 0.5)
    F = ln.features(g, 1.0, 1e4, incl)
    k = 2 + 5 * 2                                # vertex (2, 2) at (0.5, 0.5)
    assert F.shape == (25, 16)
    np.testing.assert_allclose(F[k, :9], [0, 0, 0, 0, 1, 0, 0, 0, 0])
    np.testing.assert_allclose(F[k, 9:16], [0, 1, 1 / 9, 0, 0, 0.2, 1])
    assert F[0, 12] == 1 and F[0, 13] == 1 and F[6, 12] == 0
    assert np.all(F[np.arange(25) != k, :9] == 0)


def test_twogrid_forward_equals_vcycle():
    H, _ = _setup()
    tg = ln.TwoGrid(H, nu=2)
    x0 = ri.random_vector(H.finest.grid.n, 5) * H.finest.grid.free
    xo = tg.forward(0.66, x0)[-1]
    xv = H.vcycle(x0.copy(), np.zeros_like(x0), "rav", 0.66, 2)
    np.testing.assert_allclose(xo, xv, rtol=0, atol=1e-12 * np.abs(xv).max())


def test_omega_gradient_matches_finite_differences():
    H, _ = _setup()
    tg = ln.TwoGrid(H, nu=2)
    n = tg.ps.count
    rng = np.random.default_rng(1)
    omega = rng.uniform(0.4, 0.9, n)
    x0 = ri.random_vector(H.finest.grid.n, 6) * H.finest.grid.free
    loss, g = tg.loss_and_grad(omega, x0)
    assert abs(loss - tg.loss(omega, x0)) <= 1e-13 * loss
    eps = 1e-6
    for i in rng.choice(n, 12, replace=False):
        e = np.zeros(n); e[i] = eps
        fd = (tg.loss(omega + e, x0) - tg.loss(omega - e, x0)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g).max(), 1e-12), (i, fd, g[i])


def test_theta_gradient_matches_finite_differences():
    H, incl = _setup()
    tg = ln.TwoGrid(H, nu=2)
    F = ln.features(H.finest.grid, 1.0, 50.0, incl)
    theta = ri.mlp_init(7, out_scale=0.3).astype(np.float64)
    x0 = ri.random_vector(H.finest.grid.n, 8) * H.finest.grid.free

    def total(th):
        om, _ = ln.mlp_forward(th, F)
        return tg.loss(om, x0)

    om, cache = ln.mlp_forward(theta, F)
    loss, g_om = tg.loss_and_grad(om, x0)
    gth = ln.mlp_backward(theta, cache, g_om)
    rng = np.random.default_rng(2)
    eps = 1e-6
    idx = np.concatenate([rng.choice(1024, 6, replace=False), 1024 + rng.choice(64, 2, replace=False),
                          1088 + rng.choice(4096, 6, replace=False), 5184 + rng.choice(64, 2, replace=False),
                          5248 + rng.choice(64, 4, replace=False), [5312]])
    scale = np.abs(gth).max()
    for j in idx:
        e = np.zeros_like(theta); e[j] = eps
        fd = (total(theta + e) - total(theta - e)) / (2 * eps)
        assert abs(fd - gth[j]) <= 1e-6 * scale, (j, fd, gth[j])
