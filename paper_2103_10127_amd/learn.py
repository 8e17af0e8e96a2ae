"""Training driver of the per-patch damping network.

The network (16 patch features -> 64 -> 64 -> 1, omega_i = 0.2 + sigmoid)
replaces the scalar omega of the RAV sweep (eq. 13) by one weight per
subdomain, which eq. (11) allows.  It is trained on small two-level problems:
each step draws an initial error, runs the exact two-grid cycle with the
network's weights, back-propagates the residual reduction through the
reverse sweep and the network, and takes one Adam step (``rav_learn_step``;
every stage runs in the library's kernels).  The trained parameters are then
used on any hierarchy through ``Hierarchy.learn_set_omega``.
"""
from __future__ import annotations

import numpy as np

from .capi import MLP, Hierarchy


def initial_theta(seed: int = 0, out_bias: float = -0.16, out_scale: float = 0.01) -> np.ndarray:
    """He-initialised hidden layers and a near-zero output layer whose bias
    makes every omega_i start at 0.2 + sigmoid(out_bias) (0.66 by default)."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(64 * 16) * np.sqrt(2.0 / 16), np.zeros(64),
             rng.standard_normal(64 * 64) * np.sqrt(2.0 / 64), np.zeros(64),
             rng.standard_normal(64) * out_scale, np.array([out_bias])]
    return np.concatenate(parts).astype(np.float32)


def train(problems, steps: int = 400, lr: float = 3e-3, nu: int = 2, theta0=None, seed: int = 0,
          stream=None, warm_cycles: int = 0):
    """Train on ``problems`` (dicts of :class:`Hierarchy` keyword arguments with
    ``n_levels == 2``); returns (theta, per-step losses).  Initial errors are
    standard normal on the free DoFs, one per step, problems taken in turn.
    ``warm_cycles`` > 0 first runs that many two-grid cycles (b = 0) with the
    current weights on the error, removing the pressure mean and normalising
    after each, so that the loss measures the reduction of the slowest error
    components (an estimate of the asymptotic rate) instead of one cycle from
    a random error."""
    import torch

    hs = []
    try:
        for p in problems:
            if p.get("n_levels") != 2:
                raise ValueError("training problems need two levels (exact coarse solve)")
            h = Hierarchy(**p, stream=stream)
            h.factor()
            free = (h.owner(1) >= 0).to(torch.float64)
            n_p = (p["n_cells"] + 1) ** p.get("dim", 2)
            hs.append((h, free, n_p))
        net = MLP(initial_theta(seed) if theta0 is None else theta0)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        losses = []
        for it in range(steps):
            h, free, n_p = hs[it % len(hs)]
            x0 = torch.randn(free.numel(), generator=gen, device="cuda", dtype=torch.float64) * free
            if warm_cycles > 0:
                h.set_params(h.desc.omega, nu, nu)
                h.learn_set_omega(net)
                zero = torch.zeros_like(x0)
                for _ in range(warm_cycles):
                    h.vcycle(x0, zero)
                    x0[-n_p:] -= x0[-n_p:].mean()
                    x0 /= torch.linalg.norm(x0)
                h.learn_set_omega(None)
            losses.append(h.learn_step(net, x0, nu=nu, lr=lr))
        theta = net.theta()
        net.close()
        return theta, np.asarray(losses)
    finally:
        for h, *_ in hs:
            h.close()
