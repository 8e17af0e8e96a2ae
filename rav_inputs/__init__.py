"""Seeded synthetic inputs for the restricted additive Vanka (RAV) multigrid.

This module only draws random numbers and packs them into flat arrays.  It
holds none of the method's arithmetic: the manufactured-solution forcing,
the viscosity field and every operator are evaluated separately by the CPU
oracle (``oracle/``) and by the HIP library, each from the packed draws.

Workloads (the paper's cavity/cylinder runs on adaptive grids are replaced by
uniform-grid Taylor-Hood Q2/Q1 Stokes problems of comparable size, Sec. 4):

* ``2d-32``   : 2D 32x32, 3 levels, eta = 1, all-Dirichlet, seed 1001
* ``2d-512``  : 2D 512x512, 7 levels, seed 1002
* ``3d-64``   : 3D 64^3, 5 levels, element patches, seed 1003
* ``batch256``: 256 2D problems, N in {64,128,256}, coarsest 16x16,
                1-8 circular inclusions at viscosity contrast 1e3, seeds 2000+i
* ``2d-1024`` : 2D 1024x1024, 8 levels, inclusions at contrast 1e4, seed 1005
"""
from __future__ import annotations

import numpy as np

N_MODES = 4

#: Dirichlet side bits: bit 2*d is the side x_d = 0, bit 2*d+1 the side x_d = 1.
ALL_DIRICHLET_2D = 0b1111
ALL_DIRICHLET_3D = 0b111111
#: Outflow variant: natural (do-nothing) boundary on x = 1, Dirichlet elsewhere.
OUTFLOW_2D = 0b1101
OUTFLOW_3D = 0b111101


def mms_params(dim: int, seed: int, eta: float = 1.0) -> np.ndarray:
    """Draw the manufactured-solution modes and pack them into a flat array.

    Layout (float64):
      2D: [eta, a(4), m(4), n(4), c(4), r(4), s(4)]                 -> 25 values
      3D: [eta, for comp in 0..2: a(4), m(4), n(4), l(4),
                c(4), r(4), s(4), t(4)]                             -> 65 values
    a, c ~ N(0, 1); integer wave numbers are drawn uniformly from {1, 2, 3}.
    ``eta`` is the viscosity used in the forcing.
    """
    rng = np.random.default_rng(seed)
    out = [float(eta)]
    if dim == 2:
        a = rng.standard_normal(N_MODES)
        m = rng.integers(1, 4, N_MODES)
        n = rng.integers(1, 4, N_MODES)
        c = rng.standard_normal(N_MODES)
        r = rng.integers(1, 4, N_MODES)
        s = rng.integers(1, 4, N_MODES)
        for arr in (a, m, n, c, r, s):
            out.extend(float(v) for v in arr)
    elif dim == 3:
        for _comp in range(3):
            a = rng.standard_normal(N_MODES)
            m = rng.integers(1, 4, N_MODES)
            n = rng.integers(1, 4, N_MODES)
            l = rng.integers(1, 4, N_MODES)
            for arr in (a, m, n, l):
                out.extend(float(v) for v in arr)
        c = rng.standard_normal(N_MODES)
        r = rng.integers(1, 4, N_MODES)
        s = rng.integers(1, 4, N_MODES)
        t = rng.integers(1, 4, N_MODES)
        for arr in (c, r, s, t):
            out.extend(float(v) for v in arr)
    else:
        raise ValueError("dim must be 2 or 3")
    return np.asarray(out, dtype=np.float64)


def inclusions(seed: int, n_min: int = 1, n_max: int = 8,
               c_lo: float = 0.1, c_hi: float = 0.9,
               r_lo: float = 0.03, r_hi: float = 0.12) -> np.ndarray:
    """Circular inclusions as an (n, 3) array of (cx, cy, radius)."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(n_min, n_max + 1))
    cx = rng.uniform(c_lo, c_hi, k)
    cy = rng.uniform(c_lo, c_hi, k)
    rad = rng.uniform(r_lo, r_hi, k)
    return np.stack([cx, cy, rad], axis=1).astype(np.float64)


def spheres(seed: int, count: int = 6, c_lo: float = 0.15, c_hi: float = 0.85,
            r_lo: float = 0.05, r_hi: float = 0.15) -> np.ndarray:
    """Spherical inclusions as a (count, 4) array of (cx, cy, cz, radius)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(c_lo, c_hi, (count, 3))
    rad = rng.uniform(r_lo, r_hi, count)
    return np.concatenate([c, rad[:, None]], axis=1).astype(np.float64)


def random_vector(n: int, seed: int) -> np.ndarray:
    """Standard-normal float64 vector (initial iterates, test right-hand sides)."""
    return np.random.default_rng(seed).standard_normal(n)


def batch_sizes(n_problems: int = 256, seed: int = 2000) -> np.ndarray:
    """Fine-grid sizes of the batched workload, uniform over {64, 128, 256}."""
    rng = np.random.default_rng(seed)
    return np.asarray([64, 128, 256])[rng.integers(0, 3, n_problems)]


def levels_to(n_cells: int, coarsest: int) -> int:
    """Number of levels of a uniform hierarchy from n_cells down to coarsest."""
    lv = 1
    n = n_cells
    while n > coarsest:
        if n % 2:
            raise ValueError("n_cells must halve down to the coarsest grid")
        n //= 2
        lv += 1
    if n != coarsest:
        raise ValueError("coarsest grid not reached")
    return lv


#: The five synthetic workloads.  ``dmask`` = Dirichlet side bits.
CONFIGS = {
    "2d-32": dict(dim=2, n_cells=32, n_levels=3, seed=1001, dmask=ALL_DIRICHLET_2D,
                  eta_out=1.0, eta_in=1.0, contrast=None),
    "2d-512": dict(dim=2, n_cells=512, n_levels=7, seed=1002, dmask=ALL_DIRICHLET_2D,
                   eta_out=1.0, eta_in=1.0, contrast=None),
    "3d-64": dict(dim=3, n_cells=64, n_levels=5, seed=1003, dmask=ALL_DIRICHLET_3D,
                  eta_out=1.0, eta_in=1.0, contrast=None),
    "batch256": dict(dim=2, n_problems=256, coarsest=16, seed=2000,
                     dmask=ALL_DIRICHLET_2D, eta_out=1.0, contrast=1e3),
    "2d-1024": dict(dim=2, n_cells=1024, n_levels=8, seed=1005, dmask=ALL_DIRICHLET_2D,
                    eta_out=1.0, contrast=1e4),
}


#: Parameter count of the per-patch damping network 16 -> 64 -> 64 -> 1:
#: W1 (64x16), b1 (64), W2 (64x64), b2 (64), w3 (64), b3 (1), stored in that
#: order, matrices row-major (output index slow).
MLP_SIZES = ((64, 16), (64,), (64, 64), (64,), (64,), (1,))
MLP_NPARAM = sum(int(np.prod(s)) for s in MLP_SIZES)


def mlp_init(seed: int, out_bias: float = -0.16, out_scale: float = 0.01) -> np.ndarray:
    """He-normal draws for W1, W2, small normal draws for w3, zero hidden biases
    and a fixed output bias (float32, flat)."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal((64, 16)) * np.sqrt(2.0 / 16)
    w2 = rng.standard_normal((64, 64)) * np.sqrt(2.0 / 64)
    w3 = rng.standard_normal(64) * out_scale
    parts = [w1.ravel(), np.zeros(64), w2.ravel(), np.zeros(64), w3, np.array([out_bias])]
    return np.concatenate(parts).astype(np.float32)


# ---- adaptive cavity grids (Sec. 4.1, Table 1) -------------------------------
# Leaf cells (x0, y0, s) of quadtrees over the unit square in integer lattice
# units (lattice(n) per side).  Grid 1 is the uniform 8 x 8 grid; step l
# refines every leaf of the current finest size within BANDS[l-1] such cells of
# the boundary (our reading of the refinement towards the boundary in Sec. 4.1;
# these widths give the element counts of Table 1).
BASE = 8
BANDS = (2, 3, 5, 8, 13, 19, 27, 31, 17)


def lattice(n_grids: int) -> int:
    """Lattice units per side of the unit square for a hierarchy of n_grids."""
    return BASE << n_grids


def cavity_grids(n_grids: int = 10, bands=BANDS):
    """The hierarchy Omega^1 .. Omega^n as leaf arrays (n_leaves, 3) of
    (x0, y0, s) in units of half the finest cell of the last grid."""
    M = lattice(n_grids)                   # lattice units per side
    s0 = 1 << n_grids
    ii, jj = np.meshgrid(np.arange(BASE), np.arange(BASE), indexing="ij")
    leaves = np.stack([ii.ravel() * s0, jj.ravel() * s0, np.full(BASE * BASE, s0)], axis=1).astype(np.int64)
    grids = [leaves]
    for l in range(1, n_grids):
        s = leaves[:, 2]
        fine = s.min()
        x0, y0 = leaves[:, 0], leaves[:, 1]
        # distance to the boundary in finest-cell units, measured from the cell's near side
        dist = np.minimum.reduce([x0, y0, M - (x0 + s), M - (y0 + s)]) // fine
        refine = (s == fine) & (dist < bands[l - 1])
        keep = leaves[~refine]
        r = leaves[refine]
        h = r[:, 2:3] // 2
        kids = np.concatenate([np.concatenate([r[:, 0:1] + dx * h, r[:, 1:2] + dy * h, h], axis=1)
                               for dx in (0, 1) for dy in (0, 1)])
        leaves = np.concatenate([keep, kids])
        grids.append(leaves)
    return grids


def random_quadtree_grids(n_grids: int = 4, base: int = 4, frac: float = 0.3, seed: int = 0):
    """A nested hierarchy of 2:1-balanced quadtree grids over the unit square
    with randomly placed refinement (a stress case for hanging nodes: chains
    of constrained corners, patches of every shape).  Grid 1 is the uniform
    base x base grid; each next grid refines a random fraction `frac` of the
    refinable leaves and then every leaf whose edge meets a leaf smaller than
    half its size, until the grid is balanced.  Leaves (x0, y0, s) in units of
    half the smallest possible cell; returns (grids, lattice units per side)."""
    rng = np.random.default_rng(seed)
    s0 = 1 << n_grids
    M = base * s0
    leaves = {(i * s0, j * s0, s0) for i in range(base) for j in range(base)}
    grids = [np.array(sorted(leaves), dtype=np.int64)]

    def split(leaf):
        x0, y0, sz = leaf
        h = sz // 2
        return {(x0 + dx * h, y0 + dy * h, h) for dx in (0, 1) for dy in (0, 1)}

    for _ in range(1, n_grids):
        cand = sorted(lf for lf in leaves if lf[2] >= 4)
        pick = rng.random(len(cand)) < frac
        for lf, p in zip(cand, pick):
            if p:
                leaves.remove(lf)
                leaves |= split(lf)
        while True:   # 2:1 balance: no leaf corner at a quarter point of a larger leaf's edge
            corners = {(x0 + a * sz, y0 + b * sz) for x0, y0, sz in leaves for a in (0, 1) for b in (0, 1)}
            bad = set()
            for x0, y0, sz in leaves:
                if sz < 4:
                    continue
                for q in (sz // 4, 3 * sz // 4):
                    if {(x0 + q, y0), (x0 + q, y0 + sz), (x0, y0 + q), (x0 + sz, y0 + q)} & corners:
                        bad.add((x0, y0, sz))
                        break
            if not bad:
                break
            for lf in bad:
                leaves.remove(lf)
                leaves |= split(lf)
        grids.append(np.array(sorted(leaves), dtype=np.int64))
    return grids, M


# ---- channel with a cylindrical obstacle (Sec. 4.2, Table 2) ------------------
# The paper's coarse mesh (758 quadrilaterals fitted to the cylinder) is not
# given.  Stand-in: square coarse cells of size H / 12 over the channel, 64 x 12
# cells (length 64/12 H = 2.187 m against 2.2 m), the cells whose centres lie
# inside the cylinder (centre (0.2, 0.2) m, radius 0.05 m) removed: 762 cells
# and 844 vertices against Table 2's 758 and 842.  Lengths are in units of the
# height H (0.41 m).  Grids 2 and 3 refine uniformly (as Table 2's counts do);
# step l >= 3 refines every leaf of the current finest size within
# CHANNEL_BANDS[l-1] such cells of a no-slip boundary (the walls and the
# obstacle), then closes the grid under 2:1 balance.
CHANNEL_CELLS = (64, 12)
CHANNEL_HEIGHT = 0.41
CYLINDER = (0.2, 0.2, 0.05)                 # centre x, y and radius (m)
UNIFORM = 1 << 30
CHANNEL_BANDS = (UNIFORM, UNIFORM, 11, 18, 29, 19)


def _split(leaves):
    h = leaves[:, 2:3] // 2
    return np.concatenate([np.concatenate([leaves[:, 0:1] + dx * h, leaves[:, 1:2] + dy * h, h], axis=1)
                           for dx in (0, 1) for dy in (0, 1)])


def _balance(leaves):
    """Refines leaves until no leaf corner lies at a quarter point of another
    leaf's edge (2:1 balance)."""
    while True:
        x0, y0, s = leaves[:, 0], leaves[:, 1], leaves[:, 2]
        key = lambda x, y: (x << 32) + y
        corners = np.unique(np.concatenate([key(x0 + a * s, y0 + b * s) for a in (0, 1) for b in (0, 1)]))
        big = s >= 4
        bad = np.zeros(len(leaves), dtype=bool)
        for f in (1, 3):
            q = s * f // 4
            for px, py in ((x0 + q, y0), (x0 + q, y0 + s), (x0, y0 + q), (x0 + s, y0 + q)):
                bad |= big & np.isin(key(px, py), corners)
        if not bad.any():
            return leaves
        leaves = np.concatenate([leaves[~bad], _split(leaves[bad])])


def channel_grids(n_grids: int = 7, bands=CHANNEL_BANDS, cells=CHANNEL_CELLS):
    """The hierarchy Omega^1 .. Omega^n of the channel as leaf arrays
    (n_leaves, 3) of (x0, y0, s), in units of half the finest cell of the
    last grid; returns (grids, lattice_x, lattice_y).  Velocity data: inflow
    on x = 0, no slip on y = 0, y = H and the obstacle, outflow x = max open
    (Dirichlet mask 0b1101)."""
    nx, ny = cells
    s0 = 1 << n_grids
    cx, cy, r = (c / CHANNEL_HEIGHT * ny for c in CYLINDER)   # in coarse cells
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    hole = (ii + 0.5 - cx) ** 2 + (jj + 0.5 - cy) ** 2 <= r * r
    leaves = np.stack([ii[~hole] * s0, jj[~hole] * s0, np.full((~hole).sum(), s0)], axis=1).astype(np.int64)
    obst = np.stack([ii[hole] * s0, jj[hole] * s0], axis=1).astype(np.int64)
    Mx, My = nx * s0, ny * s0
    grids = [leaves]
    for l in range(1, n_grids):
        s = leaves[:, 2]
        fine = s.min()
        x0, y0 = leaves[:, 0], leaves[:, 1]
        dist = np.minimum(y0, My - (y0 + s))
        for ox, oy in obst:
            gx = np.maximum.reduce([np.zeros_like(x0), ox - (x0 + s), x0 - (ox + s0)])
            gy = np.maximum.reduce([np.zeros_like(y0), oy - (y0 + s), y0 - (oy + s0)])
            dist = np.minimum(dist, np.maximum(gx, gy))
        refine = (s == fine) & (dist // fine < bands[l - 1])
        leaves = _balance(np.concatenate([leaves[~refine], _split(leaves[refine])]))
        grids.append(leaves)
    return grids, Mx, My

