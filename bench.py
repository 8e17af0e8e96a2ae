#!/usr/bin/env python3
"""Benchmark: RAV-smoothed DoFs/s and time to a 1e-8 residual reduction.

Workload (N=1): 2D Taylor-Hood Q2/Q1 Stokes on a 512x512 grid (2,364,419
DoFs), 7 levels, viscosity 1, Dirichlet velocity on the whole boundary,
seeded manufactured forcing; geometric multigrid V(2,2) with RAV smoothing,
omega = 0.66, FP64 (Sec. 4: solve until the initial residual is reduced by
1e8).  One step = one full solve from x0 = 0 with all inputs resident in HBM.

value = smoothed DoFs per second over the whole solve: every RAV sweep on
every level counts its level's DoFs, divided by the wall time of the solve
(transfers, coarse solves and the per-cycle norm readback included).

Extra fields: per-step iterations, the finest-level sweep rate and its HBM
fraction, FP32/BF16 inverse-row solves, a roofline object for the dominant
kernel (the finest-level RAV apply, timed with HIP events on the launch stream
during the timed solves) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import rav_inputs as ri  # noqa: E402

HBM_PEAK_GBS = 8000.0


def sum_owned_times_patch(N: int) -> int:
    """sum_i (owned rows x patch columns) of all-Dirichlet 2D vertex patches:
    the algorithmic entry count of the stored RAV inverse rows."""
    k = np.arange(N + 1)
    span = np.minimum(2 * k + 2, 2 * N - 1) - np.maximum(2 * k - 2, 1) + 1
    own = np.maximum(np.minimum(2 * k + 1, 2 * N - 1) - np.maximum(2 * k, 1) + 1, 0)
    n_i = 2 * np.outer(span, span) + 1
    o_i = 2 * np.outer(own, own) + 1
    return int(np.sum(n_i * o_i))


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=20000, help="patches in the oracle sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also launch the plain copy kernel on 1 GiB (for HBM counter scaling)")
    return ap.parse_args()


def cpu_baseline(sample: int) -> dict:
    """Oracle RAV sweep on the 512x512 level, timed on a bounded sample (one
    thread).  Runs in a child process with single-threaded BLAS."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    code = f"""
import json, time, sys
import numpy as np, scipy.linalg as sla
sys.path.insert(0, {ROOT!r})
import rav_inputs as ri
from oracle import assemble as A, patches as pt, smoothers as sm
from oracle.grid import Grid
g = Grid(2, 512, ri.ALL_DIRICHLET_2D)
L = A.assemble_matrix(g)
owner = pt.owner_of_dofs(g, pt.VERTEX)
rng = np.random.default_rng(7)
idx = np.sort(rng.choice(g.nP, {sample}, replace=False))
dofs = [pt.patch_dofs(g, pt.VERTEX, int(i)) for i in idx]
lus = sm.factor(L, dofs)
own = [np.nonzero(owner[I] == i)[0] for I, i in zip(dofs, idx)]
x = ri.random_vector(g.n, 1) * g.free
b = ri.random_vector(g.n, 2) * g.free
best = None
for rep in range(5):
    t0 = time.perf_counter()
    r = sm.residual(L, x, b, g.free)
    t1 = time.perf_counter()
    dx = np.zeros(g.n)
    for I, o, lu in zip(dofs, own, lus):
        y = sla.lu_solve(lu, r[I])
        dx[I[o]] += 0.66 * y[o]
    t2 = time.perf_counter()
    sweep = (t1 - t0) + (t2 - t1) * g.nP / len(idx)
    best = sweep if best is None else min(best, sweep)
print(json.dumps(dict(sweep_s=best, n=int(g.n))))
"""
    t0 = time.time()
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True)
    if out.returncode != 0:
        return {"error": out.stderr[-400:]}
    res = json.loads(out.stdout.strip().splitlines()[-1])
    return {"value": res["n"] / res["sweep_s"], "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": (f"one FP64 RAV sweep of the 512x512 level (residual SpMV over all "
                       f"{res['n']} DoFs + LU solves of {sample} of {513 * 513} vertex patches, "
                       f"scaled to all patches; best of 5, single-threaded scipy)"),
            "wall_s": round(time.time() - t0, 1)}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2103_10127_amd import Hierarchy

    cfg = ri.CONFIGS["2d-512"]
    N, nl = cfg["n_cells"], cfg["n_levels"]
    nu, omega, rtol = 2, 0.66, 1e-8
    torch.cuda.set_device(0)
    params = ri.mms_params(2, cfg["seed"])

    def setup(prec):
        t0 = time.perf_counter()
        H = Hierarchy(dim=2, n_cells=N, n_levels=nl, dmask=cfg["dmask"], smoother="rav", omega=omega,
                      nu_pre=nu, nu_post=nu, precision=prec)
        H.factor()
        torch.cuda.synchronize()
        return H, time.perf_counter() - t0

    H, setup_s = setup("fp64")
    n_fine, n_free = H.dofs(nl - 1)
    level_n = [H.dofs(l)[0] for l in range(nl)]
    b = torch.zeros(n_fine, dtype=torch.float64, device="cuda")
    H.assemble_rhs(params, b)
    x = torch.zeros_like(b)

    def run(Hh, steps, profile=False):
        iters = []
        if profile:
            Hh.profile_begin(nl - 1, 8192)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            x.zero_()
            st, it, rr = Hh.solve(x, b, rtol, 200)
            if st != 0:
                raise RuntimeError(f"solve did not converge: status {st}, {it} cycles, rel {rr}")
            iters.append(it)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = Hh.profile_end() if profile else None
        return dt, iters, prof

    run(H, args.warmup)
    dt, iters, prof = run(H, args.steps, profile=True)
    smoothed_per_cycle = sum(2 * nu * level_n[l] for l in range(1, nl))
    smoothed = sum(iters) * smoothed_per_cycle
    value = smoothed / dt
    ms_step = 1e3 * dt / args.steps
    ms_res, ms_apply, n_apply = prof

    # Algorithmic bytes (per launch, finest level).
    sum_on = sum_owned_times_patch(N)
    apply_bytes = 8 * sum_on + 8 * n_fine + 16 * n_free          # W rows + r read + x read/write
    resid_bytes = 24 * n_fine + 8 * N * N                          # x, b read + r write + one coefficient per cell
    sweep_s = 1e-3 * (ms_res + ms_apply)
    sweep_rate = n_fine / sweep_s
    roof_apply = apply_bytes / (1e-3 * ms_apply) / 1e9
    roof_res = resid_bytes / (1e-3 * ms_res) / 1e9
    # HBM bytes per apply launch from the committed PMC summary (None once the kernel changed)
    from paper_2103_10127_amd.profiling import read_traffic
    traffic = read_traffic(os.path.join(ROOT, "profiles", "rav_apply_2d512_fp64_traffic.md"))

    out = {
        "metric": "RAV smoothed DoFs/s (whole V(2,2) solve to a 1e-8 residual reduction)",
        "value": value, "unit": "DoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded manufactured-solution forcing)",
        "config": {"workload": "2D Taylor-Hood Q2/Q1 Stokes 512x512, 7 levels, RAV V(2,2) omega 0.66, "
                               "solve from x0=0 to ||r|| <= 1e-8 ||r0||",
                   "dofs": n_fine, "levels": nl, "smoother": "rav", "nu": [nu, nu], "omega": omega,
                   "inverse_rows": "fp64"},
        "time_to_1e-8_ms": ms_step, "iters": int(np.median(iters)),
        "setup_s": round(setup_s, 3),
        "sweep": {"level": "512x512", "ms_residual": ms_res, "ms_apply": ms_apply,
                  "dofs_per_s": sweep_rate, "launches_timed": n_apply,
                  "pct_hbm_peak": 100.0 * (apply_bytes + resid_bytes) / sweep_s / 1e9 / HBM_PEAK_GBS},
        "roofline": {"bound": "hbm", "kernel": "k_rav_apply<2,VERTEX,0,double> (512x512 level)",
                     "achieved": roof_apply, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": roof_apply / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes": apply_bytes},
        "roofline_residual": {"bound": "hbm", "achieved": roof_res, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": roof_res / HBM_PEAK_GBS, "algorithmic_bytes": resid_bytes},
    }

    if args.copy_calibration:
        from paper_2103_10127_amd import stream_copy
        n = (1 << 30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            stream_copy(dst, src)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(10):
            stream_copy(dst, src)
        ev1.record()
        torch.cuda.synchronize()
        out["copy_GBs"] = 2 * n * 8 * 10 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
        del src, dst

    if not args.no_mixed:
        H.close()
        mixed = {}
        for prec in ("fp32", "bf16"):
            Hm, st_s = setup(prec)
            run(Hm, 1)
            dtm, itm, pm = run(Hm, max(1, args.steps // 2), profile=True)
            k = max(1, args.steps // 2)
            mixed[prec] = {"time_to_1e-8_ms": 1e3 * dtm / k, "iters": int(np.median(itm)),
                           "dofs_per_s": sum(itm) * smoothed_per_cycle / dtm,
                           "ms_apply": pm[1], "ms_residual": pm[0], "setup_s": round(st_s, 3),
                           "apply_GBs": ((2 if prec == "bf16" else 4) * sum_on + 8 * n_fine + 16 * n_free)
                           / (1e-3 * pm[1]) / 1e9}
            Hm.close()
        out["mixed"] = mixed
    else:
        H.close()

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
