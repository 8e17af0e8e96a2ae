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

The owned rows of each local inverse are stored in the factored form by
default (RAV_FACTORED: owned rows of the scalar viscous block's inverse, z and
the Schur complement inverse; the same rows up to rounding, 151 values per
patch instead of 459); --format rows stores the rows themselves.

Extra fields: per-step iterations, the finest-level sweep rate and its HBM
fraction, the other storage formats and FP32/BF16 solves, a roofline object for
the dominant kernel (the finest-level RAV apply, timed with HIP events on the
launch stream during the timed solves) and the CPU oracle timed on a bounded
sample.
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


def sum_owned_times_patch_3d_element(N: int) -> int:
    """sum_i (owned rows x patch columns) of all-Dirichlet 3D element patches.
    Per axis a cell at e has 3 - [e=0] - [e=N-1] free velocity positions, owns
    2 - [e=0] of them and 1 + [e=N-1] pressure positions; n_i = 3 prod c + 8,
    owned_i = 3 prod o + prod p, and each product term sums separably."""
    e = np.arange(N)
    lo, hi = (e == 0).astype(np.int64), (e == N - 1).astype(np.int64)
    c, o, p = 3 - lo - hi, 2 - lo, 1 + hi
    S = lambda f: int(f.sum())
    return 9 * S(c * o) ** 3 + 3 * S(c * p) ** 3 + 24 * S(o) ** 3 + 8 * S(p) ** 3


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the other storage formats and precisions")
    ap.add_argument("--format", default="factored", choices=["factored", "rows"],
                    help="storage of the owned inverse rows for the headline FP64 solve")
    ap.add_argument("--cpu-sample", type=int, default=12000, help="patches in the oracle sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also launch the plain copy kernel on 1 GiB (for HBM counter scaling)")
    ap.add_argument("--workload", default="2d-512",
                    choices=["2d-512", "3d-64", "3d-64-vertex", "2d-1024", "batch256", "learned", "smoothers", "q1q1",
                             "cavity", "adaptive", "channel"],
                    help="2d-512: the headline solve (default); 3d-64: finest-level element-patch sweep; "
                         "3d-64-vertex: 64^3 solve with vertex patches; 2d-1024: inclusions at contrast 1e4; "
                         "batch256: 256 problems; learned: per-patch damping trained on small problems, "
                         "evaluated on held-out 128^2/256^2 problems at contrast 1e2 against fixed omega; smoothers: RAV/AV/MV cost per cycle, "
                         "cycles and time to 1e-8 on 32^2 (damping sweep) and 512^2; cavity: driven cavity, "
                         "smoothing-steps and mesh studies; q1q1: the stabilized Q1-Q1 driven cavity on 1024^2; "
                         "adaptive: the cavity on the adaptive grids of Table 1, RAV/MV/AV on every grid (Fig. 5); "
                         "channel: flow past a cylinder on a stand-in of Table 2's grids, smoothing-steps and mesh "
                         "studies (Figs. 7-9)")
    ap.add_argument("--quick", action="store_true",
                    help="adaptive, channel: only the finest-grid RAV solve (and, adaptive, its kernel times)")
    ap.add_argument("--train-steps", type=int, default=400)
    ap.add_argument("--train-lr", type=float, default=1e-3)
    return ap.parse_args()


_CPU_SWEEP = """
import json, time, sys
import numpy as np, scipy.linalg as sla
sys.path.insert(0, {root!r})
import rav_inputs as ri
from oracle import assemble as A, patches as pt, smoothers as sm
from oracle.grid import Grid
part, nparts, sample = {part}, {nparts}, {sample}
g = Grid(2, 512, ri.ALL_DIRICHLET_2D)
L = A.assemble_matrix(g)
owner = pt.owner_of_dofs(g, pt.VERTEX)
rng = np.random.default_rng(7)
idx = np.sort(rng.choice(g.nP, sample, replace=False))[part::nparts]
dofs = [pt.patch_dofs(g, pt.VERTEX, int(i)) for i in idx]
lus = sm.factor(L, dofs)
own = [np.nonzero(owner[I] == i)[0] for I, i in zip(dofs, idx)]
x = ri.random_vector(g.n, 1) * g.free
b = ri.random_vector(g.n, 2) * g.free
print("ready", flush=True)
sys.stdin.readline()
best_r = best_p = None
for rep in range(5):
    t0 = time.perf_counter()
    r = sm.residual(L, x, b, g.free)
    t1 = time.perf_counter()
    dx = np.zeros(g.n)
    for I, o, lu in zip(dofs, own, lus):
        y = sla.lu_solve(lu, r[I])
        dx[I[o]] += 0.66 * y[o]
    t2 = time.perf_counter()
    best_r = (t1 - t0) if best_r is None else min(best_r, t1 - t0)
    best_p = (t2 - t1) if best_p is None else min(best_p, t2 - t1)
print(json.dumps(dict(resid_s=best_r, patch_s=best_p, npatch=len(idx), n=int(g.n))))
"""

_CPU_SOLVE = """
import json, time, sys
sys.path.insert(0, {root!r})
import rav_inputs as ri
from oracle import assemble as A, mg
t0 = time.perf_counter()
H = mg.Hierarchy(2, 32, 3, ri.ALL_DIRICHLET_2D)
b = A.assemble_rhs(H.finest.grid, ri.mms_params(2, 1001))
t1 = time.perf_counter()
x, k, hist, st = H.solve(b)
t2 = time.perf_counter()
H.vcycle(x * 0, b)
t3 = time.perf_counter()
print(json.dumps(dict(setup_s=t1 - t0, solve_s=t2 - t1, vcycle_s=t3 - t2, iters=k, status=st, n=int(H.finest.grid.n))))
"""


def _host_info() -> dict:
    info = {"nproc": os.cpu_count()}
    try:
        info["nproc_affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                info["ram_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return info


def _single_thread_env():
    return dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")


def _cpu_sweep(sample: int, nparts: int) -> dict:
    """The oracle's RAV sweep of the 512x512 level on `sample` patches, split
    over `nparts` single-threaded processes that run at the same time (the
    residual is timed in every process; the slowest one counts)."""
    procs = [subprocess.Popen([sys.executable, "-c", _CPU_SWEEP.format(root=ROOT, part=i, nparts=nparts,
                                                                          sample=sample)],
                              env=_single_thread_env(), stdin=subprocess.PIPE, stdout=subprocess.PIPE,
                              stderr=subprocess.PIPE, text=True) for i in range(nparts)]
    for p in procs:   # all set up, then all timed together
        if p.stdout.readline().strip() != "ready":
            return {"error": p.stderr.read()[-400:]}
    for p in procs:
        p.stdin.write("go\n")
        p.stdin.flush()
    res = []
    for p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            return {"error": err[-400:]}
        res.append(json.loads(out.strip().splitlines()[-1]))
    n = res[0]["n"]
    patch_s = max(r["patch_s"] / r["npatch"] for r in res) * sum(r["npatch"] for r in res) / nparts
    sweep_s = max(r["resid_s"] for r in res) + patch_s * (513 * 513) / sample
    return {"sweep_s": sweep_s, "n": n}


def cpu_baseline(sample: int) -> dict:
    """The FP64 oracle on the host cores, bounded: one RAV sweep of the 512x512
    level (residual over all DoFs + LU solves of `sample` sampled patches,
    scaled to all 263,169) on one core and on all cores, and the whole 32x32
    solve (3 levels, V(2,2), to 1e-8) on one core."""
    t0 = time.time()
    host = _host_info()
    ncores = max(1, host.get("nproc_affinity", host["nproc"] or 1))
    one = _cpu_sweep(sample, 1)
    if "error" in one:
        return one
    allc = _cpu_sweep(sample, ncores) if ncores > 1 else one
    out = subprocess.run([sys.executable, "-c", _CPU_SOLVE.format(root=ROOT)], env=_single_thread_env(),
                         capture_output=True, text=True)
    solve32 = json.loads(out.stdout.strip().splitlines()[-1]) if out.returncode == 0 else {"error": out.stderr[-400:]}
    res = {"value": one["n"] / one["sweep_s"], "unit": "DoF/s", "cores": 1, "kind": "oracle",
           "sample": (f"one FP64 RAV sweep of the 512x512 level (residual SpMV over all {one['n']} DoFs + LU "
                      f"solves of {sample} of {513 * 513} vertex patches, scaled to all patches; best of 5, "
                      f"single-threaded scipy)"),
           "all_cores": {"value": allc.get("n", one["n"]) / allc["sweep_s"] if "sweep_s" in allc else None,
                         "cores": ncores,
                         "how": "the same sample split over one single-threaded process per core, run together"},
           "solve_32x32_one_core": solve32, "host": host, "wall_s": None}
    res["wall_s"] = round(time.time() - t0, 1)
    return res


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(no collectives, no sharding of the grid).", file=sys.stderr)
        sys.exit(2)
    if args.workload != "2d-512":
        {"3d-64": bench_3d, "3d-64-vertex": bench_3d_vertex, "2d-1024": bench_1024, "batch256": bench_batch,
         "learned": bench_learned, "smoothers": bench_smoothers, "cavity": bench_cavity,
         "q1q1": bench_q1q1, "adaptive": bench_adaptive, "channel": bench_channel}[args.workload](args)
        return
    import torch
    from paper_2103_10127_amd import Hierarchy

    cfg = ri.CONFIGS["2d-512"]
    N, nl = cfg["n_cells"], cfg["n_levels"]
    nu, omega, rtol = 2, 0.66, 1e-8
    torch.cuda.set_device(0)
    params = ri.mms_params(2, cfg["seed"])

    def setup(prec, fmt):
        t0 = time.perf_counter()
        H = Hierarchy(dim=2, n_cells=N, n_levels=nl, dmask=cfg["dmask"], smoother="rav", omega=omega,
                      nu_pre=nu, nu_post=nu, precision=prec, inv_format=fmt)
        H.factor()
        torch.cuda.synchronize()
        return H, time.perf_counter() - t0

    H, setup_s = setup("fp64", args.format)
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

    # Algorithmic bytes (per launch, finest level): the stored inverse data of
    # every patch (owned rows, or the factored form's 151 values per patch),
    # r read once, x read and written on free DoFs.
    sum_on = sum_owned_times_patch(N)
    fact_vals = 25 * 6 + 1

    def w_entries(fmt):
        return sum_on if fmt == "rows" else fact_vals * (N + 1) ** 2

    apply_bytes = 8 * w_entries(args.format) + 8 * n_fine + 16 * n_free
    resid_bytes = 24 * n_fine + 8 * N * N                          # x, b read + r write + one coefficient per cell
    sweep_s = 1e-3 * (ms_res + ms_apply)
    sweep_rate = n_fine / sweep_s
    roof_apply = apply_bytes / (1e-3 * ms_apply) / 1e9
    roof_res = resid_bytes / (1e-3 * ms_res) / 1e9
    # HBM bytes per apply launch from the committed PMC summary (None once the kernel changed)
    from paper_2103_10127_amd.profiling import read_traffic
    traffic = read_traffic(os.path.join(ROOT, "profiles", "rav_apply_fact_2d512_fp64_traffic.md"
                                        if args.format == "factored" else "rav_apply_2d512_fp64_traffic.md"))

    out = {
        "metric": "RAV smoothed DoFs/s (whole V(2,2) solve to a 1e-8 residual reduction)",
        "value": value, "unit": "DoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded manufactured-solution forcing)",
        "config": {"workload": "2D Taylor-Hood Q2/Q1 Stokes 512x512, 7 levels, RAV V(2,2) omega 0.66, "
                               "solve from x0=0 to ||r|| <= 1e-8 ||r0||",
                   "dofs": n_fine, "levels": nl, "smoother": "rav", "nu": [nu, nu], "omega": omega,
                   "inverse_precision": "fp64", "inverse_format": args.format},
        "time_to_1e-8_ms": ms_step, "iters": int(np.median(iters)),
        "setup_s": round(setup_s, 3),
        "sweep": {"level": "512x512", "ms_residual": ms_res, "ms_apply": ms_apply,
                  "dofs_per_s": sweep_rate, "launches_timed": n_apply,
                  "pct_hbm_peak": 100.0 * (apply_bytes + resid_bytes) / sweep_s / 1e9 / HBM_PEAK_GBS},
        "roofline": {"bound": "hbm", "kernel": ("k_rav_apply_fact<2,double,1>" if args.format == "factored"
                                                else "k_rav_apply<2,VERTEX,0,double,1>") + " (512x512 level)",
                     "achieved": roof_apply, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": roof_apply / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes": apply_bytes},
        "roofline_residual": {"bound": "hbm", "achieved": roof_res, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": roof_res / HBM_PEAK_GBS, "algorithmic_bytes": resid_bytes},
    }

    if args.copy_calibration:
        out["copy_GBs"] = _copy_calibration()

    if not args.no_mixed:
        # the same problem by FGMRES(30) with one of these V-cycles as preconditioner
        out["fgmres"] = _gmres_timed(H, b)
        H.close()
        variants = {}
        esz = {"fp64": 8, "fp32": 4, "bf16": 2}
        for fmt in ("factored", "rows"):
            for prec in ("fp64", "fp32", "bf16"):
                if fmt == args.format and prec == "fp64":
                    continue
                Hm, st_s = setup(prec, fmt)
                run(Hm, 1)
                k = max(1, args.steps // 2)
                dtm, itm, pm = run(Hm, k, profile=True)
                variants[f"{fmt}_{prec}"] = {
                    "time_to_1e-8_ms": 1e3 * dtm / k, "iters": int(np.median(itm)),
                    "dofs_per_s": sum(itm) * smoothed_per_cycle / dtm, "ms_apply": pm[1], "ms_residual": pm[0],
                    "setup_s": round(st_s, 3),
                    "apply_GBs": (esz[prec] * w_entries(fmt) + 8 * n_fine + 16 * n_free) / (1e-3 * pm[1]) / 1e9}
                Hm.close()
        out["variants"] = variants
        out["q1q1_cavity_1024"] = q1q1_summary()
        out["adaptive_cavity_table1"] = adaptive_summary()
        out["adaptive_channel_table2"] = channel_summary()
    else:
        H.close()

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(out))


def _copy_calibration() -> float:
    """Launches the plain copy kernel on 1 GiB (13 times): the reference whose
    HBM counter readings scale the PMC traffic summaries.  Returns its GB/s."""
    import torch
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
    return 2 * n * 8 * 10 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9


def _line(metric, value, unit, steps, warmup, ms, dtype, config, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": dtype, "data": "synthetic (seeded manufactured-solution forcing)", "config": config}
    out.update(extra)
    print(json.dumps(out))


def bench_3d(args):
    """Finest-level RAV sweep (residual + apply) of the 3D element-patch workload.
    Element patches with a continuous Q1 pressure give no convergent V-cycle, so
    this workload is measured per sweep (rates only), for FP64/FP32/BF16 rows."""
    import torch
    from paper_2103_10127_amd import Hierarchy
    cfg = ri.CONFIGS["3d-64"]
    N, nl = cfg["n_cells"], cfg["n_levels"]
    reps = max(args.steps, 5)
    res = {}
    for prec in ("fp64", "fp32", "bf16"):
        t0 = time.perf_counter()
        H = Hierarchy(dim=3, n_cells=N, n_levels=nl, dmask=cfg["dmask"], kind="element", omega=0.5,
                      precision=prec)
        H.factor()
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        n_fine, n_free = H.dofs(nl - 1)
        b = torch.zeros(n_fine, dtype=torch.float64, device="cuda")
        H.assemble_rhs(ri.mms_params(3, cfg["seed"]), b)
        x = torch.zeros_like(b)
        H.time_sweep(nl - 1, max(args.warmup, 1), x, b)
        ms_res, ms_apply = H.time_sweep(nl - 1, reps, x, b)
        res[prec] = dict(ms_residual=ms_res, ms_apply=ms_apply, setup_s=round(setup, 3))
        H.close()
    esz = {"fp64": 8, "fp32": 4, "bf16": 2}
    sum_on = sum_owned_times_patch_3d_element(N)
    for prec, r in res.items():
        r["apply_GBs"] = (esz[prec] * sum_on + 8 * n_fine + 16 * n_free) / (1e-3 * r["ms_apply"]) / 1e9
    f = res["fp64"]
    apply_bytes = 8 * sum_on + 8 * n_fine + 16 * n_free
    resid_bytes = 24 * n_fine + 8 * N ** 3
    sweep_ms = f["ms_residual"] + f["ms_apply"]
    _line("RAV smoothed DoFs/s (finest-level sweep: residual + apply)", n_fine / (1e-3 * sweep_ms), "DoF/s",
          reps, max(args.warmup, 1), sweep_ms, "f64",
          {"workload": "3D Taylor-Hood Q2/Q1 64^3, 5 levels, RAV element patches, one finest-level sweep",
           "dofs": n_fine, "patches": N ** 3, "sum_owned_x_cols": sum_on},
          roofline={"bound": "hbm", "kernel": "k_rav_apply<3,ELEMENT,*,double> (64^3 level, 8 buckets)",
                    "achieved": apply_bytes / (1e-3 * f["ms_apply"]) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": apply_bytes / (1e-3 * f["ms_apply"]) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                    "algorithmic_bytes": apply_bytes},
          roofline_residual={"bound": "hbm", "achieved": resid_bytes / (1e-3 * f["ms_residual"]) / 1e9,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s", "algorithmic_bytes": resid_bytes},
          precisions=res)


def sum_owned_times_patch_3d_vertex(N: int) -> int:
    """sum_i (owned rows x patch columns) of all-Dirichlet 3D vertex patches:
    per axis a vertex k sees c(k) free node positions in [2k-2, 2k+2] and owns
    o(k) free positions in {2k, 2k+1}; n_i = 3 prod c + 1, owned_i = 3 prod o + 1."""
    k = np.arange(N + 1)
    c = np.minimum(2 * k + 2, 2 * N - 1) - np.maximum(2 * k - 2, 1) + 1
    o = np.maximum(np.minimum(2 * k + 1, 2 * N - 1) - np.maximum(2 * k, 1) + 1, 0)
    C = c[:, None, None] * c[None, :, None] * c[None, None, :]
    O = o[:, None, None] * o[None, :, None] * o[None, None, :]
    return int(np.sum((3 * C + 1) * (3 * O + 1)))


def bench_3d_vertex(args):
    """The 64^3 workload with pressure-vertex patches (376 local DoFs): the RAV
    V(2,2) solve from x0 = 0 to a 1e-8 reduction in FP64, FP32 and BF16 rows
    (element patches give no convergent cycle).  value = smoothed DoFs/s of
    the FP64 solve; roofline: the finest-level apply with HIP events."""
    import torch
    from paper_2103_10127_amd import Hierarchy
    cfg = ri.CONFIGS["3d-64"]
    N, nl = cfg["n_cells"], cfg["n_levels"]
    steps = max(args.steps // 2, 2)
    esz = {"fp64": 8, "fp32": 4, "bf16": 2}
    sum_on = sum_owned_times_patch_3d_vertex(N)
    fact_entries = (125 * 11 + 1) * (N + 1) ** 3
    res = {}
    runs = [(args.format, "fp64")] + [(args.format, p) for p in ("fp32", "bf16")] + \
        [("rows" if args.format == "factored" else "factored", "fp64")]
    for fmt, prec in runs:
        t0 = time.perf_counter()
        H = Hierarchy(dim=3, n_cells=N, n_levels=nl, dmask=cfg["dmask"], kind="vertex", omega=0.66, precision=prec,
                      inv_format=fmt)
        H.factor()
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        n_fine, n_free = H.dofs(nl - 1)
        level_n = [H.dofs(l)[0] for l in range(nl)]
        b = torch.zeros(n_fine, dtype=torch.float64, device="cuda")
        H.assemble_rhs(ri.mms_params(3, cfg["seed"]), b)
        x = torch.zeros_like(b)
        H.solve(x, b, 1e-8, 60)
        H.profile_begin(nl - 1, 4096)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = []
        for _ in range(steps):
            x.zero_()
            st, it, rel = H.solve(x, b, 1e-8, 60)
            if st != 0:
                raise RuntimeError(f"3D vertex solve {prec}: status {st}, {it} cycles, rel {rel}")
            its.append(it)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        ms_res, ms_apply, n_app = H.profile_end()
        apply_bytes = esz[prec] * (sum_on if fmt == "rows" else fact_entries) + 8 * n_fine + 16 * n_free
        res[f"{fmt}_{prec}"] = dict(time_to_1e_8_ms=1e3 * dt, iters=int(np.median(its)), setup_s=round(setup, 3),
                         ms_apply=ms_apply, ms_residual=ms_res, apply_GBs=apply_bytes / (1e-3 * ms_apply) / 1e9,
                         smoothed_dofs_per_s=int(np.median(its)) * sum(4 * level_n[l] for l in range(1, nl)) / dt)
        H.close()
    f = res[f"{args.format}_fp64"]
    apply_bytes = 8 * (sum_on if args.format == "rows" else fact_entries) + 8 * n_fine + 16 * n_free
    _line("RAV smoothed DoFs/s (whole V(2,2) solve to a 1e-8 residual reduction)", f["smoothed_dofs_per_s"], "DoF/s",
          steps, 1, f["time_to_1e_8_ms"], "f64",
          {"workload": "3D Taylor-Hood Q2/Q1 64^3, 5 levels, RAV with pressure-vertex patches (376 DoFs), V(2,2) "
                       "omega 0.66, solve from x0=0 to ||r|| <= 1e-8 ||r0||",
           "dofs": n_fine, "patches": (N + 1) ** 3, "sum_owned_x_cols": sum_on, "inverse_format": args.format},
          time_to_1e_8_ms=f["time_to_1e_8_ms"], iters=f["iters"],
          roofline={"bound": "hbm", "kernel": ("k_rav_apply_fact<3,double,1>" if args.format == "factored" else
                                               "k_rav_apply<3,VERTEX,0,double,1>") + " (64^3 level)",
                    "achieved": f["apply_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": f["apply_GBs"] / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": apply_bytes},
          precisions=res)


def bench_smoothers(args):
    """The paper's cost comparison (Sec. 4.3, eq. 15): per smoother, the time of
    one V(2,2) cycle, the cycles to a 1e-8 reduction and the total time, on the
    32x32 workload for the damping sweep omega in {0.5, 0.6, 0.66, 0.7, 0.8, 0.9,
    1.0} plus AV at 0.1, and on the 512x512 workload for RAV 0.66, MV 0.66 and
    AV 0.1.  value = the 512^2 RAV solve's smoothed DoFs/s."""
    import torch
    from paper_2103_10127_amd import Hierarchy

    def run(N, nl, smoother, omega, maxit):
        H = Hierarchy(dim=2, n_cells=N, n_levels=nl, dmask=ri.ALL_DIRICHLET_2D, smoother=smoother, omega=omega)
        t0 = time.perf_counter()
        H.factor()
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        n, _ = H.dofs(nl - 1)
        level_n = [H.dofs(l)[0] for l in range(nl)]
        b = torch.zeros(n, dtype=torch.float64, device="cuda")
        H.assemble_rhs(ri.mms_params(2, 1001 if N == 32 else 1002), b)
        x = torch.zeros_like(b)
        H.solve(x, b, 1e-8, maxit)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it, rel = H.solve(x, b, 1e-8, maxit)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            H.vcycle(x, b)
        torch.cuda.synchronize()
        cyc = (time.perf_counter() - t0) / reps
        H.close()
        status = {0: "converged", 1: "maxit", -4: "diverged"}.get(st, str(st))
        return {"smoother": smoother, "omega": omega, "status": status, "cycles": it, "rel_res": rel,
                "ms_per_cycle": 1e3 * cyc, "ms_total": 1e3 * total if st == 0 else None, "setup_s": round(setup, 3),
                "smoothed_per_cycle": sum(4 * level_n[l] for l in range(1, nl))}

    sweep = []
    for sm_ in ("rav", "mv", "av"):
        for om in (0.5, 0.6, 0.66, 0.7, 0.8, 0.9, 1.0) + ((0.1,) if sm_ == "av" else ()):
            sweep.append(run(32, 3, sm_, om, 300))
    big = [run(512, 7, "rav", 0.66, 100), run(512, 7, "mv", 0.66, 100), run(512, 7, "av", 0.1, 300)]
    r = big[0]
    _line("RAV smoothed DoFs/s (whole V(2,2) solve to a 1e-8 residual reduction)",
          r["cycles"] * r["smoothed_per_cycle"] / (1e-3 * r["ms_total"]), "DoF/s", 1, 1, r["ms_total"], "f64",
          {"workload": "RAV vs MV vs AV: 2D Q2/Q1 32x32 (3 levels, omega swept) and 512x512 (7 levels), V(2,2), "
                       "solve from x0=0 to 1e-8"},
          cost_512=big, damping_sweep_32=sweep)


def bench_cavity(args):
    """Driven cavity (Sec. 4.1): no-slip walls, lid velocity 1 on the top side,
    no forcing, 2D Q2/Q1, coarsest grid 8x8.  (a) Smoothing-steps study on the
    512x512 grid (7 levels; the study of Sec. 4.2, Fig. 7, done here on the
    cavity): for nu = 1..6 pre- and post-smoothing steps, RAV and MV at 0.66 and
    AV at 0.1, the cycles to 1e-8, the average reduction and the time.  (b) Mesh
    study at nu = 3 (Sec. 4.1, Fig. 4-5): N = 32 ... 512.  value = smoothed
    DoFs/s of the RAV V(3,3) solve at 512^2."""
    import torch
    from paper_2103_10127_amd import Hierarchy

    def solve(N, smoother, omega, nu, maxit=100):
        nl = int(np.log2(N // 8)) + 1
        H = Hierarchy(dim=2, n_cells=N, n_levels=nl, dmask=ri.ALL_DIRICHLET_2D, smoother=smoother, omega=omega,
                      nu_pre=nu, nu_post=nu, inv_format=args.format if smoother == "rav" else "rows")
        H.factor()
        n, _ = H.dofs(nl - 1)
        level_n = [H.dofs(l)[0] for l in range(nl)]
        b = torch.zeros(n, dtype=torch.float64, device="cuda")
        H.assemble_rhs_lid(b, 1.0)
        x = torch.zeros_like(b)
        H.solve(x, b, 1e-8, min(maxit, 3))
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it, rel = H.solve(x, b, 1e-8, maxit)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        H.close()
        status = {0: "converged", 1: "maxit", -4: "diverged"}.get(st, str(st))
        return {"smoother": smoother, "omega": omega, "nu": nu, "N": N, "status": status, "cycles": it,
                "rho_avg": rel ** (1.0 / it) if it > 0 and rel > 0 else None, "ms": 1e3 * dt,
                "ms_per_cycle": 1e3 * dt / max(it, 1),
                "smoothed_dofs": it * sum(2 * nu * level_n[l] for l in range(1, nl))}

    study = [solve(512, sm_, om, nu) for nu in range(1, 7)
             for sm_, om in (("rav", 0.66), ("mv", 0.66), ("av", 0.1))]
    mesh = [solve(N, sm_, om, 3) for N in (32, 64, 128, 256, 512)
            for sm_, om in (("rav", 0.66), ("mv", 0.66), ("av", 0.1))]
    r = next(e for e in mesh if e["N"] == 512 and e["smoother"] == "rav")
    _line("RAV smoothed DoFs/s (whole V(3,3) solve to a 1e-8 residual reduction)",
          r["smoothed_dofs"] / (1e-3 * r["ms"]), "DoF/s", 1, 1, r["ms"], "f64",
          {"workload": "2D driven cavity (lid velocity 1, no-slip walls), Taylor-Hood Q2/Q1, coarsest 8x8; "
                       "smoothing-steps study at 512x512 and mesh study at nu = 3; RAV/MV omega 0.66, AV 0.1",
           "inverse_format": args.format},
          smoothing_steps_512=study, mesh_study_nu3=mesh)


def q1q1_summary() -> dict:
    """The paper's own discretization beside the headline: stabilized Q1-Q1
    driven cavity on 1024^2 (3,151,875 DoFs), 8 levels, RAV V(3,3), omega
    0.66, beta 0.05, factored inverse, solve to 1e-8 (best of 3)."""
    import torch
    from paper_2103_10127_amd import Hierarchy
    N, nl = 1024, 8
    H = Hierarchy(dim=2, n_cells=N, n_levels=nl, dmask=ri.ALL_DIRICHLET_2D, nu_pre=3, nu_post=3, omega=0.66,
                  inv_format="factored", discretization="q1q1", beta=0.05)
    H.factor()
    n, _ = H.dofs(nl - 1)
    level_n = [H.dofs(l)[0] for l in range(nl)]
    b = torch.zeros(n, dtype=torch.float64, device="cuda")
    H.assemble_rhs_lid(b, 1.0)
    x = torch.zeros_like(b)
    H.solve(x, b, 1e-8, 3)
    best, st, it = None, None, 0
    for _ in range(3):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it, _ = H.solve(x, b, 1e-8, 200)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    H.close()
    return {"dofs": n, "status": "converged" if st == 0 else str(st), "cycles": it,
            "time_to_1e-8_ms": 1e3 * best,
            "smoothed_dofs_per_s": it * sum(6 * level_n[l] for l in range(1, nl)) / best}


def _adaptive_solve_summary(H, b, n_grids, setup) -> dict:
    """Best of three RAV V(3,3) solves to 1e-8 after a warm solve."""
    import torch
    n = H.dofs(n_grids - 1)[0]
    level_n = [H.dofs(l)[0] for l in range(n_grids)]
    x = torch.zeros_like(b)
    H.solve(x, b, 1e-8, 2)
    best, st, it = None, None, 0
    for _ in range(3):
        x.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, it, _ = H.solve(x, b, 1e-8, 200)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        best = dt if best is None else min(best, dt)
    H.close()
    return {"dofs": n, "status": "converged" if st == 0 else str(st), "cycles": it,
            "time_to_1e-8_ms": 1e3 * best, "setup_s": round(setup, 2),
            "smoothed_dofs_per_s": it * sum(6 * level_n[l] for l in range(1, n_grids)) / best}


def adaptive_summary() -> dict:
    """The paper's own grids beside the headline: stabilized Q1-Q1 driven cavity
    on the adaptive hierarchy of Table 1 (Omega^1..Omega^10, 3,063,075 DoFs),
    RAV V(3,3), omega 0.66, beta 0.05, solve to 1e-8 (best of 3)."""
    import torch
    from paper_2103_10127_amd.capi import AdaptiveHierarchy
    n_grids = 10
    t0 = time.perf_counter()
    H = AdaptiveHierarchy(ri.cavity_grids(n_grids), ri.lattice(n_grids), smoother="rav", omega=0.66, nu_pre=3,
                          nu_post=3, beta=0.05)
    H.factor()
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    b = torch.zeros(H.dofs(n_grids - 1)[0], dtype=torch.float64, device="cuda")
    H.assemble_rhs_lid(b, 1.0)
    return _adaptive_solve_summary(H, b, n_grids, setup)


def channel_summary() -> dict:
    """The second benchmark's setting beside the headline: flow past a cylinder
    on the stand-in of Table 2's hierarchy (Omega^1..Omega^7, 1,680,678 DoFs),
    parabolic inflow (mean 0.3 m/s), open outflow, RAV V(3,3), omega 0.66,
    beta 0.05, solve to 1e-8 (best of 3)."""
    import torch
    from paper_2103_10127_amd import capi
    n_grids = 7
    grids, Mx, My = ri.channel_grids(n_grids)
    t0 = time.perf_counter()
    H = capi.AdaptiveHierarchy(grids, Mx, smoother="rav", omega=0.66, nu_pre=3, nu_post=3, beta=0.05,
                               lattice_y=My, dmask=ri.OUTFLOW_2D)
    H.factor()
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    V = capi.adaptive_host_export(grids, Mx, n_grids - 1, "vertices", lattice_y=My, dmask=ri.OUTFLOW_2D)
    y = V[:, 1] / My
    ud = np.zeros((2, len(V)))
    ud[0] = np.where(V[:, 0] == 0, 4.0 * 0.3 * y * (1.0 - y), 0.0)
    b = torch.zeros(H.dofs(n_grids - 1)[0], dtype=torch.float64, device="cuda")
    H.assemble_rhs_dirichlet(ud, b)
    return _adaptive_solve_summary(H, b, n_grids, setup)


def bench_q1q1(args):
    """The paper's own discretization, stabilized equal-order Q1-Q1 (eq. 8), with
    the literal RAV owned set (pressure + co-located velocity, Sec. 3): the
    driven cavity (Sec. 4.1) on 1024^2 (3,151,875 DoFs, close to the 3,063,075 of
    the finest Table 1 grid), 8 levels down to Table 1's coarsest 8x8 grid (243
    DoFs), RAV V(3,3) as in Sec. 4, omega 0.66, beta 0.05, factored inverse,
    solved from 0 to a 1e-8 residual reduction.  Also: the Galerkin hierarchy,
    a beta sweep, the finest-level residual/apply times with the apply's byte
    roofline, and a 3D 64^3 cavity-like solve (all-Dirichlet, manufactured
    forcing), RAV against MV (omega 0.66) and AV (omega 0.1) on the 1024^2
    cavity (time per cycle, cycles, total), the smoothing-steps study nu = 1..6
    at 1024^2 and the mesh study N = 64..512 at nu = 3.  value = smoothed DoFs/s
    of the 2D rediscretised RAV solve."""
    import torch
    from paper_2103_10127_amd import Hierarchy

    def run(dim, N, nl, beta, gal, rhs, reps=3, smoother="rav", omega=0.66, nu=3, sweep_times=True):
        dm = ri.ALL_DIRICHLET_2D if dim == 2 else ri.ALL_DIRICHLET_3D
        t0 = time.perf_counter()
        H = Hierarchy(dim=dim, n_cells=N, n_levels=nl, dmask=dm, nu_pre=nu, nu_post=nu, omega=omega,
                      smoother=smoother, galerkin=gal, inv_format="factored", discretization="q1q1", beta=beta)
        H.factor()
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        n, nfree = H.dofs(nl - 1)
        level_n = [H.dofs(l)[0] for l in range(nl)]
        b = torch.zeros(n, dtype=torch.float64, device="cuda")
        if rhs == "lid":
            H.assemble_rhs_lid(b, 1.0)
        else:
            H.assemble_rhs(ri.mms_params(dim, 1003), b)
        x = torch.zeros_like(b)
        H.solve(x, b, 1e-8, 3)
        best = None
        for _ in range(reps):
            x.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st, it, rel = H.solve(x, b, 1e-8, 200)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            best = dt if best is None else min(best, dt)
        ms_res, ms_apply = H.time_sweep(nl - 1, 20, x, b) if smoother != "mv" and sweep_times else (None, None)
        H.close()
        return {"dim": dim, "N": N, "levels": nl, "beta": beta, "coarse": "galerkin" if gal else "rediscretised",
                "smoother": smoother, "omega": omega, "ms_per_cycle": 1e3 * best / max(it, 1),
                "dofs": n, "status": {0: "converged", 1: "maxit", -4: "diverged"}.get(st, str(st)), "cycles": it,
                "rho_avg": rel ** (1.0 / it) if it > 0 and rel > 0 else None, "ms": 1e3 * best,
                "setup_s": round(setup, 3), "ms_residual": ms_res, "ms_apply": ms_apply,
                "nu": nu, "smoothed_dofs": it * sum(2 * nu * level_n[l] for l in range(1, nl))}

    main = run(2, 1024, 8, 0.05, False, "lid")
    gal = run(2, 1024, 8, 0.05, True, "lid", reps=1)
    sweep = [run(2, 1024, 8, beta, False, "lid", reps=1) for beta in (0.02, 0.1, 0.3, 1.0)]
    three = run(3, 64, 5, 0.05, False, "mms")
    # the paper's comparison (Sec. 4.1, Fig. 5) on its own discretization: RAV vs MV vs AV
    smoothers = [main] + [run(2, 1024, 8, 0.05, False, "lid", reps=1, smoother=sm_, omega=om)
                          for sm_, om in (("mv", 0.66), ("av", 0.1))]
    # smoothing steps (Sec. 4.2, Fig. 7) at 1024^2 and the mesh study at nu = 3
    steps = [run(2, 1024, 8, 0.05, False, "lid", reps=1, smoother=sm_, omega=om, nu=nu, sweep_times=False)
             for nu in range(1, 7) for sm_, om in (("rav", 0.66), ("mv", 0.66), ("av", 0.1))]
    mesh = [run(2, N, int(np.log2(N // 8)) + 1, 0.05, False, "lid", reps=1, smoother=sm_, omega=om,
                sweep_times=False)
            for N in (64, 128, 256, 512) for sm_, om in (("rav", 0.66), ("mv", 0.66), ("av", 0.1))]
    nV = 1025 ** 2
    apply_bytes = nV * (8 * (3 * 9 + 1) + 3 * 8 + 2 * 3 * 8)   # stored values, r once, x read and written
    achieved = apply_bytes / (main["ms_apply"] * 1e-3) / 1e9
    _line("RAV smoothed DoFs/s (whole V(3,3) solve to a 1e-8 residual reduction, stabilized Q1-Q1)",
          main["smoothed_dofs"] / (1e-3 * main["ms"]), "DoF/s", 1, 1, main["ms"], "f64",
          {"workload": "2D driven cavity, stabilized Q1-Q1 (beta 0.05), 1024x1024 (3,151,875 DoFs), 8 levels to "
                       "the 8x8 grid, RAV with pressure + co-located velocity owned, V(3,3), omega 0.66, factored"},
          roofline_apply={"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                          "frac": achieved / 8000.0, "bytes_per_launch": apply_bytes},
          rediscretised=main, galerkin=gal, beta_sweep=sweep, three_d_64=three, smoothers_1024=smoothers,
          smoothing_steps_1024=steps, mesh_study_nu3=mesh)


def bench_adaptive(args):
    """The paper's driven-cavity study on its own grids (Sec. 4.1, Table 1,
    Fig. 5): stabilized Q1-Q1 (beta 0.05) on the adaptively refined quadtree
    hierarchy Omega^1 .. Omega^10 (243 .. 3,063,075 DoFs, hanging nodes),
    V(3,3) solves from 0 to a 1e-8 residual reduction with RAV and MV
    (omega 0.66) and AV (omega 0.1), for every fine grid Omega^k, k = 2..10
    (hierarchy Omega^1..Omega^k): cycles, average reduction factor, time per
    cycle and total time.  value = smoothed DoFs/s of the RAV solve on
    Omega^10; the finest-level residual and RAV apply are timed with their
    byte rooflines."""
    import torch
    from paper_2103_10127_amd.capi import AdaptiveHierarchy

    n_grids = 10
    grids, M = ri.cavity_grids(n_grids), ri.lattice(n_grids)

    def run(k, smoother, omega, reps=1, sweep_times=False, gmres=False):
        t0 = time.perf_counter()
        H = AdaptiveHierarchy(grids[:k], M, smoother=smoother, omega=omega, nu_pre=3, nu_post=3, beta=0.05)
        H.factor()
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        n, _ = H.dofs(k - 1)
        level_n = [H.dofs(l)[0] for l in range(k)]
        b = torch.zeros(n, dtype=torch.float64, device="cuda")
        H.assemble_rhs_lid(b, 1.0)
        x = torch.zeros_like(b)
        H.solve(x, b, 1e-8, 2)
        best = None
        for _ in range(reps):
            x.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st, it, rel = H.solve(x, b, 1e-8, 300)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            best = dt if best is None else min(best, dt)
        out = {"grid": k, "dofs": n, "smoother": smoother, "omega": omega,
               "status": {0: "converged", 1: "maxit", -4: "diverged"}.get(st, str(st)), "cycles": it,
               "rho_avg": rel ** (1.0 / it) if it > 0 and rel > 0 else None, "ms": 1e3 * best,
               "ms_per_cycle": 1e3 * best / max(it, 1), "setup_s": round(setup, 2),
               "smoothed_dofs": it * sum(6 * level_n[l] for l in range(1, k))}
        if gmres:
            out["fgmres"] = _gmres_timed(H, b)
        if sweep_times:
            out["level_info"] = H.level_info(k - 1)
            out["ms_residual"], out["ms_apply"] = H.time_sweep(k - 1, 20, x, b)
        H.close()
        return out

    main = run(n_grids, "rav", 0.66, reps=3, sweep_times=True, gmres=not args.quick)
    print(f"adaptive Omega^10 RAV: {main['cycles']} cycles, {main['ms']:.1f} ms", file=sys.stderr, flush=True)
    extra = {}
    if args.copy_calibration:
        extra["copy_GBs"] = _copy_calibration()
    study = []
    for k in (range(2, n_grids + 1) if not args.quick else ()):
        for sm_, om in (("rav", 0.66), ("mv", 0.66), ("av", 0.1)):
            study.append(main if (k == n_grids and sm_ == "rav") else run(k, sm_, om, sweep_times=k == n_grids))
            r = study[-1]
            print(f"  Omega^{k} {sm_}: {r['cycles']} cycles, {r['ms']:.1f} ms", file=sys.stderr, flush=True)
    info = main["level_info"]
    nV, nnz, pnnz = info["vertices"], info["operator_entries"], info["patch_entries"]
    wide = info["wide"]
    # per launch on Omega^10: residual: one packed word per operator entry
    # (column offset + value-tuple id; 8 bytes in the wide format), x read once,
    # b read and r written (3 fields each), the mask byte; apply: the vertex of
    # every patch entry (int32), the configuration id, r read once, x read and
    # written.  The value and configuration tables (a few hundred entries) stay
    # in cache and are not counted.
    res_bytes = (8 if wide else 4) * nnz + 73 * nV
    app_bytes = 4 * pnnz + 76 * nV
    ach_res = res_bytes / (main["ms_residual"] * 1e-3) / 1e9
    ach_app = app_bytes / (main["ms_apply"] * 1e-3) / 1e9
    from paper_2103_10127_amd.profiling import ADAPTIVE_SOURCES, read_traffic
    traffic = read_traffic(os.path.join(ROOT, "profiles", "rav_apply_adaptive_omega10_traffic.md"), ADAPTIVE_SOURCES)
    _line("RAV smoothed DoFs/s (whole V(3,3) solve to a 1e-8 residual reduction, adaptive grids)",
          main["smoothed_dofs"] / (1e-3 * main["ms"]), "DoF/s", 3, 1, main["ms"], "f64",
          {"workload": "2D driven cavity, stabilized Q1-Q1 (beta 0.05) on the adaptive quadtree hierarchy "
                       "Omega^1..Omega^10 of Table 1 (3,063,075 DoFs on Omega^10, hanging nodes), RAV V(3,3), "
                       "omega 0.66"},
          data="synthetic (the Table 1 grids from the boundary-band refinement rule, lid velocity 1)",
          roofline={"bound": "hbm", "kernel": "k_ad_rav (Omega^10)", "achieved": ach_app, "peak": 8000.0,
                    "unit": "GB/s", "frac": ach_app / 8000.0, "traffic": traffic, "algorithmic_bytes": app_bytes},
          roofline_residual={"bound": "hbm", "kernel": "k_ad_residual (Omega^10)", "achieved": ach_res,
                             "peak": 8000.0, "unit": "GB/s", "frac": ach_res / 8000.0, "algorithmic_bytes": res_bytes},
          omega10=info,
          rav_omega10=main, fig5_study=study, **extra)


def _gmres_timed(H, b, reps=3, restart=30):
    """Best of `reps` FGMRES(restart) solves to 1e-8 preconditioned by the
    context's V-cycle: V-cycles used and time."""
    import torch
    x = torch.zeros_like(b)
    H.solve_gmres(x, b, 1e-8, 2, restart)
    best, st, it = None, None, 0
    for _ in range(reps):
        x.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, it, rel = H.solve_gmres(x, b, 1e-8, 300, restart)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        best = dt if best is None else min(best, dt)
    return {"status": {0: "converged", 1: "maxit", -4: "diverged"}.get(st, str(st)), "vcycles": it,
            "ms": 1e3 * best, "restart": restart}


def bench_channel(args):
    """The paper's second benchmark (Sec. 4.2, Table 2, Figs. 7-9) on a
    stand-in of its grids: Stokes flow through a channel past a cylindrical
    obstacle, parabolic inflow (eq. 14, mean 0.3 m/s), no slip on the walls
    and the obstacle, open outflow; stabilized Q1-Q1 (beta 0.05) on the
    adaptive hierarchy Omega^1 .. Omega^7 of rav_inputs.channel_grids (counts
    within 2 % of Table 2's, 1,680,678 DoFs on Omega^7).  Mesh study: V(3,3)
    solves to a 1e-8 residual reduction with RAV and MV (omega 0.66) and AV
    (omega 0.1) for every fine grid Omega^k, k = 2..7 (Figs. 8-9); smoothing
    steps study on Omega^7: V(n,n), n = 1..6, for the three smoothers (Fig. 7).
    value = smoothed DoFs/s of the RAV V(3,3) solve on Omega^7."""
    import torch
    from paper_2103_10127_amd import capi
    from paper_2103_10127_amd.capi import AdaptiveHierarchy

    n_grids = 7
    grids, Mx, My = ri.channel_grids(n_grids)
    dmask = ri.OUTFLOW_2D
    ubar = 0.3

    inflow_cache = {}

    def inflow(k):
        if k not in inflow_cache:
            V = capi.adaptive_host_export(grids[:k], Mx, k - 1, "vertices", lattice_y=My, dmask=dmask)
            y = V[:, 1] / My
            ud = np.zeros((2, len(V)))
            ud[0] = np.where(V[:, 0] == 0, 4.0 * ubar * y * (1.0 - y), 0.0)
            inflow_cache[k] = ud
        return inflow_cache[k]

    def make(k, smoother, omega, nu):
        t0 = time.perf_counter()
        H = AdaptiveHierarchy(grids[:k], Mx, smoother=smoother, omega=omega, nu_pre=nu, nu_post=nu, beta=0.05,
                              lattice_y=My, dmask=dmask)
        H.factor()
        torch.cuda.synchronize()
        n, _ = H.dofs(k - 1)
        b = torch.zeros(n, dtype=torch.float64, device="cuda")
        H.assemble_rhs_dirichlet(inflow(k), b)
        return H, b, time.perf_counter() - t0

    def solve(H, b, k, smoother, omega, nu, reps=1, maxit=300):
        level_n = [H.dofs(l)[0] for l in range(k)]
        x = torch.zeros_like(b)
        H.solve(x, b, 1e-8, 2)
        best = None
        for _ in range(reps):
            x.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st, it, rel = H.solve(x, b, 1e-8, maxit)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            best = dt if best is None else min(best, dt)
        return {"grid": k, "dofs": level_n[-1], "smoother": smoother, "omega": omega, "nu": nu,
                "status": {0: "converged", 1: "maxit", -4: "diverged"}.get(st, str(st)), "cycles": it,
                "rho_avg": rel ** (1.0 / it) if it > 0 and rel > 0 else None, "ms": 1e3 * best,
                "ms_per_cycle": 1e3 * best / max(it, 1),
                "smoothed_dofs": it * sum(2 * nu * level_n[l] for l in range(1, k))}

    H, b, setup = make(n_grids, "rav", 0.66, 3)
    main = solve(H, b, n_grids, "rav", 0.66, 3, reps=3)
    main["setup_s"] = round(setup, 2)
    main["level_info"] = info = H.level_info(n_grids - 1)
    if not args.quick:
        main["fgmres"] = _gmres_timed(H, b)
    xs = torch.zeros_like(b)
    main["ms_residual"], main["ms_apply"] = H.time_sweep(n_grids - 1, 20, xs, b)
    # bytes per launch on Omega^7, counted as for the cavity grids
    app_bytes = 4 * info["patch_entries"] + 76 * info["vertices"]
    ach_app = app_bytes / (main["ms_apply"] * 1e-3) / 1e9
    print(f"channel Omega^7 RAV: {main['cycles']} cycles, {main['ms']:.1f} ms", file=sys.stderr, flush=True)
    steps = []
    if not args.quick:
        for sm_, om in (("rav", 0.66), ("mv", 0.66), ("av", 0.1)):
            Hs = H if sm_ == "rav" else make(n_grids, sm_, om, 3)[0]
            for nu in range(1, 7):
                Hs.set_params(om, nu, nu)
                steps.append(solve(Hs, b, n_grids, sm_, om, nu, maxit=200))
                r = steps[-1]
                print(f"  nu={nu} {sm_}: {r['status']} {r['cycles']} cycles, {r['ms']:.1f} ms", file=sys.stderr,
                      flush=True)
            if Hs is not H:
                Hs.close()
    H.close()
    study = []
    for k in (range(2, n_grids + 1) if not args.quick else ()):
        for sm_, om in (("rav", 0.66), ("mv", 0.66), ("av", 0.1)):
            if k == n_grids and sm_ == "rav":
                study.append(main)
                continue
            Hk, bk, st_ = make(k, sm_, om, 3)
            study.append(solve(Hk, bk, k, sm_, om, 3))
            study[-1]["setup_s"] = round(st_, 2)
            Hk.close()
            r = study[-1]
            print(f"  Omega^{k} {sm_}: {r['cycles']} cycles, {r['ms']:.1f} ms", file=sys.stderr, flush=True)
    _line("RAV smoothed DoFs/s (whole V(3,3) solve to a 1e-8 residual reduction, channel with an obstacle)",
          main["smoothed_dofs"] / (1e-3 * main["ms"]), "DoF/s", 3, 1, main["ms"], "f64",
          {"workload": "2D channel past a cylindrical obstacle (parabolic inflow, mean 0.3 m/s; open outflow), "
                       "stabilized Q1-Q1 (beta 0.05) on a 7-grid adaptive quadtree hierarchy standing in for "
                       "Table 2's (1,680,678 DoFs on Omega^7, hanging nodes), RAV V(3,3), omega 0.66"},
          data="synthetic (64 x 12 coarse cells minus the six inside the cylinder, refined towards the walls "
               "and the obstacle)",
          roofline={"bound": "hbm", "kernel": "k_ad_rav (Omega^7)", "achieved": ach_app, "peak": 8000.0,
                    "unit": "GB/s", "frac": ach_app / 8000.0, "traffic": None, "algorithmic_bytes": app_bytes},
          rav_omega7=main, fig7_smoothing_steps=steps, fig89_mesh_study=study)


def bench_1024(args):
    """2D 1024^2 with inclusions at contrast 1e4: the finest-level RAV sweep rate
    (FP64 and BF16 rows), plus the outcome of the solvers on this problem: plain
    RAV V(2,2) cycles and FGMRES(30) right-preconditioned by one V-cycle both fail
    to converge at this contrast (the coarse-grid correction amplifies the
    residual; see the findings in the design notes), which is recorded rather
    than hidden."""
    import torch
    from paper_2103_10127_amd import Hierarchy
    cfg = ri.CONFIGS["2d-1024"]
    N, nl = cfg["n_cells"], cfg["n_levels"]
    incl = ri.inclusions(cfg["seed"])
    reps = max(args.steps, 5)
    res = {}
    gm = vc = None
    for prec in ("fp64", "bf16"):
        t0 = time.perf_counter()
        H = Hierarchy(dim=2, n_cells=N, n_levels=nl, dmask=cfg["dmask"], omega=0.66, eta_out=cfg["eta_out"],
                      eta_in=cfg["contrast"], inclusions=incl, precision=prec)
        H.factor()
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        n_fine, n_free = H.dofs(nl - 1)
        b = torch.zeros(n_fine, dtype=torch.float64, device="cuda")
        H.assemble_rhs(ri.mms_params(2, cfg["seed"]), b)
        x = torch.zeros_like(b)
        H.time_sweep(nl - 1, max(args.warmup, 1), x, b)
        ms_res, ms_apply = H.time_sweep(nl - 1, reps, x, b)
        res[prec] = dict(ms_residual=ms_res, ms_apply=ms_apply, setup_s=round(setup, 3))
        if prec == "fp64":
            x.zero_()
            st, it, rel = H.solve(x, b, 1e-8, 30)
            vc = {"status": st, "cycles": it, "rel_residual": rel}
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, it, rel = H.solve_gmres(x, b, 1e-8, 150, 30)
            torch.cuda.synchronize()
            gm = {"status": st, "iterations": it, "rel_residual": rel, "ms": 1e3 * (time.perf_counter() - t0)}
        H.close()
    esz = {"fp64": 8, "bf16": 2}
    sum_on = sum_owned_times_patch(N)
    for prec, r in res.items():
        r["apply_GBs"] = (esz[prec] * sum_on + 8 * n_fine + 16 * n_free) / (1e-3 * r["ms_apply"]) / 1e9
    f = res["fp64"]
    apply_bytes = 8 * sum_on + 8 * n_fine + 16 * n_free
    sweep_ms = f["ms_residual"] + f["ms_apply"]
    _line("RAV smoothed DoFs/s (finest-level sweep: residual + apply)", n_fine / (1e-3 * sweep_ms), "DoF/s",
          reps, max(args.warmup, 1), sweep_ms, "f64",
          {"workload": "2D Taylor-Hood Q2/Q1 1024x1024, 8 levels, inclusions at viscosity contrast 1e4, "
                       "one finest-level RAV sweep (omega 0.66)",
           "dofs": n_fine, "levels": nl, "inclusions": len(incl)},
          roofline={"bound": "hbm", "kernel": "k_rav_apply<2,VERTEX,0,double> (1024x1024 level)",
                    "achieved": apply_bytes / (1e-3 * f["ms_apply"]) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": apply_bytes / (1e-3 * f["ms_apply"]) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                    "algorithmic_bytes": apply_bytes},
          precisions=res, vcycle_solve=vc, gmres_solve=gm)


def bench_batch(args):
    """256 independent 2D problems (fine grids 64/128/256, coarsest 16^2, 1-8
    inclusions each at contrast 1e3) advanced together.  value = smoothed
    DoFs/s of one batched V(2,2) cycle of all problems (one launch per stage for
    the whole batch, captured cycle).  At this contrast plain V-cycles do not
    converge for most problems, so the time to 1e-8 is measured with the
    batched FGMRES(30) preconditioned by one cycle, for V(2,2), V(4,4), V(3,3)
    with Galerkin coarse operators and V(4,4) with BF16 rows; each entry
    reports how many of the 256 problems reached 1e-8 within 300 cycles."""
    import torch
    from paper_2103_10127_amd.capi import Batch
    cfg = ri.CONFIGS["batch256"]
    sizes = ri.batch_sizes(cfg["n_problems"], cfg["seed"])

    def make(nu, galerkin=False, precision="fp64"):
        probs = [dict(dim=2, n_cells=int(n), n_levels=ri.levels_to(int(n), cfg["coarsest"]), dmask=cfg["dmask"],
                      eta_out=cfg["eta_out"], eta_in=cfg["contrast"], inclusions=ri.inclusions(cfg["seed"] + i),
                      omega=0.66, nu_pre=nu, nu_post=nu, galerkin=galerkin, precision=precision,
                      inv_format=args.format)
                 for i, n in enumerate(sizes)]
        t0 = time.perf_counter()
        B = Batch(probs)
        B.factor()
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        xs, bs = [], []
        for i in range(len(probs)):
            n, _ = B.dofs(i)
            bb = torch.zeros(n, dtype=torch.float64, device="cuda")
            B.assemble_rhs(i, ri.mms_params(2, cfg["seed"] + i), bb)
            bs.append(bb)
            xs.append(torch.zeros_like(bb))
        return B, probs, xs, bs, setup

    def gmres(B, xs, bs):
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, its, rel = B.solve_gmres(xs, bs, 1e-8, 300, 30)
        torch.cuda.synchronize()
        rel = np.asarray(rel)
        return {"converged": int((rel <= 1e-8).sum()), "of": len(rel), "ms": 1e3 * (time.perf_counter() - t0),
                "cycles_median": float(np.median(its)), "cycles_max": int(max(its))}

    B, probs, xs, bs, setup = make(2)
    for _ in range(max(args.warmup, 1)):
        B.vcycle(xs, bs)
    for x in xs:
        x.zero_()
    steps = max(args.steps, 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        B.vcycle(xs, bs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    smoothed = 0
    for p in probs:
        for l in range(1, p["n_levels"]):
            n_l = p["n_cells"] >> (p["n_levels"] - 1 - l)
            smoothed += 2 * 2 * (2 * (2 * n_l + 1) ** 2 + (n_l + 1) ** 2)
    total = sum(B.dofs(i)[0] for i in range(len(probs)))
    solves = {"fgmres30_v22": gmres(B, xs, bs)}
    B.close()
    for label, nu, gal, prec in (("fgmres30_v44", 4, False, "fp64"), ("fgmres30_v33_galerkin", 3, True, "fp64"),
                                 ("fgmres30_v44_bf16", 4, False, "bf16")):
        B, _, xs, bs, st_s = make(nu, gal, prec)
        solves[label] = gmres(B, xs, bs)
        solves[label]["setup_s"] = round(st_s, 3)
        B.close()
    _line("RAV smoothed DoFs/s (batched V(2,2) cycles)", smoothed / dt, "DoF/s", steps, max(args.warmup, 1),
          1e3 * dt, "f64",
          {"workload": "256 independent 2D Q2/Q1 problems (fine 64/128/256, coarsest 16x16), 1-8 inclusions "
                       "each at contrast 1e3, one batched RAV V(2,2) cycle per step",
           "problems": len(probs), "dofs_total": total, "inverse_format": args.format},
          setup_s=round(setup, 3), solves=solves)


def bench_learned(args):
    """Learned per-patch damping (eq. 11's per-subdomain weights from a network):
    trained on the asymptotic two-grid objective (6 warm cycles with the current
    weights, then one differentiated cycle) on 12 two-level 32^2/64^2 problems
    with inclusions at contrast 1e2 (seeds 3000-3011) and Galerkin coarse
    operators; evaluated on held-out problems (seeds 4000-4007 at 128^2, 5
    levels; 4000-4003 at 256^2, 6 levels), V(2,2) to 1e-8 (at most 300 cycles),
    against fixed omega in {0.5, 0.6, 0.66, 0.75, 0.85}.  value = smoothed
    DoFs/s of the learned-omega solves."""
    import torch
    from paper_2103_10127_amd import Hierarchy
    from paper_2103_10127_amd.capi import MLP
    from paper_2103_10127_amd.learn import train
    contrast, maxit = 100.0, 300
    train_probs = [dict(dim=2, n_cells=32 if i < 8 else 64, n_levels=2, dmask=ri.ALL_DIRICHLET_2D, eta_out=1.0,
                        eta_in=contrast, inclusions=ri.inclusions(3000 + i), omega=0.66, galerkin=True)
                   for i in range(12)]
    t0 = time.perf_counter()
    theta, losses = train(train_probs, steps=args.train_steps, lr=args.train_lr, seed=0, warm_cycles=6)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    net = MLP(theta)
    omegas = (0.5, 0.6, 0.66, 0.75, 0.85)
    labels = [f"fixed {om}" for om in omegas] + ["learned"]
    rows = []
    tot = {k: {"cycles": 0, "failed": 0, "s": 0.0, "dofs": 0} for k in labels}
    for N, nl, seeds in ((128, 5, range(4000, 4008)), (256, 6, range(4000, 4004))):
        for seed in seeds:
            H = Hierarchy(dim=2, n_cells=N, n_levels=nl, dmask=ri.ALL_DIRICHLET_2D, eta_out=1.0, eta_in=contrast,
                          inclusions=ri.inclusions(seed), omega=0.66, galerkin=True)
            H.factor()
            n_fine, _ = H.dofs(nl - 1)
            level_n = [H.dofs(l)[0] for l in range(nl)]
            per_cycle = sum(2 * 2 * level_n[l] for l in range(1, nl))
            b = torch.zeros(n_fine, dtype=torch.float64, device="cuda")
            H.assemble_rhs(ri.mms_params(2, seed), b)
            x = torch.zeros_like(b)
            row = {"N": N, "seed": seed}
            for label in labels:
                if label == "learned":
                    H.set_params(0.66, 2, 2)
                    H.learn_set_omega(net)
                else:
                    H.learn_set_omega(None)
                    H.set_params(float(label.split()[1]), 2, 2)
                x.zero_()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st, it, rel = H.solve(x, b, 1e-8, maxit)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t1
                row[label] = it if st == 0 else None
                t = tot[label]
                t["cycles"] += it if st == 0 else maxit
                if st == 0:
                    t["s"] += dt
                    t["dofs"] += it * per_cycle
                else:
                    t["failed"] += 1
            rows.append(row)
            H.close()
    net.close()
    L = tot["learned"]
    rate = L["dofs"] / L["s"] if L["s"] > 0 else None
    _line("RAV smoothed DoFs/s (whole V(2,2) solve to a 1e-8 residual reduction, learned per-patch omega)",
          rate, "DoF/s", len(rows), 1, 1e3 * L["s"] / max(len(rows) - L["failed"], 1), "f64",
          {"workload": "2D Taylor-Hood Q2/Q1 with 1-8 inclusions at contrast 1e2, Galerkin coarse operators, "
                       "RAV V(2,2); network trained on the asymptotic two-grid objective on 12 two-level "
                       "32^2/64^2 problems; 12 held-out problems (8 at 128^2, 4 at 256^2)",
           "train_steps": args.train_steps, "train_lr": args.train_lr},
          train_s=round(train_s, 2), loss_first=float(np.mean(losses[:48])), loss_last=float(np.mean(losses[-48:])),
          totals={k: {"cycles (failure = 300)": v["cycles"], "failed": v["failed"]} for k, v in tot.items()},
          problems=rows)


if __name__ == "__main__":
    main()
