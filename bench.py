"""Benchmark: batched ADMM plan-iterations/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 1]

Workload (default): the medium multi-target case, three targets, N = 40,000
dose points x 1,440 shot columns (60 isocentres x 8 sectors x 3 collimators),
81 plans from a 9 x 9 slider grid, FP32 dose block and iterates, FP64 Schur
complement inverse and small side.  The case is built and made resident in HBM
before timing (the setup time is reported beside the result).

A step is one pass of the whole iteration path over the 81-plan batch: 50 ADMM
iterations (right-hand-side product, Schur solve, small-side update, closed-form
x-step with the fused z- and y-steps) followed by one convergence check (the
planning objective of the current shot times, the duality gap and the
primal/dual residuals of every plan).  Plans are not frozen during the timed
steps, so every step does the same work.  value = plans x iterations / time.

Beside it: per-kernel device times from HIP events on the solver's stream over
the timed region (the roofline entry uses the dominant kernel), the FP64 CPU
oracle timed on a bounded sample of the same workload, and the wall time of a
full 81-plan sweep solved to a 1e-3 relative gap.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published dense peaks
    "f32_mfma_tflops": 157.3,
    "f64_mfma_tflops": 78.6,
    "hbm_gbs": 8000.0,
}
ITERS_PER_STEP = 50


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--precision", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def cpu_baseline(case, w, rho0, budget_s):
    """The FP64 oracle ADMM on the host cores, on a bounded sample of iterations."""
    from threadpoolctl import threadpool_info
    from oracle import lp as olp
    from oracle import admm as oadmm
    from synth import cases
    lp = olp.assemble(case, w)
    slp = olp.precondition(lp, olp.bot_scale(case))
    rho = olp.rho_rule(w[:, 3], rho0, cases.W0_BOT)
    fac, _ = oadmm.schur_factor(slp)
    st = oadmm.admm_iterate(slp, rho, 1, factor=fac)     # warm-up
    iters = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        st = oadmm.admm_iterate(slp, rho, 2, st, fac)
        iters += 2
    dt = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    return dict(value=iters * w.shape[0] / dt, unit="plan-iterations/s", cores=int(threads),
                kind="oracle",
                sample=f"{iters} FP64 reference-ADMM iterations x {w.shape[0]} plans of the "
                       f"same case ({dt:.1f} s; setup excluded)")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}))
        sys.exit(2)
    from synth import cases
    from paper_2509_08602_amd import ladmm

    cfg = args.config
    precision = args.precision or {0: "f64", 1: "f32", 2: "f32"}[cfg]
    case = cases.make_case(cfg)
    w = cases.config_weights(cfg)
    k = w.shape[0]
    rho0 = 1000.0
    ctx = ladmm.Context(0)
    dc = ladmm.Case.from_case(ctx, case, precision)
    setup_ms = dc.setup_ms
    fixed = ladmm.Options(max_iter=ITERS_PER_STEP, check_every=ITERS_PER_STEP, tol_gap=0.0,
                          rho0=rho0, w0_bot=cases.W0_BOT)
    b = ladmm.Batch(dc, w, opts=fixed)
    for _ in range(args.warmup):
        b.iterate(ITERS_PER_STEP)
    b.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.iterate(ITERS_PER_STEP)     # synchronous: returns after the check is read back
    wall = time.perf_counter() - t0
    ktimes = b.kernel_times()
    tiles = b.tiles()
    b.set_profiling(False)
    res = b.results(with_t=False)
    b.close()
    ms_per_step = wall * 1000.0 / args.steps
    value = k * ITERS_PER_STEP * args.steps / wall

    # roofline of the dominant kernel (by accumulated device time)
    N, n_t = case.n_points, case.n_t
    flops_gemm = 2.0 * N * n_t * k
    dom = max(("gemm1", "gemm2"), key=lambda c: ktimes[c][0])
    tot, cnt = ktimes[dom]
    avg_ms = tot / max(cnt, 1)
    achieved = flops_gemm / (avg_ms * 1e-3) / 1e12
    peak = PEAKS["f32_mfma_tflops"] if precision == "f32" else PEAKS["f64_mfma_tflops"]
    roofline = dict(bound="mfma", achieved=round(achieved, 3), peak=peak, unit="TFLOP/s",
                    frac=round(achieved / peak, 4), traffic=None, kernel=dom,
                    avg_launch_ms=round(avg_ms, 5),
                    algorithmic_flops_per_launch=flops_gemm)
    kernels = {c: dict(total_ms=round(v[0], 3), launches=v[1],
                       avg_ms=round(v[0] / v[1], 5) if v[1] else None)
               for c, v in ktimes.items()}

    sweep = None
    if not args.no_sweep:
        opts = ladmm.Options(max_iter=20000, check_every=50, tol_gap=1e-3, tol_pri=1e-3,
                             tol_dual=1e-3, rho0=rho0, w0_bot=cases.W0_BOT)
        t1 = time.perf_counter()
        out = ladmm.solve_batch(dc, w, opts=opts)
        sweep = dict(plans=k, seconds=round(time.perf_counter() - t1, 4), tol_gap=1e-3,
                     converged=int(np.sum(out["plan_status"] == ladmm.PLAN_CONVERGED)),
                     max_iters=int(out["iters"].max()), median_iters=float(np.median(out["iters"])),
                     max_rel_gap=float(out["rel_gap"].max()))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(case, w, rho0, args.cpu_seconds)

    line = {
        "metric": "plan-iterations/s",
        "value": round(value, 1),
        "unit": "plan-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": precision,
        "data": "synthetic",
        "config": {"workload": f"{case.name}: {N} dose points x {n_t} shot columns, "
                               f"{k} plans ({cases.CONFIG_PLANS[cfg]}x{cases.CONFIG_PLANS[cfg]} "
                               f"slider grid), {precision} dose block",
                   "points": N, "shots": n_t, "plans": k,
                   "iterations_per_step": ITERS_PER_STEP, "setup_ms": round(setup_ms, 2),
                   "tiles": {"gemm1": tiles[0], "gemm2": tiles[1]}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "sweep_1e-3": sweep,
        "last_check": {"max_rel_gap": float(np.max(res["rel_gap"])),
                       "max_r_pri": float(np.max(res["r_pri"]))},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
