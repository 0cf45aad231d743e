"""Benchmark: batched ADMM plan-iterations/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2]

Workload (default): the large case, nine targets, N = 200,000 dose points x
4,800 shot columns (200 isocentres x 8 sectors x 3 collimators), 441 plans from
a 21 x 21 slider grid, solved with the BF16 dose block and iterative
refinement (precision mode bf16: single BF16 products of the change since the
last refresh, a three-term pair refresh every check, FP32 iterates, FP64 Schur
complement inverse and small side).  The case is built and made resident in
HBM before timing (the setup time is reported beside the result).

A step is one pass of the whole iteration path over the 441-plan batch: 50
ADMM iterations (right-hand-side product, Schur solve, small-side update,
closed-form x-step with the fused z- and y-steps; the last one a refresh)
followed by one convergence check (the planning objective of the current shot
times, the duality gap, the certified lower bound and the primal/dual
residuals of every plan).  Plans are not frozen during the timed steps, so
every step does the same work.  value = plans x iterations / time.

Beside it: per-kernel device times from HIP events on the solver's stream over
the timed steps (the roofline entry uses the dominant dose-matrix product,
counting the method's own 2 N n_t k flops per product), the FP64 CPU oracle
timed on a bounded sample of the same workload, the wall time of the 441-plan
sweep solved until every plan's certified gap is <= 1e-3 (its objective
provably within 1e-3 of the exact optimum) with residuals <= 1e-4, both passes
of Sec. 2.C under the same rule, and the plain FP64 GPU ADMM on the same GPU
under the same rule.
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

PEAKS = {  # MI355X published dense peaks (TFLOP/s)
    "f64": 78.6,
    "f32": 157.3,
    "bf16x3": 2500.0,    # the BF16 matrix cores
    "bf16": 2500.0,
}
HBM_PEAK_GBS = 8000.0
# MFMA passes per dose-matrix product: the BF16-pair product executes three
TERMS = {"f64": 1, "f32": 1, "bf16x3": 3, "bf16": 1}
# bytes per dose-block entry read by one product in the hot iterations
DOSE_BYTES = {"f64": 8, "f32": 4, "bf16x3": 8, "bf16": 2}
DEFAULT_PRECISION = {0: "f64", 1: "f32", 2: "bf16"}
ITERS_PER_STEP = 50
RHO0 = 1e4      # step-size rule constant (Eq. rho_rule), from a grid over 30..1e4
COPY_PROBE_BYTES = 256 << 20
# HBM traffic per launch of the dose-matrix products, from rocprofv3 counter
# runs (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size); valid
# only while the kernels' sources are the ones that were measured.
# One record per product precision: the file and the sources its kernels come from.
TRAFFIC = {
    "f32": (os.path.join(ROOT, "profiles", "gemm_c1_f32_traffic.txt"),
            ("gemm_impl.h", "gemm_f32.hip", "kernels.h")),
    "bf16x3": (os.path.join(ROOT, "profiles", "gemm_c2_bf16_traffic.txt"),
               ("gemm_bf16.hip", "kernels.h")),
    "bf16": (os.path.join(ROOT, "profiles", "gemm_c2_bf16r_traffic.txt"),
             ("gemm_bf16.hip", "kernels.h")),
}


def copy_probe():
    """A plain device-to-device copy of COPY_PROBE_BYTES through the HIP
    runtime (executed as the runtime's copy kernel), three times: the reference
    that scales the HBM byte counters."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    src, dst = ctypes.c_void_p(), ctypes.c_void_p()
    for p in (src, dst):
        if hip.hipMalloc(ctypes.byref(p), ctypes.c_size_t(COPY_PROBE_BYTES)) != 0:
            raise RuntimeError("hipMalloc failed")
    try:
        if hip.hipMemset(src, 1, ctypes.c_size_t(COPY_PROBE_BYTES)) != 0:
            raise RuntimeError("hipMemset failed")
        for _ in range(3):
            for a, b in ((dst, src), (src, dst)):
                if hip.hipMemcpy(a, b, ctypes.c_size_t(COPY_PROBE_BYTES), 3) != 0:   # device to device
                    raise RuntimeError("hipMemcpy failed")
        hip.hipDeviceSynchronize()
    finally:
        hip.hipFree(src)
        hip.hipFree(dst)


def two_pass_sweep(ctx, case, w, precision, opts, max_vox=60000):
    """Both passes of Sec. 2.C for every plan: pass 1, the low-dose band of the
    pass-1 dose on candidate voxels (D_LD = D_T / 2, width D_T / 10), Algorithm 1
    (N_LD = 5,000 per plan, capped at the candidate count / 4) and pass 2 on the
    rebuilt case.  Candidates: an even subsample of the case's low-dose region."""
    from paper_2509_08602_amd import ladmm
    from synth import cases
    cand = case.ld_candidates
    if len(cand) == 0:
        return None
    cand = cand[np.linspace(0, len(cand) - 1, min(len(cand), max_vox)).astype(np.int64)]
    phi = case.kernel.dose_rate(cand)
    ld_group = [g.type for g in case.groups].index(cases.LD)
    n_ld = min(5000, len(cand) // 4)
    t0 = time.perf_counter()
    r1, r2, P, n2, tms = ladmm.two_pass(ctx, case, w, phi, 0.5 * case.prescription_mean,
                                        0.1 * case.prescription_mean, n_ld, 7, ld_group,
                                        precision=precision, opts=opts)
    wall = time.perf_counter() - t0
    return dict(seconds=round(wall, 4), candidates=int(len(cand)), selected_points=int(len(P)),
                pass2_points=int(n2), times_ms=dict(zip(("setup1", "pass1", "band_alg1", "setup2",
                                                         "pass2"), [round(x, 2) for x in tms])),
                pass2_converged=int(np.sum(r2["plan_status"] == ladmm.PLAN_CONVERGED)),
                pass2_max_iters=int(r2["iters"].max()))


def kernel_source_hash(precision):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC[precision][1]:
        h.update(open(os.path.join(ROOT, "paper_2509_08602_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, config_name, precision):
    """Bytes per launch recorded for `kernel` on this workload, or None."""
    if precision not in TRAFFIC or not os.path.exists(TRAFFIC[precision][0]):
        return None
    rec = {}
    for line in open(TRAFFIC[precision][0]):
        line = line.strip()
        if line.startswith("#") or "=" not in line:
            continue
        key, val = line.split("=", 1)
        rec[key.strip()] = val.strip()
    if rec.get("source_hash") != kernel_source_hash(precision) or rec.get("workload") != config_name:
        return None
    v = rec.get(f"{kernel}_bytes_per_launch")
    return float(v) if v else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--precision", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-f64-sweep", action="store_true",
                    help="skip the plain FP64 GPU ADMM sweep of the same case")
    ap.add_argument("--tol-cert", type=float, default=1e-3,
                    help="certified gap at which a sweep plan stops (with residuals <= 1e-4)")
    ap.add_argument("--workload", default="step", choices=("step", "uneven", "serve"),
                    help="step: iterations of one configuration (default); uneven: 32 cases "
                         "of uneven size served together; serve: Poisson request arrivals")
    ap.add_argument("--cases", type=int, default=None)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--alpha", type=float, default=1.0,
                    help="over-relaxation of the sweeps (1: the paper's ADMM)")
    ap.add_argument("--warm-store", type=int, default=256,
                    help="serving: solved plans kept per case for warm starts (0: cold starts)")
    ap.add_argument("--launch", default="graph", choices=("graph", "eager"),
                    help="timed region: replayed HIP graphs of each check chunk, or one-by-one launches")
    return ap.parse_args()


_T0 = time.perf_counter()
PHASES = {}


def log(msg):
    """Progress on stderr (a long run keeps printing while it works)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


class phase:
    """Times one phase of the benchmark into PHASES and logs its start and end."""

    def __init__(self, name):
        self.name = name

    def __enter__(self):
        log(self.name + " ...")
        self.t = time.perf_counter()

    def __exit__(self, *exc):
        PHASES[self.name] = round(time.perf_counter() - self.t, 2)
        log(f"{self.name}: {PHASES[self.name]} s")


def host_cpu():
    """Host cores and model of the machine running the oracle (nproc, lscpu)."""
    info = {"nproc": os.cpu_count()}
    try:
        info["nproc"] = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            key, _, val = line.partition(":")
            if key.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core",
                               "CPU(s)"):
                info[key.strip()] = val.strip()
    except Exception:
        pass
    return info


def cpu_baseline(case, w, rho0, budget_s, gpu_plan_iterations=None):
    """The FP64 oracle ADMM on the host cores, on a bounded sample of iterations
    of every plan (at least one after a warm-up iteration; setup excluded)."""
    from threadpoolctl import threadpool_info
    from oracle import lp as olp
    from oracle import admm as oadmm
    from synth import cases
    t_setup = time.perf_counter()
    lp = olp.assemble(case, w)
    slp = olp.precondition(lp, olp.bot_scale(case))
    del lp
    rho = olp.rho_rule(w[:, 3], rho0, cases.W0_BOT)
    log("oracle: LP assembled and preconditioned")
    fac, _ = oadmm.schur_factor(slp)
    log("oracle: Schur complement factored")
    st = oadmm.admm_iterate(slp, rho, 1, factor=fac)     # warm-up
    log("oracle: warm-up iteration done")
    setup_s = time.perf_counter() - t_setup
    iters = 0
    t0 = time.perf_counter()
    while iters == 0 or time.perf_counter() - t0 < budget_s:
        st = oadmm.admm_iterate(slp, rho, 1, st, fac)
        iters += 1
        log(f"oracle: {iters} timed iterations")
    dt = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    value = iters * w.shape[0] / dt
    out = dict(value=value, unit="plan-iterations/s", cores=int(threads), kind="oracle",
               sample=f"{iters} FP64 reference-ADMM iterations x {w.shape[0]} plans of the same "
                      f"case ({dt:.1f} s; setup {setup_s:.1f} s excluded)",
               host=host_cpu())
    if gpu_plan_iterations:
        out["sweep_seconds_extrapolated"] = round(gpu_plan_iterations / value, 1)
        out["sweep_note"] = ("the GPU sweep's plan-iterations at this oracle rate: extrapolated, "
                             "not run")
    return out


def uneven(args):
    """32 seeded cases between the small and the large configuration, 81 plans
    each, FP32, all resident and served together (one lane per case, each on
    its own stream): aggregate plan-iterations/s over a fixed iteration budget."""
    from synth import cases
    from paper_2509_08602_amd import ladmm
    n_cases = args.cases or 32
    iters = ITERS_PER_STEP * max(1, args.steps // 4)
    ctx = ladmm.Context(0)
    dcs, sizes, setup = [], [], 0.0
    for s in range(1000, 1000 + n_cases):
        c = cases.uneven_case(s)
        dc = ladmm.Case.from_case(ctx, c, "f32")
        setup += dc.setup_ms
        dcs.append(dc)
        sizes.append((c.n_points, c.n_t))
        del c
    w = cases.config_weights(1)
    fixed = lambda n: ladmm.Options(max_iter=n, check_every=ITERS_PER_STEP, tol_gap=0.0,
                                    rho0=RHO0, w0_bot=cases.W0_BOT)

    def run(eager):
        srv = ladmm.Server(ctx, slots=96, check_every=ITERS_PER_STEP, autotune=True, eager=eager)
        for t in [srv.submit(dc, w, opts=fixed(ITERS_PER_STEP)) for dc in dcs]:   # lanes + tiles
            t.wait()
        t0 = time.perf_counter()
        ts = [srv.submit(dc, w, opts=fixed(iters)) for dc in dcs]
        for t in ts:
            t.wait()
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return wall, st

    k = w.shape[0]
    wall, st = run(args.launch == "eager")
    other_wall, _ = run(args.launch != "eager")
    value = n_cases * k * iters / wall
    other = n_cases * k * iters / other_wall
    launch = dict(mode=args.launch, plan_iterations_per_s={
        args.launch: round(value, 1), ("eager" if args.launch == "graph" else "graph"): round(other, 1)})
    flops = sum(4.0 * N * nt * k for N, nt in sizes) * iters
    print(json.dumps({
        "metric": "plan-iterations/s", "value": round(value, 1), "unit": "plan-iterations/s",
        "n_gpus": 1, "steps": iters // ITERS_PER_STEP, "warmup": 1,
        "ms_per_step": round(wall * 1000 * ITERS_PER_STEP / iters, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{n_cases} uneven cases (N {min(s[0] for s in sizes)}-"
                               f"{max(s[0] for s in sizes)}, n_t {min(s[1] for s in sizes)}-"
                               f"{max(s[1] for s in sizes)}), {k} plans each, f32, served "
                               f"together", "cases": n_cases, "plans_per_case": k,
                   "iterations": iters, "setup_ms_total": round(setup, 1)},
        "launch": launch,
        "dose_product_tflops": round(flops / wall / 1e12, 2),
        "lanes": st["lanes"], "hbm_gb": round(ctx.used_bytes / 1e9, 2)}))


def serve(args):
    """Serving: resident cases of uneven size, Poisson arrivals of requests of
    1, 9, 81 or 441 plans (probabilities 0.5 / 0.3 / 0.15 / 0.05) on a random
    case, solved to a 1e-3 gap.  Capacity is measured closed-loop first; then
    arrivals at 0.5, 0.8 and 0.95 of it; p50 / p99 latency per level."""
    from synth import cases
    from paper_2509_08602_amd import ladmm
    n_cases = args.cases or 16
    ctx = ladmm.Context(0)
    dcs = []
    for s in range(1000, 1000 + n_cases):
        c = cases.uneven_case(s)
        dcs.append(ladmm.Case.from_case(ctx, c, "f32"))
        del c
    rng = np.random.default_rng(2000)
    grids = {9: cases.config_weights(0), 81: cases.config_weights(1),
             441: cases.config_weights(2)}

    def draw():
        size = int(rng.choice([1, 9, 81, 441], p=[0.5, 0.3, 0.15, 0.05]))
        w = (cases.slider_weights(rng.uniform(size=1), rng.uniform(size=1)) if size == 1
             else grids[size])
        return int(rng.integers(n_cases)), w

    opts = ladmm.Options(max_iter=3000, check_every=ITERS_PER_STEP, tol_gap=1e-3, tol_pri=1e-3,
                         tol_dual=1e-3, rho0=RHO0, w0_bot=cases.W0_BOT, adapt_rho=True)
    # warm-up: one lane per case (tile choice included)
    srv = ladmm.Server(ctx, slots=96, check_every=ITERS_PER_STEP, autotune=True)
    for t in [srv.submit(dc, grids[9][:1], opts=opts) for dc in dcs]:
        t.wait()
    srv.close()

    reqs = [draw() for _ in range(args.requests)]   # the same sequence at every level

    warm = args.warm_store

    def run(load_rps, n):
        arr = np.random.default_rng(2001)
        gaps = arr.exponential(1.0 / load_rps, size=n) if load_rps else np.zeros(n)
        s = ladmm.Server(ctx, slots=96, check_every=ITERS_PER_STEP, autotune=True, warm_store=warm)
        if warm:
            # solved weightings already in the store: the 3x3 slider grid of every case
            for t in [s.submit(dc, grids[9], opts=opts) for dc in dcs]:
                t.wait()
        s.reset_stats()
        t0 = time.perf_counter()
        due, ts = t0, []
        for (ci, w), g in zip(reqs, gaps):
            due += g
            delay = due - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            ts.append(s.submit(dcs[ci], w, opts=opts))
        for t in ts:
            t.wait()
        wall = time.perf_counter() - t0
        st = s.stats()
        s.close()
        plans = sum(w.shape[0] for _, w in reqs)
        return dict(requests=n, plans=plans, seconds=round(wall, 3), p50_ms=round(st["p50_ms"], 2),
                    p99_ms=round(st["p99_ms"], 2), max_ms=round(st["max_ms"], 2),
                    plan_iterations_per_s=round(st["plan_iterations"] / wall, 1),
                    completed=st["completed"], warm_starts=st["warm_starts"])

    cal = run(0.0, args.requests)
    capacity = cal["requests"] / cal["seconds"]
    levels = []
    for load in (0.5, 0.8, 0.95):
        r = run(load * capacity, args.requests)
        r.update(load=load, offered_rps=round(load * capacity, 4))
        levels.append(r)
    mid = levels[1]
    print(json.dumps({
        "metric": "p99 latency at 0.8 of capacity", "value": mid["p99_ms"], "unit": "ms",
        "n_gpus": 1, "steps": args.requests, "warmup": 1, "ms_per_step": mid["p50_ms"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"serving: {n_cases} resident uneven cases, Poisson arrivals of "
                               "1/9/81/441-plan requests (p 0.5/0.3/0.15/0.05), 1e-3 gap, " +
                               (f"warm start from the nearest solved weighting (store of {warm} "
                                "plans per case, seeded with the 3x3 slider grid)" if warm else
                                "cold start"), "cases": n_cases, "requests_per_level": args.requests,
                   "warm_store": warm},
        "capacity_rps": round(capacity, 4), "closed_loop": cal, "levels": levels,
        "hbm_gb": round(ctx.used_bytes / 1e9, 2)}))


def product_bytes(kernel, precision, N, n_t, k, kp):
    """Algorithmic HBM bytes of one launch of a hot dose-matrix product: the
    dose block once at its storage width, the plan-side operand, and the
    result (GEMM1: the n_t x k right-hand side once; GEMM2: the epilogue's
    iterate traffic), per padded plan column as the kernels move them."""
    s_it = 8 if precision == "f64" else 4
    dose = DOSE_BYTES[precision] * N * n_t
    if precision == "bf16":
        operand = 2 * N * kp if kernel == "gemm1" else 2 * n_t * kp
        # q read + written, X_ref and W_ref read, dW written
        epi = (4 * 4 + 2) * N * kp if kernel == "gemm2" else 4 * n_t * kp
    elif precision == "bf16x3":
        operand = 4 * N * kp if kernel == "gemm1" else 4 * n_t * kp
        epi = (2 * 4 + 4) * N * kp if kernel == "gemm2" else 4 * n_t * kp
    else:
        operand = s_it * (N if kernel == "gemm1" else n_t) * kp
        epi = 3 * s_it * N * kp if kernel == "gemm2" else s_it * n_t * kp
    return float(dose + operand + epi)


def sweep(dc, w, opts, label):
    from paper_2509_08602_amd import ladmm
    t1 = time.perf_counter()
    b = ladmm.Batch(dc, w, opts=opts)
    b.run(progress=lambda running: log(f"{label}: {running} plans still running"))
    out = b.results()
    b.close()
    sec = time.perf_counter() - t1
    conv = out["plan_status"] == ladmm.PLAN_CONVERGED
    return dict(label=label, plans=int(w.shape[0]), seconds=round(sec, 4),
                converged=int(conv.sum()), max_iters=int(out["iters"].max()),
                median_iters=float(np.median(out["iters"])),
                plan_iterations=int(out["iters"].sum()),
                max_cert_gap=float(np.nanmax(out["cert_gap"])),
                max_rel_gap=float(out["rel_gap"].max()), max_r_pri=float(out["r_pri"].max()),
                max_r_dual=float(out["r_dual"].max()))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; use --gpus 1"}))
        sys.exit(2)
    if args.workload == "uneven":
        return uneven(args)
    if args.workload == "serve":
        return serve(args)
    from synth import cases
    from paper_2509_08602_amd import ladmm

    cfg = args.config
    precision = args.precision or DEFAULT_PRECISION[cfg]
    with phase("case build"):
        case = cases.make_case(cfg)
    case_s = PHASES["case build"]
    w = cases.config_weights(cfg)
    k = w.shape[0]
    rho0 = RHO0
    ctx = ladmm.Context(0)
    with phase("case setup on the device"):
        dc = ladmm.Case.from_case(ctx, case, precision)
    setup_ms = dc.setup_ms
    fixed = ladmm.Options(max_iter=ITERS_PER_STEP, check_every=ITERS_PER_STEP, tol_gap=0.0,
                          rho0=rho0, w0_bot=cases.W0_BOT)
    b = ladmm.Batch(dc, w, opts=fixed)

    def timed(steps):
        t0 = time.perf_counter()
        for _ in range(steps):
            b.iterate(ITERS_PER_STEP)     # synchronous: returns after the check is read back
        return time.perf_counter() - t0

    # timed region: each step replays the captured graph of one check chunk
    b.set_graphs(args.launch == "graph")
    with phase("warm-up steps"):
        for _ in range(args.warmup):
            b.iterate(ITERS_PER_STEP)
    with phase("timed steps"):
        wall = timed(args.steps)
    # kernel durations: HIP events around every launch on the batch's stream
    # (this launches kernel by kernel), the same number of steps right after
    b.set_profiling(True)
    with phase("steps with kernel events"):
        wall_prof = timed(args.steps)
    ktimes = b.kernel_times()
    b.set_profiling(False)
    # one-by-one launches without events, for the launch-mode comparison
    b.set_graphs(False)
    with phase("steps launched one by one"):
        wall_eager = timed(args.steps)
    tiles = b.tiles()
    res = b.results(with_t=False)
    kp = -(-k // 32) * 32
    b.close()
    ms_per_step = wall * 1000.0 / args.steps
    value = k * ITERS_PER_STEP * args.steps / wall
    launch_modes = {"graph" if args.launch == "graph" else "eager_timed": round(value, 1),
                    "eager": round(k * ITERS_PER_STEP * args.steps / wall_eager, 1),
                    "eager_with_kernel_events": round(k * ITERS_PER_STEP * args.steps / wall_prof, 1)}

    # roofline of the dominant hot dose-matrix product (by accumulated device
    # time): the method's own flops, 2 N n_t k per product for the k plans, and
    # its algorithmic bytes; the bound is the resource its algorithmic work
    # needs more time on at peak
    N, n_t = case.n_points, case.n_t
    flops_gemm = 2.0 * N * n_t * k
    dom = max(("gemm1", "gemm2"), key=lambda c: ktimes[c][0])
    tot, cnt = ktimes[dom]
    avg_ms = tot / max(cnt, 1)
    peak = PEAKS[precision]
    rows = {}
    for kern in ("gemm1", "gemm2"):
        kt, kc = ktimes[kern]
        if not kc:
            continue
        a_ms = kt / kc
        byt = product_bytes(kern, precision, N, n_t, k, kp)
        rows[kern] = dict(avg_launch_ms=round(a_ms, 5), tflops=round(flops_gemm / (a_ms * 1e-3) / 1e12, 2),
                          mfma_frac=round(flops_gemm / (a_ms * 1e-3) / 1e12 / peak, 4),
                          algorithmic_bytes=byt,
                          hbm_gbs=round(byt / (a_ms * 1e-3) / 1e9, 1),
                          hbm_frac=round(byt / (a_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    r = rows[dom]
    t_mfma = flops_gemm / (peak * 1e12)
    t_hbm = r["algorithmic_bytes"] / (HBM_PEAK_GBS * 1e9)
    traffic = measured_traffic(dom, case.name, precision)
    if t_mfma >= t_hbm:
        roofline = dict(bound="mfma", achieved=r["tflops"], peak=peak, unit="TFLOP/s",
                        frac=r["mfma_frac"])
    else:
        roofline = dict(bound="hbm", achieved=r["hbm_gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=r["hbm_frac"])
    roofline.update(traffic=traffic, kernel=dom, avg_launch_ms=round(avg_ms, 5),
                    algorithmic_flops_per_launch=flops_gemm,
                    algorithmic_bytes_per_launch=r["algorithmic_bytes"],
                    mfma_frac=r["mfma_frac"], hbm_frac=r["hbm_frac"],
                    mfma_passes=TERMS[precision], products=rows)
    kernels = {c: dict(total_ms=round(v[0], 3), launches=v[1],
                       avg_ms=round(v[0] / v[1], 5) if v[1] else None)
               for c, v in ktimes.items()}

    sweeps = None
    gpu_plan_iterations = None
    if not args.no_sweep:
        # every plan to a certified gap <= tol_cert (objective provably within
        # tol_cert of F*) with plain gap <= tol_cert and residuals <= 1e-4
        opts = ladmm.Options(max_iter=20000, check_every=50, tol_gap=args.tol_cert, tol_pri=1e-4,
                             tol_dual=1e-4, tol_cert=args.tol_cert, rho0=rho0,
                             w0_bot=cases.W0_BOT, alpha=args.alpha)
        with phase("sweep, pass 1"):
            sweeps = {"pass1": sweep(dc, w, opts, f"{precision}, pass 1")}
        gpu_plan_iterations = sweeps["pass1"]["plan_iterations"]
        sweeps["pass1"]["paper_budget_2x3000_seconds"] = round(2 * 3000 * k / value, 2)
        with phase("sweep, both passes"):
            two = two_pass_sweep(ctx, case, w, precision, opts)
        if two:
            sweeps["two_pass"] = two
        if not args.no_f64_sweep and precision != "f64":
            dc.close()
            with phase("FP64 case setup"):
                d64 = ladmm.Case.from_case(ctx, case, "f64")
            with phase("sweep, plain FP64 GPU ADMM"):
                sweeps["f64_pass1"] = sweep(d64, w, opts, "plain FP64 GPU ADMM, pass 1")
            sweeps["f64_pass1"]["speedup_of_" + precision] = round(
                sweeps["f64_pass1"]["seconds"] / sweeps["pass1"]["seconds"], 2)
            d64.close()

    if args.copy_probe:
        copy_probe()

    cpu = None
    if not args.no_cpu_baseline:
        with phase("CPU oracle baseline"):
            cpu = cpu_baseline(case, w, rho0, args.cpu_seconds, gpu_plan_iterations)

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
                   "case_build_s": round(case_s, 1),
                   "tiles": {"gemm1": tiles[0], "gemm2": tiles[1]}},
        "launch": dict(mode=args.launch, plan_iterations_per_s=launch_modes),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "sweeps": sweeps,
        "last_check": {"max_rel_gap": float(np.max(res["rel_gap"])),
                       "max_r_pri": float(np.max(res["r_pri"]))},
        "phase_seconds": PHASES,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
