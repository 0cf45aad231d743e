"""The library's own HIP sources, run on the CPU through a host emulation.

The kernels and the C ABI of libladmm are compiled for the host with the HIP
shim in tests/hostemu (one fiber per GPU thread, exact workgroup barriers,
emulated wavefront shuffles and MFMA) and AddressSanitizer.  A driver calls the
C ABI on small synthetic cases; the test checks that no access leaves its
buffer (ASan aborts the driver otherwise) and that the results match the FP64
oracle like the GPU parity tests.  This catches indexing and launch-shape
errors before any kernel reaches a GPU.  Not a product path: the product
library is only ever built by hipcc for gfx950.
"""
import concurrent.futures
import os
import shutil
import subprocess

import numpy as np
import pytest

from synth import cases
from oracle import lp as olp
from oracle import admm as oadmm
from oracle import alg1 as oalg1
from oracle import dose as odose

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "hostemu")
CSRC = os.path.join(ROOT, "paper_2509_08602_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "hostemu")


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.fixture(scope="module")
def driver():
    cxx = _clang()
    if cxx is None:
        pytest.skip("clang++ not available")
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "driver")
    srcs = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith((".hip", ".cpp"))]
    srcs += [os.path.join(EMU, "hostemu.cpp"), os.path.join(EMU, "driver.cpp")]
    flags = ["-std=c++17", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
             "-Wno-unused-result", "-Wno-unused-value", "-I", EMU, "-I", os.path.join(ROOT, "include"),
             "-I", CSRC]
    objs = []

    def compile_one(src):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        r = subprocess.run([cxx, *flags, "-c", "-x", "c++", src, "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=6) as ex:
        objs = list(ex.map(compile_one, srcs))
    res = subprocess.run([cxx, "-fsanitize=address", *objs, "-o", exe], capture_output=True,
                         text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    return exe


PRECISION = {"f64": 0, "f32": 1, "bf16x3": 2, "bf16": 3}


def write_inputs(d, case, w, precision, iters, mask=None, vols=None, n_ld=None, seed=0,
                 vox=None, d_ld=0.0, delta=1.0, solve_iters=0, rho0=1000.0, tiles=(-1, -1),
                 two_pass=False, serve=False, compact_iters=0):
    os.makedirs(d, exist_ok=True)
    k = w.shape[0]
    n_vols = 0 if vols is None else vols.shape[0]
    n_vox = 0 if vols is None else vols.shape[1]
    band = 0 if vox is None else vox.shape[0]
    with open(os.path.join(d, "meta.txt"), "w") as f:
        f.write(f"{case.n_points} {case.n_iso} {case.n_sectors} {case.n_collimators} "
                f"{len(case.groups)} {PRECISION[precision]} {k} {iters} {rho0!r} "
                f"{cases.W0_BOT!r} {case.prescription_mean!r} {case.phi_cal!r} "
                f"{0 if mask is None else 1} {n_vols} {n_vox} {seed} {band} {d_ld!r} {delta!r} "
                f"{solve_iters} {tiles[0]} {tiles[1]} {int(two_pass)} {int(serve)} {compact_iters}\n")
    np.ascontiguousarray(case.dose, np.float64).tofile(os.path.join(d, "dose.f64"))
    np.ascontiguousarray(case.group, np.int32).tofile(os.path.join(d, "group.i32"))
    with open(os.path.join(d, "groups.txt"), "w") as f:
        for g in case.groups:
            f.write(f"{g.type} {g.structure} {g.threshold!r} {g.share!r}\n")
    np.ascontiguousarray(w, np.float64).tofile(os.path.join(d, "weights.f64"))
    if mask is not None:
        cases.pack_bits(mask).tofile(os.path.join(d, "mask.u64"))
    if vols is not None:
        cases.pack_bits(vols).tofile(os.path.join(d, "vols.u64"))
        np.ascontiguousarray(n_ld, np.int32).tofile(os.path.join(d, "nld.i32"))
    if vox is not None:
        np.ascontiguousarray(vox, np.float64).tofile(os.path.join(d, "vox.f64"))


def rd(d, name, shape, dtype=np.float64):
    return np.fromfile(os.path.join(d, name), dtype).reshape(shape)


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref))) / max(float(np.max(np.abs(ref))), 1e-300)


def small_case(seed=0, oar=False):
    spec = cases.mini_spec(n_iso=2, sectors=8, collimators=3, radius=3.0, n_ring=90, n_ld=60,
                           oar=oar)
    return cases.build_case(spec, seed)


# Every emulated run is prepared and started at once (the runs are independent
# single-threaded processes), then each test checks its own run's outputs.
ITER_CASES = [("f64", 1e-11, (0, 0), 0, 5),
              ("f32", 2e-3, (-1, -1), 12, 5),
              ("bf16x3", 2e-4, (-1, -1), 0, 5),
              ("bf16x3", 2e-4, (4, 4), 0, 70),
              # single BF16 products of the change since the last refresh: from
              # zero iterates the first changes are the full values, so the
              # iterates carry BF16 rounding (2^-9 relative per operand) until
              # the refresh that ends the chunk
              ("bf16", 3e-2, (-1, -1), 12, 5),
              # the single-operand tiles of the ring-pipelined kernel: 64, 112
              # and 96 plan columns per workgroup, and 448 (waves split rows
              # and columns)
              ("bf16", 3e-2, (6, 6), 0, 448),
              ("bf16", 3e-2, (7, 7), 0, 448),
              ("bf16", 3e-2, (8, 8), 0, 96),
              ("bf16", 3e-2, (9, 9), 0, 448)]


# compaction runs: enough plans for the launched width to shrink (FP32 in
# 32-column steps, BF16 in widths that admit a 64-, 96- or 224-column tile)
COMPACT_CASES = [("f32", 70), ("bf16", 120)]


def _iter_name(precision, tiles, k):
    return f"iter-{precision}-{tiles[0]}{tiles[1]}-{k}"


def _iter_spec(k, wide=False):
    """wide: 8 isocentres (192 shot columns, 512 padded points), so that the
    single-operand tiles of 192 shot rows and 128 point rows apply."""
    if wide:
        spec = cases.mini_spec(n_iso=8, sectors=8, collimators=3, radius=3.0, n_ring=90, n_ld=60)
        return cases.build_case(spec, 1), cases.random_weights(k, 2)
    return small_case(1), cases.random_weights(k, 2)


def _wide(tiles):
    return tiles[0] >= 6


def _mask_spec():
    case = small_case(3, oar=True)
    w = cases.random_weights(4, 5)
    types = case.point_types()
    rng = np.random.default_rng(1)
    mask = np.zeros((4, case.n_points), bool)
    ld = np.nonzero(types == cases.LD)[0]
    for j in range(4):
        mask[j, ld[rng.random(ld.size) < 0.6]] = True
    vols = cases.random_volumes(6, 700, 4)
    n_ld = np.array([50, 0, 120, 33, 500, 80])
    vox = case.kernel.dose_rate(case.ld_candidates[:333])
    return dict(case=case, w=w, mask=mask, vols=vols, n_ld=n_ld, vox=vox)


def _tp_spec(levels=None):
    if levels is None:
        case = small_case(5)
    else:
        spec = cases.mini_spec(n_iso=2, sectors=8, collimators=3, radius=3.0, n_ring=90, n_ld=60)
        case = cases.build_case(dict(spec, ld_levels=levels), 5)
    w = cases.random_weights(2, 8)
    cand = case.ld_candidates[::7][:200]
    return dict(case=case, w=w, cand=cand, vox=case.kernel.dose_rate(cand))


def _serve_spec():
    case = small_case(7)
    k = 36
    w = cases.random_weights(k, 9)
    types = case.point_types()
    rng = np.random.default_rng(4)
    mask = np.zeros((k, case.n_points), bool)
    ld = np.nonzero(types == cases.LD)[0]
    for j in range(k):
        mask[j, ld[rng.random(ld.size) < 0.5]] = True
    return dict(case=case, w=w, mask=mask)


def _prepare(root):
    runs = {}
    for precision, _, tiles, solve, k in ITER_CASES:
        d = os.path.join(root, _iter_name(precision, tiles, k))
        case, w = _iter_spec(k, _wide(tiles))
        write_inputs(d, case, w, precision, 4, solve_iters=solve, tiles=tiles)
        runs[_iter_name(precision, tiles, k)] = d
    m = _mask_spec()
    d = os.path.join(root, "mask")
    write_inputs(d, m["case"], m["w"], "f64", 3, mask=m["mask"], vols=m["vols"], n_ld=m["n_ld"],
                 seed=77, vox=m["vox"], d_ld=0.05, delta=0.1, tiles=(2, 1))
    runs["mask"] = d
    t = _tp_spec()
    d = os.path.join(root, "tp")
    write_inputs(d, t["case"], t["w"], "f64", 2, seed=41, vox=t["vox"], d_ld=0.05, delta=0.1,
                 tiles=(1, 3), two_pass=True)
    runs["tp"] = d
    t = _tp_spec([0.5, 0.3])
    d = os.path.join(root, "tp2")
    write_inputs(d, t["case"], t["w"], "f64", 2, seed=41, vox=t["vox"], d_ld=0.05, delta=0.1,
                 tiles=(1, 3), two_pass=True)
    runs["tp2"] = d
    t = _tp_spec()
    d = os.path.join(root, "tp3")
    write_inputs(d, t["case"], t["w"], "f64", 2, seed=41, vox=t["vox"], d_ld=0.05, delta=0.1,
                 tiles=(1, 3), two_pass=3)
    runs["tp3"] = d
    v = _serve_spec()
    d = os.path.join(root, "serve")
    write_inputs(d, v["case"], v["w"], "f32", 1, mask=v["mask"], tiles=(0, 0), serve=True)
    runs["serve"] = d
    d = os.path.join(root, "serve-bf16")
    write_inputs(d, v["case"], v["w"], "bf16", 1, mask=v["mask"], tiles=(0, 0), serve=True)
    runs["serve-bf16"] = d
    for precision in ("bf16", "bf16x3"):
        case, w = _iter_spec(5)
        d = os.path.join(root, "refresh-" + precision)
        write_inputs(d, case, w, precision, 1, tiles=(0, 0))
        runs["refresh-" + precision] = d
    for precision, k in COMPACT_CASES:
        case, w = _iter_spec(k, precision == "bf16")
        d = os.path.join(root, f"compact-{precision}")
        write_inputs(d, case, w, precision, 1, tiles=(0, 0), compact_iters=12)
        runs[f"compact-{precision}"] = d
    return runs


@pytest.fixture(scope="module")
def emu(driver, tmp_path_factory):
    runs = _prepare(str(tmp_path_factory.mktemp("emu")))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")

    def go(d):
        return subprocess.run([driver, d], capture_output=True, text=True, env=env, timeout=900)

    with concurrent.futures.ThreadPoolExecutor(max_workers=max(1, min(len(runs), os.cpu_count() or 4))) as ex:
        futs = {name: ex.submit(go, d) for name, d in runs.items()}
        return {name: (runs[name], f.result()) for name, f in futs.items()}


def finished(emu, name):
    d, res = emu[name]
    assert res.returncode == 0, (res.stdout + res.stderr)[-6000:]
    return d


@pytest.mark.parametrize("precision,tol,tiles,solve,k", ITER_CASES)
def test_emulated_iterations_match_oracle(emu, precision, tol, tiles, solve, k):
    """tiles (-1, -1): the autotuner launches every tile configuration; (4, 4)
    at 70 plans (96 columns): the direct-A BF16-pair kernels of both products.  The
    BF16-pair products carry about 2^-16 relative error per product, of the
    order of the FP32 path's, hence the same kind of tolerance."""
    d = finished(emu, _iter_name(precision, tiles, k))
    case, w = _iter_spec(k, _wide(tiles))
    if tiles[0] >= 0:   # the pinned configurations are the ones that ran
        assert np.fromfile(os.path.join(d, "tiles.i32"), np.int32).tolist() == list(tiles)
    iters = 4
    lp = olp.assemble(case, w)
    slp = olp.precondition(lp, olp.bot_scale(case))
    m, n = slp.A.shape
    S_ref = slp.A @ slp.A.T + np.eye(m)
    assert rel_err(rd(d, "S.f64", (m, m)), S_ref) < 1e-13
    assert rel_err(rd(d, "Sinv.f64", (m, m)), np.linalg.inv(S_ref)) < 1e-10
    assert rel_err(rd(d, "E.f64", (m,)), slp.E) < 1e-13
    rho = olp.rho_rule(w[:, 3], 1000.0, cases.W0_BOT)
    st = oadmm.admm_iterate(slp, rho, iters)
    k = w.shape[0]
    for name, ref in (("z1", st.z1), ("y1", st.y1), ("z2", st.z2), ("y2", st.y2)):
        got = rd(d, name + ".f64", ref.shape)
        print(precision, name, rel_err(got, ref))
        assert rel_err(got, ref) < tol, (name, rel_err(got, ref))
    if precision == "bf16":
        # the state re-imported and one iteration: a chunk of one iteration is a
        # refresh (pair products), so it follows the oracle's step from the
        # exported state to the pair products' accuracy
        got = oadmm.ADMMState(*(rd(d, nm + ".f64", ref.shape) for nm, ref in
                                (("z1", st.z1), ("y1", st.y1), ("z2", st.z2), ("y2", st.y2))))
        st2 = oadmm.admm_iterate(slp, rho, 1, got)
        assert rel_err(rd(d, "z1b.f64", st2.z1.shape), st2.z1) < 2e-4
    else:
        st2 = oadmm.admm_iterate(slp, rho, 1, st)
        assert rel_err(rd(d, "z1b.f64", st2.z1.shape), st2.z1) < tol
    t = rd(d, "t.f64", (k, lp.n_t))
    F = olp.planning_objective(case, w, t.T)[0]
    res = rd(d, "res.f64", (7, k))
    assert rel_err(res[0], F) < (1e-10 if precision == "f64" else 1e-5 if precision == "f32" else 2e-4)
    # the device's certified bounds are the oracle's for the same iterate (the
    # oracle's dual point from the exported z1, the same global BOT repair)
    cert = olp.certify(case, w, t.T, rd(d, "z1.f64", st.z1.shape)[:case.n_points], lp=lp)
    tol_c = 1e-10 if precision == "f64" else 1e-5 if precision == "f32" else 2e-4
    assert rel_err(res[5], cert["L"]) < tol_c, (res[5], cert["L"])
    assert np.max(np.abs(res[6] - cert["cert_gap"])) < 10 * tol_c, (res[6], cert["cert_gap"])


def test_emulated_refresh_chunks_equal_pair_products(emu):
    """LADMM_BF16 with every chunk one iteration long runs only refresh
    iterations, whose products are the three-term pair products of
    LADMM_BF16X3: the two modes give the same bits."""
    a = finished(emu, "refresh-bf16")
    b = finished(emu, "refresh-bf16x3")
    case, w = _iter_spec(5)
    n_A = case.n_points + case.n_iso * case.n_sectors
    for name in ("z1", "y1", "z1b"):
        x = rd(a, name + ".f64", (n_A, 5))
        y = rd(b, name + ".f64", (n_A, 5))
        assert np.array_equal(x, y), name


def test_emulated_ld_mask_oar_band_and_alg1(emu):
    d = finished(emu, "mask")
    m = _mask_spec()
    case, w, mask, vols, n_ld, vox = m["case"], m["w"], m["mask"], m["vols"], m["n_ld"], m["vox"]
    lp = olp.assemble(case, w, mask)
    slp = olp.precondition(lp, olp.bot_scale(case))
    rho = olp.rho_rule(w[:, 3], 1000.0, cases.W0_BOT)
    st = oadmm.admm_iterate(slp, rho, 3)
    assert rel_err(rd(d, "z1.f64", st.z1.shape), st.z1) < 1e-11
    assert rel_err(rd(d, "y2.f64", st.y2.shape), st.y2) < 1e-11
    # Algorithm 1, bit-exact
    Pref, pref = oalg1.select_ld_points(vols, n_ld, 77)
    P = np.fromfile(os.path.join(d, "P.i64"), np.int64)
    assert P.tolist() == Pref
    W = (700 + 63) // 64
    masks = rd(d, "masks.u64", (6, W), np.uint64)
    assert np.array_equal(cases.unpack_bits(masks, len(Pref)), oalg1.masks_over(Pref, pref))
    # the allocation-free entry point: the same bits, then a smaller second call
    for rep, kk in ((0, 6), (1, 3)):
        Pk, pk = (Pref, pref) if kk == 6 else oalg1.select_ld_points(vols[:kk], n_ld[:kk], 77)
        Ps = np.fromfile(os.path.join(d, f"P_static{rep}.i64"), np.int64)
        assert Ps.tolist() == Pk
        ms = rd(d, f"masks_static{rep}.u64", (kk, W), np.uint64)
        assert np.array_equal(cases.unpack_bits(ms, len(Pk)), oalg1.masks_over(Pk, pk))
    # low-dose band of the current shot times
    t = rd(d, "t.f64", (4, lp.n_t))
    band = cases.unpack_bits(rd(d, "band.u64", (4, (333 + 63) // 64), np.uint64), 333)
    ref = odose.ld_band(odose.dose(vox, t.T), 0.05, 0.1)
    assert np.array_equal(band, ref)


@pytest.mark.parametrize("run,levels,passes", [("tp", None, 2), ("tp2", [0.5, 0.3], 2),
                                               ("tp3", None, 3)])
def test_emulated_two_pass(emu, run, levels, passes):
    """Both passes through ladmm_two_pass (one low-dose group),
    ladmm_two_pass_sets (two low-dose groups with thresholds d and d / 2, App.
    A) and three passes through ladmm_passes: every set's last-pass point set
    equals the oracle's band + Algorithm 1 from the previous pass's shot times,
    and the last pass's objective is the oracle's F of the returned shot times
    on the rebuilt case."""
    d = finished(emu, run)
    t = _tp_spec(levels)
    case, w, cand, vox = t["case"], t["w"], t["cand"], t["vox"]
    k, n_t = w.shape[0], case.n_t
    ld_groups = [g for g, grp in enumerate(case.groups) if grp.type == cases.LD]
    counts = np.fromfile(os.path.join(d, "tp_n.i64"), np.int64)
    assert len(counts) == len(ld_groups) + 1
    P_all = np.fromfile(os.path.join(d, "tp_P.i64"), np.int64)
    t_prev = rd(d, "tp_t1.f64" if passes == 2 else f"tp_tmid{passes - 1}.f64", (k, n_t))
    dose1 = odose.dose(vox, t_prev.T)
    keep = np.nonzero(~np.isin(case.group, ld_groups))[0]
    extra, blocks, at = [], [], 0
    for i, g in enumerate(ld_groups):
        vols = odose.ld_band(dose1, 0.05 / (i + 1), 0.1)
        Pref, pref = oalg1.select_ld_points(vols, np.full(k, 25), 42 + i)
        assert P_all[at:at + counts[i]].tolist() == Pref, i
        at += int(counts[i])
        extra.append((cand[np.array(Pref, dtype=np.int64)], g))
        blocks.append(oalg1.masks_over(Pref, pref) if len(Pref) else np.zeros((k, 0), bool))
    case2 = case.with_points(keep, extra=extra)
    assert case2.n_points == counts[-1]
    mask2 = np.concatenate([np.zeros((k, len(keep)), bool)] + blocks, axis=1)
    t2 = rd(d, "tp_t2.f64", (k, n_t))
    F2 = olp.planning_objective(case2, w, t2.T, mask2)[0]
    assert rel_err(rd(d, "tp_f2.f64", (k,)), F2) < 1e-10


@pytest.mark.parametrize("run", ["serve", "serve-bf16"])
def test_emulated_serving(emu, run):
    """Continuous batching through ladmm_submit/wait/cancel: a cancelled request,
    then two requests whose plans share 32 slots (later plans start in slots
    freed by earlier ones).  Every plan's shot times, objective and iteration
    count equal those of ladmm_solve_batch on its own request, bitwise, and the
    objective is the oracle's F of the returned shot times."""
    d = finished(emu, run)
    v = _serve_spec()
    case, w, mask = v["case"], v["w"], v["mask"]
    k = w.shape[0]
    n_t = case.n_t
    for tag, sl, iters in (("A", slice(0, k - 6), 4), ("B", slice(k - 6, k), 2)):
        kk = sl.stop - sl.start
        t = rd(d, f"serve_t{tag}.f64", (kk, n_t))
        assert np.array_equal(t, rd(d, f"alone_t{tag}.f64", (kk, n_t))), tag
        f = rd(d, f"serve_f{tag}.f64", (kk,))
        assert np.array_equal(f, rd(d, f"alone_f{tag}.f64", (kk,))), tag
        it = np.fromfile(os.path.join(d, f"serve_i{tag}.i32"), np.int32)
        assert it.tolist() == [iters] * kk
        assert np.array_equal(it, np.fromfile(os.path.join(d, f"alone_i{tag}.i32"), np.int32))
        F = olp.planning_objective(case, w[sl], t.T, mask[sl])[0]
        assert rel_err(f, F) < 1e-5
    # warm starts: 2 iterations from the stored state of the same plans after 2
    # iterations equal 4 iterations from cold (up to the rounding of the
    # rebuilt W' columns)
    # rebuilt W' columns).  In the BF16 refinement mode a warm-started column
    # starts with zero references, so its first iteration multiplies the full
    # operands as single BF16 values (2^-9 relative rounding each) before the
    # refresh that ends the chunk.
    kk = 6
    tol_f, tol_t = (1e-6, 1e-5) if run == "serve" else (2e-3, 2e-2)
    assert np.fromfile(os.path.join(d, "warm_i.i32"), np.int32).tolist() == [2] * kk
    assert rel_err(rd(d, "warm_f.f64", (kk,)), rd(d, "cold2_f.f64", (kk,))) < tol_f
    assert rel_err(rd(d, "warm_t.f64", (kk, n_t)), rd(d, "cold2_t.f64", (kk, n_t))) < tol_t


@pytest.mark.parametrize("precision,k", COMPACT_CASES)
def test_emulated_compaction_gives_identical_results(emu, precision, k):
    """ladmm_batch_run with the running plans compacted into the lowest columns
    between checks, and without: the same bits for every plan, and plans that
    stopped at different checks."""
    d = finished(emu, f"compact-{precision}")
    case, w = _iter_spec(k, precision == "bf16")
    n_A = case.n_points + case.n_iso * case.n_sectors
    it_on = np.fromfile(os.path.join(d, "compact_it_on.i32"), np.int32)
    it_off = np.fromfile(os.path.join(d, "compact_it_off.i32"), np.int32)
    assert np.array_equal(it_on, it_off)
    assert len(set(it_on.tolist())) > 1, it_on     # plans stopped at different checks
    for name, shape in (("compact_t", (k, case.n_t)), ("compact_res", (7, k)), ("compact_z1", (n_A, k))):
        a = rd(d, name + "_on.f64", shape)
        b = rd(d, name + "_off.f64", shape)
        assert np.array_equal(a, b, equal_nan=True), name
