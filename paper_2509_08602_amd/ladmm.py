"""Python binding of libladmm (ctypes).  Argument marshalling only.

Every step of the solver runs in the HIP library; this module converts NumPy
arrays to the C structures of include/ladmm.h and back.  There is no fallback:
if the library is not built, importing works but the first call raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import dataclasses
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libladmm.so")

OK, PENDING = 0, 1
E_INVALID, E_NOMEM, E_DEVICE, E_NUMERIC, E_STATE, E_CANCELLED = -1, -2, -3, -4, -5, -6
F64, F32, BF16X3, BF16 = 0, 1, 2, 3
PT_TS, PT_TI, PT_RING, PT_LD, PT_OAR = 0, 1, 2, 3, 4
PLAN_CONVERGED, PLAN_MAX_ITER, PLAN_NUMERIC, PLAN_RUNNING = 0, 1, 2, 3
PRECISIONS = {"f64": F64, "f32": F32, "bf16x3": BF16X3, "bf16": BF16}


class LadmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ladmm error {code}: {msg}")
        self.code = code


class _Group(C.Structure):
    _fields_ = [("type", C.c_int32), ("structure", C.c_int32), ("threshold", C.c_double),
                ("share", C.c_double)]


class _CaseDesc(C.Structure):
    _fields_ = [("n_points", C.c_int32), ("n_iso", C.c_int32), ("n_sectors", C.c_int32),
                ("n_collimators", C.c_int32), ("dose", C.POINTER(C.c_double)),
                ("point_group", C.POINTER(C.c_int32)), ("n_groups", C.c_int32),
                ("groups", C.POINTER(_Group)), ("prescription_mean", C.c_double),
                ("phi_cal", C.c_double), ("precision", C.c_int32), ("row_normalize", C.c_int32),
                ("beta", C.c_double), ("beta_denominator", C.c_double)]


class _Weights(C.Structure):
    _fields_ = [("w_t", C.c_double), ("w_r", C.c_double), ("w_ld", C.c_double),
                ("w_bot", C.c_double)]


class _Opts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("check_every", C.c_int32), ("tol_gap", C.c_double),
                ("tol_pri", C.c_double), ("tol_dual", C.c_double), ("rho0", C.c_double),
                ("w0_bot", C.c_double), ("autotune", C.c_int32), ("adapt_rho", C.c_int32),
                ("adapt_mu", C.c_double), ("adapt_tau", C.c_double), ("alpha", C.c_double),
                ("tol_cert", C.c_double)]


_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int32)


class _Pass2(C.Structure):
    _fields_ = [("n_vox", C.c_int64), ("phi_vox", C.POINTER(C.c_double)), ("d_ld", C.c_double),
                ("delta", C.c_double), ("n_ld", C.POINTER(C.c_int32)), ("seed", C.c_uint64),
                ("ld_group", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("t", _DP), ("bot", _DP), ("objective", _DP), ("dual_obj", _DP),
                ("rel_gap", _DP), ("r_pri", _DP), ("r_dual", _DP), ("iters", _IP),
                ("plan_status", _IP), ("lower_bound", _DP), ("cert_gap", _DP)]


class _ServerOpts(C.Structure):
    _fields_ = [("slots", C.c_int32), ("check_every", C.c_int32), ("max_lanes", C.c_int32),
                ("autotune", C.c_int32), ("eager", C.c_int32), ("warm_store", C.c_int32)]


class _ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("cancelled", C.c_int64),
                ("failed", C.c_int64), ("plans_completed", C.c_int64),
                ("plan_iterations", C.c_int64), ("warm_starts", C.c_int64),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("max_ms", C.c_double), ("mean_ms", C.c_double), ("busy_ms", C.c_double),
                ("lanes", C.c_int32), ("busy_slots", C.c_int32)]


_lib = None
_EXITING = False
_SERVERS = weakref.WeakSet()


@atexit.register
def _at_exit():
    # Servers are stopped first (their worker threads call the HIP runtime).
    # Other handles still alive at interpreter exit are left to the process
    # teardown: calling into the HIP runtime from finalizers after this point is
    # unsafe.
    global _EXITING
    for s in list(_SERVERS):
        try:
            s.close()
        except Exception:
            pass
    _EXITING = True

# name -> (restype, argtypes)
_SIGS = {
    "ladmm_ctx_create": (C.c_int, [C.c_int, C.c_size_t, C.POINTER(C.c_void_p)]),
    "ladmm_ctx_destroy": (C.c_int, [C.c_void_p]),
    "ladmm_ctx_used_bytes": (C.c_size_t, [C.c_void_p]),
    "ladmm_create_case": (C.c_int, [C.c_void_p, C.POINTER(_CaseDesc), C.POINTER(C.c_void_p)]),
    "ladmm_destroy_case": (C.c_int, [C.c_void_p]),
    "ladmm_case_scaling": (C.c_int, [C.c_void_p, _DP, _DP]),
    "ladmm_case_schur": (C.c_int, [C.c_void_p, _DP, _DP]),
    "ladmm_case_setup_ms": (C.c_double, [C.c_void_p]),
    "ladmm_batch_create": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(_Weights),
                                     C.POINTER(C.c_uint64), _DP, C.POINTER(_Opts),
                                     C.POINTER(C.c_void_p)]),
    "ladmm_batch_destroy": (C.c_int, [C.c_void_p]),
    "ladmm_batch_iterate": (C.c_int, [C.c_void_p, C.c_int32]),
    "ladmm_batch_run": (C.c_int, [C.c_void_p]),
    "ladmm_batch_results": (C.c_int, [C.c_void_p, C.POINTER(_Result)]),
    "ladmm_batch_export": (C.c_int, [C.c_void_p, _DP, _DP, _DP, _DP]),
    "ladmm_batch_import": (C.c_int, [C.c_void_p, _DP, _DP, _DP, _DP]),
    "ladmm_batch_timing": (C.c_int, [C.c_void_p, _DP, C.POINTER(C.c_int64)]),
    "ladmm_batch_step_sizes": (C.c_int, [C.c_void_p, _DP]),
    "ladmm_batch_set_compaction": (C.c_int, [C.c_void_p, C.c_int32]),
    "ladmm_batch_run_checks": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "ladmm_batch_set_graphs": (C.c_int, [C.c_void_p, C.c_int32]),
    "ladmm_batch_metrics": (C.c_int, [C.c_void_p, C.c_int64, _DP, _IP, C.c_int32, _DP, C.c_double,
                                      _DP]),
    "ladmm_batch_set_profiling": (C.c_int, [C.c_void_p, C.c_int32]),
    "ladmm_batch_tiles": (C.c_int, [C.c_void_p, _IP, _IP]),
    "ladmm_batch_set_tiles": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "ladmm_batch_kernel_times": (C.c_int, [C.c_void_p, _DP, C.POINTER(C.c_int64)]),
    "ladmm_solve_batch": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(_Weights),
                                    C.POINTER(C.c_uint64), C.POINTER(_Opts), C.POINTER(_Result)]),
    "ladmm_batch_ld_band": (C.c_int, [C.c_void_p, C.c_int64, _DP, C.c_double, C.c_double,
                                      C.POINTER(C.c_uint64)]),
    "ladmm_select_ld_points": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_uint64),
                                         _IP, C.c_uint64, C.POINTER(C.c_int64),
                                         C.POINTER(C.c_int64), C.POINTER(C.c_uint64)]),
    "ladmm_select_ld_points_static": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64,
                                                C.POINTER(C.c_uint64), _IP, C.c_uint64,
                                                C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                                C.POINTER(C.c_uint64)]),
    "ladmm_two_pass": (C.c_int, [C.c_void_p, C.POINTER(_CaseDesc), C.c_int32, C.POINTER(_Weights),
                                 C.POINTER(_Opts), C.POINTER(_Pass2), C.c_void_p,
                                 C.POINTER(_Result), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                 _DP]),
    "ladmm_two_pass_sets": (C.c_int, [C.c_void_p, C.POINTER(_CaseDesc), C.c_int32, C.POINTER(_Weights),
                                 C.POINTER(_Opts), C.c_int32, C.POINTER(_Pass2), C.c_void_p,
                                 C.POINTER(_Result), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                 _DP]),
    "ladmm_passes": (C.c_int, [C.c_void_p, C.POINTER(_CaseDesc), C.c_int32, C.POINTER(_Weights),
                               C.POINTER(_Opts), C.c_int32, C.POINTER(_Pass2), C.c_int32,
                               C.POINTER(_Result), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                               _DP]),
    "ladmm_server_create": (C.c_int, [C.c_void_p, C.POINTER(_ServerOpts), C.POINTER(C.c_void_p)]),
    "ladmm_server_destroy": (C.c_int, [C.c_void_p]),
    "ladmm_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(_Weights),
                               C.POINTER(C.c_uint64), C.POINTER(_Opts), C.POINTER(_Result),
                               C.POINTER(C.c_uint64)]),
    "ladmm_poll": (C.c_int, [C.c_void_p, C.c_uint64, _IP]),
    "ladmm_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int64]),
    "ladmm_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
    "ladmm_server_get_stats": (C.c_int, [C.c_void_p, C.POINTER(_ServerStats)]),
    "ladmm_server_reset_stats": (C.c_int, [C.c_void_p]),
    "ladmm_last_error": (C.c_char_p, []),
    "ladmm_version": (C.c_char_p, []),
}


def library():
    """Load libladmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2509_08602_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc):
    if rc < 0:
        raise LadmmError(rc, library().ladmm_last_error().decode())
    return rc


def _dptr(a):
    return a.ctypes.data_as(_DP) if a is not None else None


@dataclasses.dataclass
class Options:
    """Solver options (see ladmm_opts in include/ladmm.h)."""
    max_iter: int = 3000
    check_every: int = 50
    tol_gap: float = 1e-4
    tol_pri: float = 1e-4
    tol_dual: float = 1e-4
    rho0: float = 1e4          # the rule's constant, tuned on the synthetic generator
    w0_bot: float = 1e-3
    autotune: bool = True
    adapt_rho: bool = True
    adapt_mu: float = 10.0
    adapt_tau: float = 2.0
    alpha: float = 1.0         # over-relaxation (1: the paper's ADMM)
    tol_cert: float = 0.0      # > 0: also stop only at a certified gap <= tol_cert

    def c(self):
        return _Opts(int(self.max_iter), int(self.check_every), float(self.tol_gap),
                     float(self.tol_pri), float(self.tol_dual), float(self.rho0),
                     float(self.w0_bot), 1 if self.autotune else 0, 1 if self.adapt_rho else 0,
                     float(self.adapt_mu), float(self.adapt_tau), float(self.alpha),
                     float(self.tol_cert))


class Context:
    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self._h = C.c_void_p()
        _check(library().ladmm_ctx_create(device, hbm_budget, C.byref(self._h)))

    @property
    def used_bytes(self):
        return int(library().ladmm_ctx_used_bytes(self._h))

    def close(self):
        if self._h:
            library().ladmm_ctx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        if _EXITING:
            return
        try:
            self.close()
        except Exception:
            pass


def _case_desc(dose, point_group, groups, n_iso, n_sectors, n_collimators, prescription_mean,
               phi_cal, precision, row_normalize=True, beta=None, beta_denominator=2000.0):
    """The C descriptor plus the arrays it points to (kept alive by the caller)."""
    dose = np.ascontiguousarray(dose, dtype=np.float64)
    pg = np.ascontiguousarray(point_group, dtype=np.int32)
    garr = (_Group * len(groups))(*[_Group(int(t), int(s), float(th), float(sh))
                                    for (t, s, th, sh) in groups])
    desc = _CaseDesc(dose.shape[0], int(n_iso), int(n_sectors), int(n_collimators),
                     dose.ctypes.data_as(_DP), pg.ctypes.data_as(_IP), len(groups), garr,
                     float(prescription_mean), float(phi_cal), PRECISIONS[precision],
                     1 if row_normalize else 0, float(beta) if beta else 0.0,
                     float(beta_denominator))
    return desc, (dose, pg, garr)


class Case:
    """A resident case: dose matrix, Schur complement factor and inverse in HBM."""

    def __init__(self, ctx: Context, dose, point_group, groups, n_iso, n_sectors=8,
                 n_collimators=3, prescription_mean=20.0, phi_cal=3.0, precision="f64",
                 row_normalize=True, beta=None, beta_denominator=2000.0):
        self.ctx = ctx
        desc, keep = _case_desc(dose, point_group, groups, n_iso, n_sectors, n_collimators,
                                prescription_mean, phi_cal, precision, row_normalize, beta,
                                beta_denominator)
        self.n_points, self.n_t = keep[0].shape
        self.n_iso, self.n_sectors, self.n_collimators = int(n_iso), int(n_sectors), int(n_collimators)
        self.precision = precision
        self._h = C.c_void_p()
        _check(library().ladmm_create_case(ctx._h, C.byref(desc), C.byref(self._h)))

    @classmethod
    def from_case(cls, ctx, case, precision="f64", **kw):
        """Marshal any object with the fields of a synthetic case (dose, group, ...)."""
        groups = [(g.type, g.structure, g.threshold, g.share) for g in case.groups]
        return cls(ctx, case.dose, case.group, groups, case.n_iso, case.n_sectors,
                   case.n_collimators, case.prescription_mean, case.phi_cal, precision, **kw)

    @property
    def m_A(self):
        return self.n_t + self.n_iso

    def scaling(self):
        E = np.empty(self.m_A)
        beta = C.c_double()
        _check(library().ladmm_case_scaling(self._h, _dptr(E), C.byref(beta)))
        return E, beta.value

    def schur(self):
        S = np.empty((self.m_A, self.m_A))
        Si = np.empty((self.m_A, self.m_A))
        _check(library().ladmm_case_schur(self._h, _dptr(S), _dptr(Si)))
        return S, Si

    @property
    def setup_ms(self):
        return float(library().ladmm_case_setup_ms(self._h))

    def close(self):
        if self._h:
            library().ladmm_destroy_case(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        if _EXITING:
            return
        try:
            self.close()
        except Exception:
            pass


def _weights(w):
    w = np.atleast_2d(np.asarray(w, np.float64))
    arr = (_Weights * w.shape[0])(*[_Weights(*map(float, row[:4])) for row in w])
    return arr, w.shape[0]


def _mask_words(mask, n_points):
    """k x N bool (or already-packed k x words uint64) -> contiguous uint64 words."""
    if mask is None:
        return None
    mask = np.asarray(mask)
    if mask.dtype == np.uint64:
        return np.ascontiguousarray(mask)
    k = mask.shape[0]
    nw = (n_points + 63) // 64
    padded = np.zeros((k, nw * 64), bool)
    padded[:, :mask.shape[1]] = mask
    bits = padded.reshape(k, nw, 64).astype(np.uint64) << np.arange(64, dtype=np.uint64)
    return np.ascontiguousarray(np.bitwise_or.reduce(bits, axis=2))


class Batch:
    """k plans of one case with their iterates resident in HBM."""

    def __init__(self, case: Case, weights, ld_mask=None, rho=None, opts: Options | None = None):
        self.case = case
        self.opts = opts or Options()
        self._w, self.k = _weights(weights)
        self._mask = _mask_words(ld_mask, case.n_points)
        rho_arr = None if rho is None else np.ascontiguousarray(rho, np.float64)
        self._h = C.c_void_p()
        mp = self._mask.ctypes.data_as(C.POINTER(C.c_uint64)) if self._mask is not None else None
        _check(library().ladmm_batch_create(case._h, self.k, self._w, mp, _dptr(rho_arr),
                                            C.byref(self.opts.c()), C.byref(self._h)))

    def iterate(self, n: int):
        _check(library().ladmm_batch_iterate(self._h, int(n)))

    def run(self, progress=None, checks_per_call=20):
        """Iterate until every plan has stopped.  With progress(running,
        iterations_run) the run returns to Python every checks_per_call checks
        to report the plans still running."""
        if progress is None:
            _check(library().ladmm_batch_run(self._h))
            return
        running = C.c_int32(1)
        while running.value > 0:
            _check(library().ladmm_batch_run_checks(self._h, int(checks_per_call), C.byref(running)))
            progress(int(running.value))

    def results(self, with_t=True):
        k, c = self.k, self.case
        out, r = _result_buffers(k, c.n_t, c.n_iso, with_t)
        _check(library().ladmm_batch_results(self._h, C.byref(r)))
        return out

    def export(self):
        c, k = self.case, self.k
        nA = c.n_points + c.n_iso * c.n_sectors
        z1, y1 = np.empty((nA, k)), np.empty((nA, k))
        z2, y2 = np.empty((c.m_A, k)), np.empty((c.m_A, k))
        _check(library().ladmm_batch_export(self._h, _dptr(z1), _dptr(y1), _dptr(z2), _dptr(y2)))
        return z1, y1, z2, y2

    def load(self, z1, y1, z2, y2):
        arrs = [np.ascontiguousarray(a, np.float64) for a in (z1, y1, z2, y2)]
        _check(library().ladmm_batch_import(self._h, *[_dptr(a) for a in arrs]))

    def timing(self):
        ms = C.c_double()
        pit = C.c_int64()
        _check(library().ladmm_batch_timing(self._h, C.byref(ms), C.byref(pit)))
        return ms.value, pit.value

    def set_compaction(self, on: bool):
        _check(library().ladmm_batch_set_compaction(self._h, 1 if on else 0))

    def step_sizes(self):
        rho = np.empty(self.k)
        _check(library().ladmm_batch_step_sizes(self._h, _dptr(rho)))
        return rho

    KERNEL_CLASSES = ("gemm1", "rhs", "schur_solve", "post", "gemm2", "objective",
                      "shot_scale", "finalize", "certificate", "gemm1_refresh", "gemm2_refresh")

    def tiles(self):
        a, b = C.c_int32(), C.c_int32()
        _check(library().ladmm_batch_tiles(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_tiles(self, gemm1, gemm2):
        _check(library().ladmm_batch_set_tiles(self._h, int(gemm1), int(gemm2)))

    def metrics(self, phi_vox, vox_target, presc, d_ref):
        """Clinical metrics (k x 4: coverage, selectivity, gradient index, beam-on
        time) of the current shot times on a dose grid (ladmm_batch_metrics)."""
        phi = np.ascontiguousarray(phi_vox, np.float64)
        tgt = np.ascontiguousarray(vox_target, np.int32)
        pr = np.ascontiguousarray(np.atleast_1d(presc), np.float64)
        out = np.empty((self.k, 4))
        _check(library().ladmm_batch_metrics(self._h, phi.shape[0], _dptr(phi), tgt.ctypes.data_as(_IP),
                                             pr.size, _dptr(pr), float(d_ref), _dptr(out)))
        return out

    def set_graphs(self, on=True):
        """Replay captured HIP graphs of each run chunk (default) or launch one by one."""
        _check(library().ladmm_batch_set_graphs(self._h, 1 if on else 0))

    def set_profiling(self, on=True):
        _check(library().ladmm_batch_set_profiling(self._h, 1 if on else 0))

    def kernel_times(self):
        """{class: (total ms, launches)} accumulated while profiling was on."""
        ms = np.zeros(len(self.KERNEL_CLASSES))
        n = np.zeros(len(self.KERNEL_CLASSES), np.int64)
        _check(library().ladmm_batch_kernel_times(self._h, _dptr(ms),
                                                  n.ctypes.data_as(C.POINTER(C.c_int64))))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(self.KERNEL_CLASSES)}

    def ld_band(self, phi_vox, d_ld, delta, packed=False):
        """Low-dose band of every plan at the candidate voxels (k x n_vox bool)."""
        phi = np.ascontiguousarray(phi_vox, np.float64)
        n_vox = phi.shape[0]
        W = (n_vox + 63) // 64
        bits = np.zeros((self.k, W), np.uint64)
        _check(library().ladmm_batch_ld_band(self._h, n_vox, _dptr(phi), float(d_ld), float(delta),
                                             bits.ctypes.data_as(C.POINTER(C.c_uint64))))
        return bits if packed else unpack(bits, n_vox)

    def close(self):
        if self._h:
            library().ladmm_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        if _EXITING:
            return
        try:
            self.close()
        except Exception:
            pass


def _result_buffers(k, n_t, n_iso, with_t=True):
    """Host result arrays of k plans and the ladmm_result that points at them."""
    out = dict(objective=np.empty(k), dual_obj=np.empty(k), rel_gap=np.empty(k),
               r_pri=np.empty(k), r_dual=np.empty(k), iters=np.empty(k, np.int32),
               plan_status=np.empty(k, np.int32), lower_bound=np.empty(k), cert_gap=np.empty(k))
    if with_t:
        out["t"] = np.empty((k, n_t))
        out["bot"] = np.empty((k, n_iso))
    r = _Result(_dptr(out.get("t")), _dptr(out.get("bot")), _dptr(out["objective"]),
                _dptr(out["dual_obj"]), _dptr(out["rel_gap"]), _dptr(out["r_pri"]),
                _dptr(out["r_dual"]), out["iters"].ctypes.data_as(_IP),
                out["plan_status"].ctypes.data_as(_IP), _dptr(out["lower_bound"]),
                _dptr(out["cert_gap"]))
    return out, r


def two_pass(ctx: Context, case, weights, phi_vox, d_ld, delta, n_ld, seed, ld_group,
             precision="f64", opts: Options | None = None):
    """ladmm_two_pass: both passes for every plan (case: a synthetic-case-like object).

    Returns (pass1 results, pass2 results, P, n_points2, times_ms)."""
    groups = [(g.type, g.structure, g.threshold, g.share) for g in case.groups]
    desc, keep = _case_desc(case.dose, case.group, groups, case.n_iso, case.n_sectors,
                            case.n_collimators, case.prescription_mean, case.phi_cal, precision)
    w, k = _weights(weights)
    phi = np.ascontiguousarray(phi_vox, np.float64)
    nld = np.ascontiguousarray(np.broadcast_to(np.asarray(n_ld, np.int32), (k,)))
    p2 = _Pass2(phi.shape[0], _dptr(phi), float(d_ld), float(delta), nld.ctypes.data_as(_IP),
                C.c_uint64(int(seed) & ((1 << 64) - 1)), int(ld_group))
    n_t = case.dose.shape[1]
    out1, r1 = _result_buffers(k, n_t, case.n_iso)
    out2, r2 = _result_buffers(k, n_t, case.n_iso)
    P = np.zeros(phi.shape[0], np.int64)
    n2 = np.zeros(2, np.int64)
    times = np.zeros(5)
    o = (opts or Options()).c()
    _check(library().ladmm_two_pass(ctx._h, C.byref(desc), k, w, C.byref(o), C.byref(p2),
                                    C.cast(C.pointer(r1), C.c_void_p), C.byref(r2),
                                    P.ctypes.data_as(C.POINTER(C.c_int64)),
                                    n2.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(times)))
    return out1, out2, P[:n2[0]], int(n2[1]), times


def two_pass_sets(ctx: Context, case, weights, sets, precision="f64", opts: Options | None = None):
    """ladmm_two_pass_sets: both passes with several low-dose groups replaced.

    sets: list of dicts with phi_vox, d_ld, delta, n_ld, seed, ld_group.
    Returns (pass1 results, pass2 results, [P_i per set], pass-2 point count, times_ms)."""
    groups = [(g.type, g.structure, g.threshold, g.share) for g in case.groups]
    desc, keep = _case_desc(case.dose, case.group, groups, case.n_iso, case.n_sectors,
                            case.n_collimators, case.prescription_mean, case.phi_cal, precision)
    w, k = _weights(weights)
    hold, descs = [], (_Pass2 * len(sets))()
    for i, st in enumerate(sets):
        phi = np.ascontiguousarray(st["phi_vox"], np.float64)
        nld = np.ascontiguousarray(np.broadcast_to(np.asarray(st["n_ld"], np.int32), (k,)))
        hold += [phi, nld]
        descs[i] = _Pass2(phi.shape[0], _dptr(phi), float(st["d_ld"]), float(st["delta"]),
                          nld.ctypes.data_as(_IP), C.c_uint64(int(st["seed"]) & ((1 << 64) - 1)),
                          int(st["ld_group"]))
    n_t = case.dose.shape[1]
    out1, r1 = _result_buffers(k, n_t, case.n_iso)
    out2, r2 = _result_buffers(k, n_t, case.n_iso)
    P = np.zeros(sum(int(d.n_vox) for d in descs), np.int64)
    n2 = np.zeros(len(sets) + 1, np.int64)
    times = np.zeros(5)
    o = (opts or Options()).c()
    _check(library().ladmm_two_pass_sets(ctx._h, C.byref(desc), k, w, C.byref(o), len(sets), descs,
                                         C.cast(C.pointer(r1), C.c_void_p), C.byref(r2),
                                         P.ctypes.data_as(C.POINTER(C.c_int64)),
                                         n2.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(times)))
    parts, at = [], 0
    for i in range(len(sets)):
        parts.append(P[at:at + n2[i]].copy())
        at += int(n2[i])
    return out1, out2, parts, int(n2[-1]), times


def passes(ctx: Context, case, weights, sets, n_passes, precision="f64", opts: Options | None = None):
    """ladmm_passes: n_passes passes, each later one taking its low-dose points
    from the previous pass's dose (sets as for two_pass_sets).

    Returns ([results of every pass], [P_i of the last pass per set], last pass's
    point count, times_ms)."""
    groups = [(g.type, g.structure, g.threshold, g.share) for g in case.groups]
    desc, keep = _case_desc(case.dose, case.group, groups, case.n_iso, case.n_sectors,
                            case.n_collimators, case.prescription_mean, case.phi_cal, precision)
    w, k = _weights(weights)
    hold, descs = [], (_Pass2 * len(sets))()
    for i, st in enumerate(sets):
        phi = np.ascontiguousarray(st["phi_vox"], np.float64)
        nld = np.ascontiguousarray(np.broadcast_to(np.asarray(st["n_ld"], np.int32), (k,)))
        hold += [phi, nld]
        descs[i] = _Pass2(phi.shape[0], _dptr(phi), float(st["d_ld"]), float(st["delta"]),
                          nld.ctypes.data_as(_IP), C.c_uint64(int(st["seed"]) & ((1 << 64) - 1)),
                          int(st["ld_group"]))
    n_t = case.dose.shape[1]
    outs, recs = [], (_Result * n_passes)()
    for q in range(n_passes):
        o_q, r_q = _result_buffers(k, n_t, case.n_iso)
        outs.append(o_q)
        recs[q] = r_q
    P = np.zeros(sum(int(d.n_vox) for d in descs), np.int64)
    n2 = np.zeros(len(sets) + 1, np.int64)
    times = np.zeros(2 + 3 * (n_passes - 1))
    o = (opts or Options()).c()
    _check(library().ladmm_passes(ctx._h, C.byref(desc), k, w, C.byref(o), len(sets), descs,
                                  int(n_passes), recs, P.ctypes.data_as(C.POINTER(C.c_int64)),
                                  n2.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(times)))
    parts, at = [], 0
    for i in range(len(sets)):
        parts.append(P[at:at + n2[i]].copy())
        at += int(n2[i])
    return outs, parts, int(n2[-1]), times


def solve_batch(case: Case, weights, ld_mask=None, opts: Options | None = None):
    """ladmm_solve_batch: run k plans to convergence and return their results."""
    w, k = _weights(weights)
    mask = _mask_words(ld_mask, case.n_points)
    mp = mask.ctypes.data_as(C.POINTER(C.c_uint64)) if mask is not None else None
    o = (opts or Options()).c()
    out, r = _result_buffers(k, case.n_t, case.n_iso)
    _check(library().ladmm_solve_batch(case._h, k, w, mp, C.byref(o), C.byref(r)))
    return out


def unpack(words, n):
    """k x W uint64 -> k x n bool (bit b of word w = element 64 w + b)."""
    words = np.asarray(words, np.uint64)
    bits = (words[:, :, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)
    return bits.reshape(words.shape[0], -1)[:, :n].astype(bool)


def select_ld_points(ctx: Context, volumes, n_ld, seed: int, static: bool = False):
    """Algorithm 1 on the device.  volumes: k x n_vox bool.  Returns (P, mask
    words, masks) with masks k x |P| bool.  static: the allocation-free entry
    point (ladmm_select_ld_points_static)."""
    vols = np.asarray(volumes)
    k, n_vox = vols.shape
    bits = _mask_words(vols, n_vox) if k else np.zeros((0, (n_vox + 63) // 64), np.uint64)
    n = np.ascontiguousarray(np.broadcast_to(np.asarray(n_ld, np.int32), (k,)))
    W = (n_vox + 63) // 64
    P = np.zeros(n_vox, np.int64)
    nP = C.c_int64()
    masks = np.zeros((max(k, 1), W), np.uint64)
    fn = library().ladmm_select_ld_points_static if static else library().ladmm_select_ld_points
    _check(fn(
        ctx._h, k, n_vox, bits.ctypes.data_as(C.POINTER(C.c_uint64)), n.ctypes.data_as(_IP),
        C.c_uint64(int(seed) & ((1 << 64) - 1)), P.ctypes.data_as(C.POINTER(C.c_int64)),
        C.byref(nP), masks.ctypes.data_as(C.POINTER(C.c_uint64))))
    npts = nP.value
    return P[:npts], masks[:k], unpack(masks[:k], npts) if k else np.zeros((0, 0), bool)


class Ticket:
    """A request queued on a Server; owns the result arrays the library writes."""

    def __init__(self, server, case, weights, ld_mask, opts):
        self.server, self.case = server, case
        self._w, self.k = _weights(weights)
        self._mask = _mask_words(ld_mask, case.n_points)
        self.out, self._r = _result_buffers(self.k, case.n_t, case.n_iso)
        self.status = PENDING
        self.id = C.c_uint64()
        mp = self._mask.ctypes.data_as(C.POINTER(C.c_uint64)) if self._mask is not None else None
        _check(library().ladmm_submit(server._h, case._h, self.k, self._w, mp,
                                      C.byref((opts or Options()).c()), C.byref(self._r),
                                      C.byref(self.id)))

    def _final(self, rc):
        if rc != PENDING:
            self.status = rc
            self.server._done(self)
        return rc

    def poll(self):
        """(status, plans_done); status is PENDING until the request is final."""
        if self.status != PENDING:
            return self.status, self.k
        n = C.c_int32()
        rc = library().ladmm_poll(self.server._h, self.id, C.byref(n))
        if rc < 0 and rc != E_CANCELLED:
            self._final(rc)
            raise LadmmError(rc, library().ladmm_last_error().decode())
        return self._final(rc), n.value

    def wait(self, timeout: float | None = None):
        """Block until final (or timeout seconds); returns the status."""
        if self.status != PENDING:
            return self.status
        us = -1 if timeout is None else int(timeout * 1e6)
        rc = library().ladmm_wait(self.server._h, self.id, us)
        if rc < 0 and rc != E_CANCELLED:
            self._final(rc)
            raise LadmmError(rc, library().ladmm_last_error().decode())
        return self._final(rc)

    def cancel(self):
        if self.status == PENDING:
            _check(library().ladmm_cancel(self.server._h, self.id))

    def result(self):
        """Per-plan results (dict of arrays); waits for the request first."""
        if self.wait() != OK:
            raise LadmmError(self.status, "request did not complete")
        return self.out


class Server:
    """Continuous-batching server (ladmm_server_*): requests of k plans on resident cases."""

    def __init__(self, ctx: Context, slots: int = 96, check_every: int = 50, max_lanes: int = 0,
                 autotune: bool = True, eager: bool = False, warm_store: int = 0):
        self.ctx = ctx
        self.check_every = int(check_every)
        self._h = C.c_void_p()
        self._live = {}
        o = _ServerOpts(int(slots), int(check_every), int(max_lanes), 1 if autotune else 0,
                        1 if eager else 0, int(warm_store))
        _check(library().ladmm_server_create(ctx._h, C.byref(o), C.byref(self._h)))
        _SERVERS.add(self)

    def submit(self, case: Case, weights, ld_mask=None, opts: Options | None = None) -> Ticket:
        t = Ticket(self, case, weights, ld_mask, opts)
        self._live[t.id.value] = t   # keeps the buffers alive until final
        return t

    def _done(self, t):
        self._live.pop(t.id.value, None)

    def stats(self):
        s = _ServerStats()
        _check(library().ladmm_server_get_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in _ServerStats._fields_}

    def reset_stats(self):
        _check(library().ladmm_server_reset_stats(self._h))

    def close(self):
        if self._h:
            library().ladmm_server_destroy(self._h)
            self._h = C.c_void_p()
            for t in self._live.values():
                if t.status == PENDING:
                    t.status = E_CANCELLED
            self._live.clear()

    def __del__(self):
        if _EXITING:
            return
        try:
            self.close()
        except Exception:
            pass
