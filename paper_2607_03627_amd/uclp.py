"""Python binding of libuclp (include/uc_lp.h): argument marshalling only.

Every function keeps the name of the C entry point it wraps.  Arrays are
NumPy arrays on the host; the library copies them to the device itself.
Loading fails loudly when the built library is missing: there is no
fallback path.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libuclp.so")

# enums of include/uc_lp.h
UC_LP_OK, UC_LP_EINVAL, UC_LP_ENOMEM, UC_LP_EBUDGET, UC_LP_EHIP, UC_LP_ESTATE, UC_LP_ENOTSUP, UC_LP_ETIMEOUT = \
    0, -1, -2, -3, -4, -5, -6, -7
UC_LP_FP64, UC_LP_FP32_MIXED, UC_LP_FP32_MIXED_POLISH, UC_LP_FP32_REFINE = 0, 1, 2, 3
(UC_LP_IDLE, UC_LP_QUEUED, UC_LP_RUNNING, UC_LP_OPTIMAL, UC_LP_ITER_LIMIT, UC_LP_TIME_LIMIT,
 UC_LP_CANCELLED, UC_LP_NUMERICAL, UC_LP_INFEASIBLE, UC_LP_FAILED) = range(10)
UC_LP_SPMV_ROWSPLIT, UC_LP_SPMV_MERGEPATH = 0, 1
STATUS_NAMES = ["IDLE", "QUEUED", "RUNNING", "OPTIMAL", "ITER_LIMIT", "TIME_LIMIT", "CANCELLED",
                "NUMERICAL", "INFEASIBLE", "FAILED"]
TERMINAL = {UC_LP_OPTIMAL, UC_LP_ITER_LIMIT, UC_LP_TIME_LIMIT, UC_LP_CANCELLED, UC_LP_NUMERICAL,
            UC_LP_INFEASIBLE, UC_LP_FAILED}


class uc_lp_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("kkt_every", C.c_int32), ("ruiz_iters", C.c_int32),
                ("power_iters", C.c_int32), ("iter_limit", C.c_int64), ("eps_rel", C.c_double),
                ("eps_abs_feas", C.c_double), ("eps_polish", C.c_double), ("time_limit_s", C.c_double),
                ("step_scale", C.c_double), ("spmv_algo", C.c_int32), ("verbose", C.c_int32),
                ("timing", C.c_int32), ("restart_to_current", C.c_int32),
                ("restart_sufficient", C.c_double), ("restart_necessary", C.c_double),
                ("restart_artificial", C.c_double), ("pw_smoothing", C.c_double),
                ("halpern_gamma", C.c_double), ("pw_max_change", C.c_double),
                ("fp32_stall_checks", C.c_int32), ("reserved", C.c_int32), ("pw_integral", C.c_double),
                ("pw_balance", C.c_double), ("pw_balance_polish", C.c_double), ("eps_gap_rel", C.c_double),
                ("eps_refine", C.c_double), ("refine_growth", C.c_double), ("refine_max_rounds", C.c_int32),
                ("reserved2", C.c_int32), ("pw_balance_refine", C.c_double), ("refine_diverge", C.c_double)]


class uc_lp_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("precision_now", C.c_int32), ("iters", C.c_int64),
                ("iters_fp64", C.c_int64), ("restarts", C.c_int64), ("t_total_s", C.c_double),
                ("t_setup_s", C.c_double), ("t_to_eps_s", C.c_double), ("t_queue_s", C.c_double),
                ("pobj", C.c_double), ("dobj", C.c_double), ("rel_primal", C.c_double),
                ("rel_dual", C.c_double), ("rel_gap", C.c_double), ("rel_kkt", C.c_double),
                ("abs_primal_inf", C.c_double), ("pobj_at_eps", C.c_double),
                ("rel_kkt_at_eps", C.c_double), ("iters_at_eps", C.c_int64),
                ("norm_a_est", C.c_double), ("omega", C.c_double),
                ("primal_kernel_us", C.c_double), ("dual_kernel_us", C.c_double),
                ("timed_launches", C.c_int64), ("m_presolved", C.c_int32), ("n_presolved", C.c_int32),
                ("nnz_presolved", C.c_int64), ("device_bytes", C.c_int64),
                ("primal_bytes", C.c_double), ("dual_bytes", C.c_double), ("rel_gap_at_eps", C.c_double),
                ("fp_residual", C.c_double), ("norm_a_bound", C.c_double), ("eta", C.c_double),
                ("refine_rounds", C.c_int32), ("reserved_i", C.c_int32), ("rel_kkt_inner", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status_name"] = STATUS_NAMES[self.status] if 0 <= self.status < len(STATUS_NAMES) else "?"
        return d


EXPORTS = ["uc_lp_opts_default", "uc_engine_create", "uc_engine_destroy", "uc_lp_create", "uc_lp_create_device",
           "uc_lp_get_solution_device",
           "uc_lp_update_data", "uc_lp_solve", "uc_lp_status", "uc_lp_wait", "uc_lp_cancel",
           "uc_lp_get_solution", "uc_lp_destroy", "uc_lp_last_error", "uc_lp_solve_scenarios",
           "uc_lp_internal_dims", "uc_lp_get_transpose", "uc_lp_get_scaling", "uc_lp_debug_step",
           "uc_lp_debug_iterate", "uc_lp_eval_kkt", "uc_lp_debug_refine", "uc_spmv", "uc_spmv_bench", "uc_copy_bench", "uc_lp_bench_half_steps",
           "uc_spmv_merge_noalloc"]

_lib: Optional[C.CDLL] = None

_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int32)
_F = C.POINTER(C.c_float)


def _sig(lib):
    lib.uc_lp_opts_default.argtypes = [C.POINTER(uc_lp_opts)]
    lib.uc_lp_opts_default.restype = None
    lib.uc_engine_create.argtypes = [C.c_int, C.c_size_t, C.c_int32, C.POINTER(_P)]
    lib.uc_engine_destroy.argtypes = [_P]
    lib.uc_engine_destroy.restype = None
    lib.uc_lp_create.argtypes = [_P, C.c_int32, C.c_int32, C.c_int64, _I, _I, _D, _D, _D, C.c_char_p,
                                 _D, _D, C.POINTER(uc_lp_opts), C.POINTER(_P)]
    lib.uc_lp_create_device.argtypes = [_P, C.c_int32, C.c_int32, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P,
                                        C.POINTER(uc_lp_opts), _P, C.POINTER(_P)]
    lib.uc_lp_get_solution_device.argtypes = [_P, _P, _P, _P]
    lib.uc_lp_update_data.argtypes = [_P, _D, _D, _D, _D]
    lib.uc_lp_solve.argtypes = [_P, _D, _D]
    lib.uc_lp_status.argtypes = [_P, C.POINTER(uc_lp_info)]
    lib.uc_lp_wait.argtypes = [_P, C.c_double]
    lib.uc_lp_cancel.argtypes = [_P]
    lib.uc_lp_get_solution.argtypes = [_P, _D, _D]
    lib.uc_lp_destroy.argtypes = [_P]
    lib.uc_lp_destroy.restype = None
    lib.uc_lp_last_error.argtypes = []
    lib.uc_lp_last_error.restype = C.c_char_p
    lib.uc_lp_solve_scenarios.argtypes = [_P, C.c_int32, _D, _D, _D, _D, _D, _D, _D, _D,
                                          C.POINTER(uc_lp_info)]
    lib.uc_lp_internal_dims.argtypes = [_P, _I, _I, C.POINTER(C.c_int64), _I, _I, _I]
    lib.uc_lp_get_transpose.argtypes = [_P, _I, _I, _D]
    lib.uc_lp_get_scaling.argtypes = [_P, _D, _D, _D]
    lib.uc_lp_debug_step.argtypes = [_P, C.c_int32, _D, _D, _D, _D, C.c_int64, C.c_double, C.c_double,
                                     _D, _D, _D, _D]
    lib.uc_lp_debug_iterate.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32, _D, _D, _D, _D, C.c_int64,
                                        C.c_double, C.c_double, _D, _D, _D, _D, _D]
    lib.uc_lp_eval_kkt.argtypes = [_P, _D, _D, C.POINTER(uc_lp_info)]
    lib.uc_lp_debug_refine.argtypes = [_P, _D, _D, _F, _F, C.c_int32, _D, _D, _D, _D, _F, _D]
    lib.uc_spmv.argtypes = [C.c_int, C.c_int32, C.c_int32, C.c_int64, _I, _I, _D, _D, _D, C.c_int32,
                            C.c_int32]
    lib.uc_spmv_bench.argtypes = [C.c_int, C.c_int32, C.c_int32, C.c_int64, _I, _I, _D, C.c_int32,
                                  C.c_int32, C.c_int32, C.c_int32, _D]
    lib.uc_copy_bench.argtypes = [C.c_int, C.c_size_t, C.c_int32, _D]
    lib.uc_lp_bench_half_steps.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32, _D, _D, _D, _D]
    lib.uc_spmv_merge_noalloc.argtypes = [C.c_int, C.c_int32, C.c_int32, C.c_int64, _P, _P, _P, _P, _P, C.c_int32,
                                          _P]
    for name in ("uc_engine_create", "uc_lp_create", "uc_lp_create_device", "uc_lp_get_solution_device",
                 "uc_lp_update_data", "uc_lp_solve", "uc_lp_status",
                 "uc_lp_wait", "uc_lp_cancel", "uc_lp_get_solution", "uc_lp_solve_scenarios",
                 "uc_lp_internal_dims", "uc_lp_get_transpose", "uc_lp_get_scaling", "uc_lp_debug_step",
                 "uc_lp_debug_iterate", "uc_lp_eval_kkt", "uc_lp_debug_refine", "uc_spmv", "uc_spmv_bench", "uc_copy_bench",
                 "uc_lp_bench_half_steps", "uc_spmv_merge_noalloc"):
        getattr(lib, name).restype = C.c_int


def load(path: str = None) -> C.CDLL:
    """Load the built library; raises if it is missing (build it first).
    UCLP_LIB in the environment names another build of it (the host
    sanitizer build the CPU tests run against)."""
    global _lib
    if path is None:
        path = os.environ.get("UCLP_LIB", LIB_PATH)
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"libuclp not built: {path} is missing "
                               "(run `python -m paper_2607_03627_amd.build`)")
        lib = C.CDLL(path)
        _sig(lib)
        _lib = lib
    return _lib


class UcLpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"uclp error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != UC_LP_OK:
        raise UcLpError(rc, uc_lp_last_error())
    return rc


def _d(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _i(a):
    return a.ctypes.data_as(_I) if a is not None else None


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---------------------------------------------------------------------------
# thin wrappers, one per entry point
# ---------------------------------------------------------------------------

def uc_lp_last_error() -> str:
    return load().uc_lp_last_error().decode(errors="replace")


def uc_lp_opts_default(**overrides) -> uc_lp_opts:
    o = uc_lp_opts()
    load().uc_lp_opts_default(C.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def uc_engine_create(device: int = 0, hbm_budget_bytes: int = 0, max_slots: int = 64):
    h = _P()
    _check(load().uc_engine_create(device, hbm_budget_bytes, max_slots, C.byref(h)))
    return h


def uc_engine_destroy(eng) -> None:
    load().uc_engine_destroy(eng)


def uc_lp_create(lp, opts: Optional[uc_lp_opts] = None, engine=None, raw: bool = False):
    """lp: an object with m, n, row_ptr, col_idx, val, c, b, sense, lb, ub.
    raw=True returns the error code instead of raising (handle is None then)."""
    rp, ci = _i32(lp.row_ptr), _i32(lp.col_idx)
    val = _f64(lp.val)
    c, b, lb, ub = _f64(lp.c), _f64(lp.b), _f64(lp.lb), _f64(lp.ub)
    sense = np.ascontiguousarray(lp.sense, dtype=np.uint8).tobytes()
    h = _P()
    rc = load().uc_lp_create(engine, int(lp.m), int(lp.n), int(len(ci)), _i(rp), _i(ci), _d(val), _d(c),
                             _d(b), sense, _d(lb), _d(ub), C.byref(opts) if opts is not None else None,
                             C.byref(h))
    if raw:
        return rc, (h if rc == UC_LP_OK else None)
    _check(rc)
    return h


def uc_lp_create_device(m, n, nnz, row_ptr, col_idx, val, c, b, sense, lb, ub, opts: Optional[uc_lp_opts] = None,
                        engine=None, stream=None, raw: bool = False):
    """Device addresses (ints, e.g. tensor.data_ptr()) of caller-owned arrays
    (int32 row_ptr/col_idx, float64 val/c/b/lb/ub, uint8 sense); stream: a
    hipStream_t address or None.  raw=True returns (rc, handle or None)."""
    h = _P()
    rc = load().uc_lp_create_device(engine, int(m), int(n), int(nnz), _P(row_ptr), _P(col_idx) if col_idx else None,
                                    _P(val) if val else None, _P(c), _P(b), _P(sense), _P(lb), _P(ub),
                                    C.byref(opts) if opts is not None else None, _P(stream) if stream else None,
                                    C.byref(h))
    if raw:
        return rc, (h if rc == UC_LP_OK else None)
    _check(rc)
    return h


def uc_lp_get_solution_device(h, x_ptr, y_ptr, stream=None, raw: bool = False):
    """Copy the solution into caller-owned device arrays (addresses as ints, or None)."""
    rc = load().uc_lp_get_solution_device(h, _P(x_ptr) if x_ptr else None, _P(y_ptr) if y_ptr else None,
                                          _P(stream) if stream else None)
    return rc if raw else _check(rc)


def uc_lp_update_data(h, c=None, b=None, lb=None, ub=None) -> None:
    c, b, lb, ub = _f64(c), _f64(b), _f64(lb), _f64(ub)
    _check(load().uc_lp_update_data(h, _d(c), _d(b), _d(lb), _d(ub)))


def uc_lp_solve(h, x0=None, y0=None) -> None:
    x0, y0 = _f64(x0), _f64(y0)
    _check(load().uc_lp_solve(h, _d(x0), _d(y0)))


def uc_lp_status(h) -> uc_lp_info:
    info = uc_lp_info()
    _check(load().uc_lp_status(h, C.byref(info)))
    return info


def uc_lp_wait(h, timeout_s: float = -1.0) -> bool:
    rc = load().uc_lp_wait(h, float(timeout_s))
    if rc == UC_LP_ETIMEOUT:
        return False
    _check(rc)
    return True


def uc_lp_cancel(h) -> None:
    _check(load().uc_lp_cancel(h))


def uc_lp_get_solution(h, n: int, m: int) -> Tuple[np.ndarray, np.ndarray]:
    x = np.empty(n)
    y = np.empty(m)
    _check(load().uc_lp_get_solution(h, _d(x), _d(y)))
    return x, y


def uc_lp_destroy(h) -> None:
    if h:
        load().uc_lp_destroy(h)


def uc_lp_solve_scenarios(h, n: int, m: int, c, b, lb, ub, x0=None, y0=None):
    """c, lb, ub: (n_scen, n); b: (n_scen, m).  Returns x (n_scen, n), y (n_scen, m), infos."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    ns = c.shape[0]
    b = np.ascontiguousarray(b, dtype=np.float64)
    lb = np.ascontiguousarray(lb, dtype=np.float64)
    ub = np.ascontiguousarray(ub, dtype=np.float64)
    x = np.empty((ns, n))
    y = np.empty((ns, m))
    infos = (uc_lp_info * ns)()
    _check(load().uc_lp_solve_scenarios(h, ns, _d(c), _d(b), _d(lb), _d(ub), _d(_f64(x0)), _d(_f64(y0)),
                                        _d(x), _d(y), infos))
    return x, y, list(infos)


def uc_lp_internal_dims(h):
    m, n, meq = C.c_int32(), C.c_int32(), C.c_int32()
    z = C.c_int64()
    _check(load().uc_lp_internal_dims(h, C.byref(m), C.byref(n), C.byref(z), C.byref(meq), None, None))
    rmap = np.empty(m.value, np.int32)
    cmap = np.empty(n.value, np.int32)
    _check(load().uc_lp_internal_dims(h, None, None, None, None, _i(rmap), _i(cmap)))
    return dict(m=m.value, n=n.value, nnz=z.value, m_eq=meq.value, row_map=rmap, col_map=cmap)


def uc_lp_get_transpose(h, n_int: int, nnz_int: int):
    tp = np.empty(n_int + 1, np.int32)
    tc = np.empty(max(nnz_int, 1), np.int32)
    tv = np.empty(max(nnz_int, 1))
    _check(load().uc_lp_get_transpose(h, _i(tp), _i(tc), _d(tv)))
    return tp, tc[:nnz_int], tv[:nnz_int]


def uc_lp_get_scaling(h, m_int: int, n_int: int):
    dr = np.empty(max(m_int, 1))
    dc = np.empty(n_int)
    ne = C.c_double()
    _check(load().uc_lp_get_scaling(h, _d(dr), _d(dc), C.byref(ne)))
    return dr[:m_int], dc, ne.value


def uc_lp_debug_step(h, precision, x, y, x0, y0, k, tau, sigma):
    x, y, x0, y0 = _f64(x), _f64(y), _f64(x0), _f64(y0)
    xh, yh, xn, yn = np.empty_like(x), np.empty_like(y), np.empty_like(x), np.empty_like(y)
    _check(load().uc_lp_debug_step(h, int(precision), _d(x), _d(y), _d(x0), _d(y0), int(k), float(tau),
                                   float(sigma), _d(xh), _d(yh), _d(xn), _d(yn)))
    return xh, yh, xn, yn


def uc_lp_debug_iterate(h, precision, iters, x, y, x0, y0, k, tau, sigma, block_threads=0):
    """Returns x_hat, y_hat, x_next, y_next, fp_residual (see include/uc_lp.h)."""
    x, y, x0, y0 = _f64(x), _f64(y), _f64(x0), _f64(y0)
    xh, yh, xn, yn = np.empty_like(x), np.empty_like(y), np.empty_like(x), np.empty_like(y)
    r = C.c_double()
    _check(load().uc_lp_debug_iterate(h, int(precision), int(iters), int(block_threads), _d(x), _d(y), _d(x0),
                                      _d(y0), int(k), float(tau), float(sigma), _d(xh), _d(yh), _d(xn), _d(yn),
                                      C.byref(r)))
    return xh, yh, xn, yn, r.value


def uc_lp_eval_kkt(h, x, y) -> uc_lp_info:
    info = uc_lp_info()
    _check(load().uc_lp_eval_kkt(h, _d(_f64(x)), _d(_f64(y)), C.byref(info)))
    return info


def uc_lp_debug_refine(h, x_corr, y_corr, par, x_star=None, y_star=None, first=False):
    """One refinement round boundary (see include/uc_lp.h).  x_corr, y_corr
    are rounded to FP32; par = (inv_dp, inv_dd, dp_prev, dd_prev, growth,
    omega_prev).  Returns dict(x, y, c, l, u, b (FP64), c32, l32, u32, b32,
    ylo32, scal)."""
    xc = np.ascontiguousarray(x_corr, dtype=np.float32)
    yc = np.ascontiguousarray(y_corr, dtype=np.float32)
    n, m = xc.size, yc.size
    xs = _f64(x_star) if not first else None
    ys = _f64(y_star) if not first else None
    p = _f64(par, 6)
    xn, yn = np.empty(n), np.empty(max(m, 1))
    d64 = np.empty(3 * n + m)
    d32 = np.empty(3 * n + 2 * m, np.float32)
    sc = np.empty(14)
    _check(load().uc_lp_debug_refine(h, _d(xs), _d(ys), xc.ctypes.data_as(_F), yc.ctypes.data_as(_F),
                                      int(bool(first)), _d(p), _d(xn), _d(yn), _d(d64),
                                      d32.ctypes.data_as(_F), _d(sc)))
    names = ["dp", "dd", "omega", "viol2", "dres2", "viol2u", "by", "vmaxu", "dres2u", "lbub", "cx",
             "norm_b_t", "norm_c_t", "rel_kkt"]
    return dict(x=xn, y=yn[:m], c=d64[:n], l=d64[n:2 * n], u=d64[2 * n:3 * n], b=d64[3 * n:],
                c32=d32[:n], l32=d32[n:2 * n], u32=d32[2 * n:3 * n], b32=d32[3 * n:3 * n + m],
                ylo32=d32[3 * n + m:], scal=dict(zip(names, sc)))


def uc_spmv(m, n, row_ptr, col_idx, val, x, precision=UC_LP_FP64, algo=UC_LP_SPMV_ROWSPLIT, device=0):
    rp, ci, v, x = _i32(row_ptr), _i32(col_idx), _f64(val), _f64(x, n)
    y = np.empty(m)
    _check(load().uc_spmv(device, int(m), int(n), int(len(ci)), _i(rp), _i(ci), _d(v), _d(x), _d(y),
                          int(precision), int(algo)))
    return y


def uc_spmv_bench(m, n, row_ptr, col_idx, val, precision=UC_LP_FP32_MIXED, algo=UC_LP_SPMV_ROWSPLIT,
                  copies=4, reps=50, device=0) -> float:
    rp, ci, v = _i32(row_ptr), _i32(col_idx), _f64(val)
    us = C.c_double()
    _check(load().uc_spmv_bench(device, int(m), int(n), int(len(ci)), _i(rp), _i(ci), _d(v), int(precision),
                                int(algo), int(copies), int(reps), C.byref(us)))
    return us.value


def uc_lp_bench_half_steps(h, precision=UC_LP_FP32_MIXED, copies=4, reps=64):
    """Returns dict(primal_us, dual_us, primal_bytes, dual_bytes)."""
    v = [C.c_double() for _ in range(4)]
    _check(load().uc_lp_bench_half_steps(h, int(precision), int(copies), int(reps), *[C.byref(x) for x in v]))
    return dict(primal_us=v[0].value, dual_us=v[1].value, primal_bytes=v[2].value, dual_bytes=v[3].value)


def uc_spmv_merge_noalloc(m, n, nnz, row_ptr, col_idx, val, x, y, precision=UC_LP_FP64, stream=None, device=0,
                          raw=False):
    """Device addresses (ints) of caller-owned arrays; stream: a hipStream_t
    address or None.  raw=True returns the error code instead of raising."""
    rc = load().uc_spmv_merge_noalloc(int(device), int(m), int(n), int(nnz), _P(row_ptr), _P(col_idx), _P(val),
                                      _P(x), _P(y), int(precision), _P(stream) if stream else None)
    return rc if raw else _check(rc)


def uc_copy_bench(nbytes: int, reps: int = 20, device: int = 0) -> float:
    g = C.c_double()
    _check(load().uc_copy_bench(device, int(nbytes), int(reps), C.byref(g)))
    return g.value


# ---------------------------------------------------------------------------
# convenience: one blocking solve
# ---------------------------------------------------------------------------

def solve(lp, opts: Optional[uc_lp_opts] = None, x0=None, y0=None, timeout_s: float = -1.0):
    """Create, solve, wait, fetch.  Returns (x, y, info dict)."""
    h = uc_lp_create(lp, opts)
    try:
        uc_lp_solve(h, x0, y0)
        uc_lp_wait(h, timeout_s)
        info = uc_lp_status(h)
        x, y = uc_lp_get_solution(h, lp.n, lp.m) if info.status in TERMINAL - {UC_LP_INFEASIBLE, UC_LP_FAILED} \
            else (None, None)
        return x, y, info.as_dict()
    finally:
        uc_lp_destroy(h)
