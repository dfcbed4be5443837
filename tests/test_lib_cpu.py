"""CPU-side checks of the C ABI library: it loads without a GPU, exports
every entry point declared in include/uc_lp.h, and rejects malformed input
before touching any device."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2607_03627_amd import uclp
from paper_2607_03627_amd.instances import LP, make_instance

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "uc_lp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(uc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("uc_lp_create", "uc_lp_solve", "uc_lp_status", "uc_lp_cancel", "uc_lp_get_solution",
                 "uc_lp_destroy", "uc_engine_create", "uc_lp_solve_scenarios"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = uclp.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(declared_functions()) == sorted(uclp.EXPORTS)


def c_layout(struct_name, fields):
    """sizeof and field offsets of a struct of include/uc_lp.h, as the C
    compiler lays it out (gcc on the host)."""
    import shutil
    import subprocess
    import tempfile

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "uc_lp.h"', "int main(void) {",
             f'  printf("%zu\\n", sizeof({struct_name}));']
    lines += [f'  printf("%zu\\n", offsetof({struct_name}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "lay.c"), os.path.join(d, "lay")
        with open(src, "w") as f:
            f.write("\n".join(lines) + "\n")
        subprocess.run([cc, "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    vals = [int(v) for v in out]
    return vals[0], vals[1:]


@pytest.mark.parametrize("name", ["uc_lp_opts", "uc_lp_info"])
def test_binding_struct_layout_equals_the_c_layout(name):
    cls = getattr(uclp, name)
    fields = [f for f, _ in cls._fields_]
    size, offs = c_layout(name, fields)
    assert ctypes.sizeof(cls) == size
    assert [getattr(cls, f).offset for f in fields] == offs


def test_binding_structs_match_header_layout():
    # the two structs are passed by pointer; their sizes must agree with the C layout
    assert ctypes.sizeof(uclp.uc_lp_opts) == 4 * 4 + 8 + 5 * 8 + 4 * 4 + 6 * 8 + 2 * 4 + 4 * 8 + 2 * 8 + 2 * 4 + 2 * 8
    o = uclp.uc_lp_opts_default()
    assert o.eps_gap_rel == 0.0
    assert o.eps_refine == 1e-2 and o.refine_growth == 1e4 and o.refine_max_rounds == 200 and o.reserved2 == 0
    assert o.pw_balance_refine == 0.5 and o.refine_diverge == 0.0
    assert o.precision == uclp.UC_LP_FP32_MIXED_POLISH and o.kkt_every == 64
    assert o.iter_limit == 100000 and o.eps_rel == 1e-4 and o.eps_polish == 1e-8
    assert (o.restart_sufficient, o.restart_necessary, o.restart_artificial, o.pw_smoothing) == \
        (0.2, 0.9, 0.36, 0.8)
    assert o.halpern_gamma == 1.0 and o.pw_max_change == 4.0 and o.fp32_stall_checks == 24 and o.reserved == 0
    assert o.pw_integral == 0.0 and o.pw_balance == 0.5 and o.pw_balance_polish == 0.0


def small():
    lp = make_instance("tiny", 0, n_periods=2)
    return lp


def mutated(**kw):
    lp = small()
    fields = dict(m=lp.m, n=lp.n, row_ptr=lp.row_ptr.copy(), col_idx=lp.col_idx.copy(),
                  val=lp.val.copy(), c=lp.c.copy(), b=lp.b.copy(), sense=lp.sense.copy(),
                  lb=lp.lb.copy(), ub=lp.ub.copy())
    for k, f in kw.items():
        fields[k] = f(fields[k])
    return LP(**fields)


def _set(i, v):
    def f(a):
        a = a.copy()
        a[i] = v
        return a
    return f


@pytest.mark.parametrize("case", [
    dict(row_ptr=_set(0, 1)),
    dict(row_ptr=_set(5, 10**6)),
    dict(col_idx=_set(3, -1)),
    dict(col_idx=lambda a: np.where(np.arange(len(a)) == 1, a[0], a)),   # duplicate in row 0
    dict(val=_set(2, np.nan)),
    dict(c=_set(0, np.inf)),
    dict(b=_set(0, np.nan)),
    dict(lb=_set(0, 5.0), ub=_set(0, 1.0)),
    dict(sense=_set(0, ord("X"))),
    dict(lb=_set(0, np.inf)),
])
def test_create_rejects_malformed_input_without_a_device(case):
    lp = mutated(**case)
    rc, h = uclp.uc_lp_create(lp, raw=True)
    assert rc == uclp.UC_LP_EINVAL and h is None
    assert uclp.uc_lp_last_error() != ""


def test_degenerate_problems_are_refused_before_the_device():
    # every column fixed, or no row left after the minimal presolve: there is
    # no PDHG problem, and the call fails before any device work
    lp = small()
    fixed = mutated(lb=lambda a: np.zeros_like(a), ub=lambda a: np.zeros_like(a))
    rc, h = uclp.uc_lp_create(fixed, raw=True)
    assert rc == uclp.UC_LP_ENOTSUP and h is None
    empty = LP(m=2, n=3, row_ptr=np.zeros(3, np.int32), col_idx=np.zeros(0, np.int32), val=np.zeros(0),
               c=np.array([1.0, -1.0, 0.0]), b=np.zeros(2), sense=np.array([ord("E"), ord("G")], np.uint8),
               lb=np.zeros(3), ub=np.ones(3))
    rc, h = uclp.uc_lp_create(empty, raw=True)
    assert rc == uclp.UC_LP_ENOTSUP and h is None
    assert "row" in uclp.uc_lp_last_error()


def test_bad_options_are_rejected():
    lp = small()
    for kw, code in ((dict(precision=7), uclp.UC_LP_ENOTSUP), (dict(kkt_every=0), uclp.UC_LP_EINVAL),
                     (dict(step_scale=1.5), uclp.UC_LP_EINVAL), (dict(eps_rel=-1.0), uclp.UC_LP_EINVAL),
                     (dict(halpern_gamma=1.5), uclp.UC_LP_EINVAL), (dict(pw_max_change=0.5), uclp.UC_LP_EINVAL),
                     (dict(fp32_stall_checks=-1), uclp.UC_LP_EINVAL), (dict(reserved=1), uclp.UC_LP_EINVAL),
                     (dict(pw_integral=2.0), uclp.UC_LP_EINVAL), (dict(pw_balance=-0.5), uclp.UC_LP_EINVAL),
                     (dict(eps_refine=0.0), uclp.UC_LP_EINVAL), (dict(eps_refine=1.0), uclp.UC_LP_EINVAL),
                     (dict(refine_growth=1.0), uclp.UC_LP_EINVAL), (dict(refine_max_rounds=-1), uclp.UC_LP_EINVAL),
                     (dict(reserved2=3), uclp.UC_LP_EINVAL), (dict(pw_balance_refine=1.5), uclp.UC_LP_EINVAL),
                     (dict(refine_diverge=0.5), uclp.UC_LP_EINVAL), (dict(refine_diverge=float("inf")), uclp.UC_LP_EINVAL)):
        rc, h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(**kw), raw=True)
        assert rc == code and h is None


def test_null_handles_are_safe():
    lib = uclp.load()
    lib.uc_lp_destroy(None)
    lib.uc_engine_destroy(None)
    assert lib.uc_lp_cancel(None) == uclp.UC_LP_EINVAL
    assert lib.uc_lp_status(None, None) == uclp.UC_LP_EINVAL


def test_valid_lps_pass_validation_and_presolve():
    # valid inputs of every column / row kind go through validation, the
    # minimal presolve (fixed columns, empty rows, 'L' rows) and the row-block
    # and tile construction on the host; without a GPU the call then fails at
    # the device, with one it succeeds
    lp = make_instance("tiny", 1, n_periods=3)
    lb, ub = lp.lb.copy(), lp.ub.copy()
    ub[::7] = np.inf
    lb[1::7] = -np.inf
    lb[2::11] = ub[2::11] = np.clip(0.0, lp.lb[2::11], lp.ub[2::11])   # fixed columns
    sense = lp.sense.copy()
    sense[5::9] = ord("L")
    variants = [lp, lp.with_data(lb=lb, ub=ub), LP(m=lp.m, n=lp.n, row_ptr=lp.row_ptr, col_idx=lp.col_idx,
                                                     val=lp.val, c=lp.c, b=-lp.b, sense=sense, lb=lp.lb, ub=lp.ub)]
    for v in variants:
        rc, h = uclp.uc_lp_create(v, raw=True)
        if rc == uclp.UC_LP_OK:
            uclp.uc_lp_destroy(h)
        else:
            assert rc == uclp.UC_LP_EHIP and "device" in uclp.uc_lp_last_error()
