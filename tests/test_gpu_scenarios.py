"""GPU tests of scenario batches: many LPs sharing one matrix, solved with one
read of the matrix per half-step, against the oracle and against their own
single-scenario solves."""

import json
import os
import sys

import numpy as np
import pytest

from oracle.kkt import kkt
from paper_2607_03627_amd import uclp
from paper_2607_03627_amd.instances import make_instance, scenario_data

pytestmark = pytest.mark.gpu
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "objectives.json")))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def stack(lp, seeds):
    data = [scenario_data(lp, s) for s in seeds]
    return [np.stack([d[k] for d in data]) for k in range(4)]


def batch(lp, seeds, **opts):
    c, b, lb, ub = stack(lp, seeds)
    h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(**opts))
    try:
        return uclp.uc_lp_solve_scenarios(h, lp.n, lp.m, c, b, lb, ub)
    finally:
        uclp.uc_lp_destroy(h)


def test_medium_scenarios_match_highs_oracle():
    lp = make_instance("medium", 0)
    seeds = [1, 2, 3, 4]
    say("case medium scenarios", seeds)
    x, y, infos = batch(lp, seeds, precision=uclp.UC_LP_FP32_MIXED_POLISH, eps_polish=1e-8, iter_limit=400000)
    for k, s in enumerate(seeds):
        info = infos[k].as_dict()
        say("  scen", s, info["status_name"], info["iters"], info["rel_kkt"])
        assert info["status"] == uclp.UC_LP_OPTIMAL
        c, b, lb, ub = scenario_data(lp, s)
        sl = lp.with_data(c=c, b=b, lb=lb, ub=ub)
        o = kkt(sl, x[k], y[k])
        assert o.rel_kkt <= 1e-8 * 1.001
        z = GOLDEN[f"medium_scen/0/{s}"]["obj"]
        assert abs(o.pobj - z) <= 1e-6 * abs(z)


def test_batch_equals_single_scenario_bitwise():
    lp = make_instance("tiny", 6)
    seeds = list(range(1, 17))
    say("case tiny 16 scenarios")
    opts = dict(precision=uclp.UC_LP_FP32_MIXED_POLISH, eps_polish=1e-7, iter_limit=200000)
    x, y, infos = batch(lp, seeds, **opts)
    for k in (0, 7, 15):
        xs, ys, i1 = batch(lp, [seeds[k]], **opts)
        assert infos[k].iters == i1[0].iters and infos[k].status == i1[0].status == uclp.UC_LP_OPTIMAL
        assert np.array_equal(x[k], xs[0]) and np.array_equal(y[k], ys[0])
    for k, s in enumerate(seeds):
        c, b, lb, ub = scenario_data(lp, s)
        o = kkt(lp.with_data(c=c, b=b, lb=lb, ub=ub), x[k], y[k])
        assert o.rel_kkt <= 1e-7 * 1.001


def test_fp64_tail_on_compacted_lanes_equals_single_scenario_bitwise():
    # Cold, the sixteen load/cost scenarios of the 6,049-bus LP all hand over
    # to FP64 near the target; most finish within 64 FP64 iterations and a
    # few need about 2,000 more.  Once at most half the lanes still run, the
    # batch continues on arrays that hold only those scenarios.  The lane
    # layout does not enter any scenario's arithmetic, so a scenario of that
    # tail, and one that finished before the compaction, equal the same
    # scenario solved as a batch of one, bit for bit.
    lp = make_instance("large", 0)
    seeds = list(range(1, 17))
    c, b, lb, ub = stack(lp, seeds)
    h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_MIXED, eps_rel=1e-4))
    try:
        say("case large 16 scenarios, cold")
        x, y, infos = uclp.uc_lp_solve_scenarios(h, lp.n, lp.m, c, b, lb, ub)
        fp64 = [i.iters_fp64 for i in infos]
        say("fp64 iterations", fp64)
        assert all(i.status == uclp.UC_LP_OPTIMAL for i in infos)
        tail = [k for k, f in enumerate(fp64) if f > 64]
        early = [k for k, f in enumerate(fp64) if 0 < f <= 64]
        assert tail and early and 2 * len(tail) <= len(seeds)
        for k in (max(tail, key=lambda t: fp64[t]), early[0]):
            say("single", k)
            xs, ys, i1 = uclp.uc_lp_solve_scenarios(h, lp.n, lp.m, c[k:k + 1], b[k:k + 1], lb[k:k + 1],
                                                    ub[k:k + 1])
            assert i1[0].iters == infos[k].iters and i1[0].iters_fp64 == infos[k].iters_fp64
            assert np.array_equal(xs[0], x[k]) and np.array_equal(ys[0], y[k])
    finally:
        uclp.uc_lp_destroy(h)


def test_warm_start_from_nominal_solution():
    lp = make_instance("tiny", 7)
    xn, yn, info = uclp.solve(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP64, eps_rel=1e-8))
    assert info["status"] == uclp.UC_LP_OPTIMAL
    c, b, lb, ub = stack(lp, [1, 2, 3])
    h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_MIXED))
    try:
        cold = uclp.uc_lp_solve_scenarios(h, lp.n, lp.m, c, b, lb, ub)
        warm = uclp.uc_lp_solve_scenarios(h, lp.n, lp.m, c, b, lb, ub, xn, yn)
    finally:
        uclp.uc_lp_destroy(h)
    for k in range(3):
        assert warm[2][k].status == cold[2][k].status == uclp.UC_LP_OPTIMAL
        cc, bb, ll, uu = scenario_data(lp, k + 1)
        assert kkt(lp.with_data(c=cc, b=bb, lb=ll, ub=uu), warm[0][k], warm[1][k]).rel_kkt <= 1e-4
    # the warm start is used: a scenario started at its own FP64 optimum stops
    # at the first check
    lp1 = lp.with_data(c=c[0], b=b[0], lb=lb[0], ub=ub[0])
    x1, y1, i1 = uclp.solve(lp1, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP64, eps_rel=1e-8))
    assert i1["status"] == uclp.UC_LP_OPTIMAL
    h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP64, eps_rel=1e-6))
    try:
        own = uclp.uc_lp_solve_scenarios(h, lp.n, lp.m, c[:1], b[:1], lb[:1], ub[:1], x1, y1)
    finally:
        uclp.uc_lp_destroy(h)
    assert own[2][0].status == uclp.UC_LP_OPTIMAL and own[2][0].iters == 64


def test_scenario_count_limits():
    lp = make_instance("tiny", 0, n_periods=2)
    c, b, lb, ub = stack(lp, range(1, 18))
    h = uclp.uc_lp_create(lp)
    try:
        with pytest.raises(uclp.UcLpError) as e:
            uclp.uc_lp_solve_scenarios(h, lp.n, lp.m, c, b, lb, ub)
        assert e.value.code == uclp.UC_LP_ENOTSUP
    finally:
        uclp.uc_lp_destroy(h)


def test_fp32_phase_compaction_equals_single_scenario_bitwise():
    # Four of eight scenarios are the 500-bus LP itself: warm-started at its
    # FP64 optimum they meet 1e-4 at the first check, in the FP32 phase, and
    # the batch moves the other four (load / cost perturbations) to arrays of
    # their own lanes while the FP32 phase goes on.  With a stall window of
    # one check those four hand over to FP64 near the target, which finishes
    # them.  A lane of each kind equals the same scenario solved as a batch of
    # one, bit for bit.
    lp = make_instance("medium", 0)
    say("case medium 8 scenarios, FP32-phase compaction")
    xn, yn, info = uclp.solve(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP64, eps_rel=1e-8),
                              timeout_s=300)
    assert info["status"] == uclp.UC_LP_OPTIMAL
    cs, bs, ls, us = stack(lp, [1, 2, 3, 4])
    c = np.concatenate([np.tile(lp.c, (4, 1)), cs])
    b = np.concatenate([np.tile(lp.b, (4, 1)), bs])
    lb = np.concatenate([np.tile(lp.lb, (4, 1)), ls])
    ub = np.concatenate([np.tile(lp.ub, (4, 1)), us])
    h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_MIXED, eps_rel=1e-4,
                                                      fp32_stall_checks=1, iter_limit=200000))
    try:
        x, y, infos = uclp.uc_lp_solve_scenarios(h, lp.n, lp.m, c, b, lb, ub, xn, yn)
        say("iters", [i.iters for i in infos], "fp64", [i.iters_fp64 for i in infos])
        assert all(i.status == uclp.UC_LP_OPTIMAL for i in infos)
        early, late = range(4), range(4, 8)
        assert all(infos[k].iters == 64 and infos[k].iters_fp64 == 0 for k in early)
        assert all(infos[k].iters > 64 for k in late)
        assert any(infos[k].iters_fp64 > 0 for k in late)
        for k in (0, max(late, key=lambda t: (infos[t].iters_fp64, infos[t].iters))):
            say("single", k)
            xs, ys, i1 = uclp.uc_lp_solve_scenarios(h, lp.n, lp.m, c[k:k + 1], b[k:k + 1], lb[k:k + 1],
                                                    ub[k:k + 1], xn, yn)
            assert i1[0].iters == infos[k].iters and i1[0].iters_fp64 == infos[k].iters_fp64
            assert np.array_equal(xs[0], x[k]) and np.array_equal(ys[0], y[k])
    finally:
        uclp.uc_lp_destroy(h)
