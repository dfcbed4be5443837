"""GPU tests of the multi-instance engine: continuous batching, HBM-budget
admission, cancellation, and the identity of each result alone and in a mix."""

import sys
import time

import numpy as np
import pytest

from oracle.kkt import kkt
from paper_2607_03627_amd import serving, uclp
from paper_2607_03627_amd.instances import UCShape, make_instance

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def requests(n, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nb = int(rng.integers(60, 160))
        T = 24 if i % 2 == 0 else 12
        shape = UCShape(f"r{i}", nb, int(0.4 * (nb - 1)), max(3, int(round(0.12 * nb))), T, 1.0)
        out.append(make_instance(shape, 1000 + i))
    return out


OPTS = dict(precision=uclp.UC_LP_FP32_MIXED_POLISH, eps_rel=1e-4, eps_polish=1e-7, iter_limit=200000)


def test_alone_and_in_mix_are_bitwise_identical():
    lps = requests(5)
    opts = uclp.uc_lp_opts_default(**OPTS)
    alone = []
    for i, lp in enumerate(lps):
        say("alone", i, lp.m, lp.n)
        r = serving.run_stream([lp], [0.0], opts, max_slots=8, keep_solutions=True)
        alone.append(r.served[0])
    say("mix")
    mix = serving.run_stream(lps, [0.0, 0.002, 0.004, 0.03, 0.06], opts, max_slots=8, keep_solutions=True)
    for a, b, lp in zip(alone, mix.served, lps):
        assert a.info["status"] == uclp.UC_LP_OPTIMAL and b.info["status"] == uclp.UC_LP_OPTIMAL
        assert a.info["iters"] == b.info["iters"] and a.info["restarts"] == b.info["restarts"]
        assert np.array_equal(a.x, b.x) and np.array_equal(a.y, b.y)
        k = kkt(lp, b.x, b.y)
        assert k.rel_kkt <= 1e-7 * 1.001


def test_both_half_step_shapes_give_identical_iterates():
    # Alone, a 500-bus LP's half-steps are launches of a few hundred tiles and
    # run one row per thread in 512-thread workgroups; beside the
    # contingency-free 6,049-bus LP each launch holds over a thousand tiles
    # and runs two rows per thread in 256-thread workgroups.  Each row's sum
    # keeps CSR order in both shapes, so the iterates agree bit for bit.
    few_tiles = 1024
    small = make_instance("medium", 3)
    big = make_instance("large_kc0", 3)
    small_tiles_max = (small.m + small.n) // 512 + len(small.val) // 2048 + 2
    assert small_tiles_max < few_tiles
    assert min(big.m, big.n) // 512 >= few_tiles
    opts = uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_MIXED, eps_rel=1e-4)
    say("alone", small.m, small.n)
    a = serving.run_stream([small], [0.0], opts, max_slots=4, keep_solutions=True).served[0]
    say("beside", big.m, big.n)
    r = serving.run_stream([small, big], [0.0, 0.0], opts, max_slots=4, keep_solutions=True)
    b = r.served[0]
    say("iters", a.info["iters"], b.info["iters"], r.served[1].info["iters"])
    assert a.info["status"] == uclp.UC_LP_OPTIMAL and b.info["status"] == uclp.UC_LP_OPTIMAL
    assert r.served[1].info["status"] == uclp.UC_LP_OPTIMAL
    assert a.info["iters"] == b.info["iters"] and a.info["restarts"] == b.info["restarts"]
    assert np.array_equal(a.x, b.x) and np.array_equal(a.y, b.y)


def test_budget_admission_and_fifo():
    lps = requests(6, seed=1)
    need = []
    for lp in lps:
        h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(**OPTS))
        need.append(uclp.uc_lp_status(h).device_bytes)
        uclp.uc_lp_destroy(h)
    # a budget that holds about two of the largest requests
    budget = int(2.3 * max(need))
    opts = uclp.uc_lp_opts_default(**OPTS)
    r = serving.run_stream(lps, [0.0] * len(lps), opts, max_slots=16, hbm_budget_bytes=budget)
    spans = []
    for s in r.served:
        assert s.info["status"] == uclp.UC_LP_OPTIMAL
        start = s.submit_s + s.info["t_queue_s"]
        spans.append((start, start + s.info["t_total_s"], s.info["device_bytes"]))
    # at every admission instant the resident bytes stay within the budget
    for t0, _, _ in spans:
        resident = sum(b for (a, e, b) in spans if a <= t0 + 1e-9 and e > t0)
        assert resident <= budget
    assert max(s.info["t_queue_s"] for s in r.served) > 0


def test_budget_too_small_is_rejected():
    lp = requests(1)[0]
    eng = uclp.uc_engine_create(0, 1 << 16, 4)
    try:
        rc, h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(), engine=eng, raw=True)
        assert rc == uclp.UC_LP_EBUDGET and h is None
    finally:
        uclp.uc_engine_destroy(eng)


def test_cancel_one_request_in_a_batch():
    lps = requests(3, seed=2)
    eng = uclp.uc_engine_create(0, 0, 8)
    hs = []
    try:
        # a tolerance below the FP64 rounding floor of the KKT error is never met
        slow = uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP64, eps_rel=1e-30, iter_limit=10 ** 8,
                                       time_limit_s=120)
        fast = uclp.uc_lp_opts_default(**OPTS)
        for i, lp in enumerate(lps):
            h = uclp.uc_lp_create(lp, slow if i == 1 else fast, engine=eng)
            uclp.uc_lp_solve(h)
            hs.append(h)
        time.sleep(0.2)
        uclp.uc_lp_cancel(hs[1])
        for h in hs:
            assert uclp.uc_lp_wait(h, 120)
        st = [uclp.uc_lp_status(h).status for h in hs]
        assert st == [uclp.UC_LP_OPTIMAL, uclp.UC_LP_CANCELLED, uclp.UC_LP_OPTIMAL]
    finally:
        for h in hs:
            uclp.uc_lp_destroy(h)
        uclp.uc_engine_destroy(eng)


def test_stream_statistics():
    lps = requests(8, seed=3)
    arr = list(np.cumsum(np.random.default_rng(5).exponential(0.01, 8)) - 0.0)
    r = serving.run_stream(lps, arr, uclp.uc_lp_opts_default(**OPTS), max_slots=64)
    st = r.stats
    assert st["n"] == 8 and st["statuses"] == {"OPTIMAL": 8}
    assert 0 < st["p50_s"] <= st["p99_s"] <= st["max_s"]
    assert st["solves_per_s"] > 0
