"""Benchmark: time to 1e-4 relative KKT of the 6,049-bus-shaped UC LP relaxation
on one MI355X, with the roofline of the dominant kernel and the CPU oracle.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large]
                    [--no-cpu] [--no-extra] [--no-serving] [--no-scenarios]

One step = one solve through the C ABI (uc_lp_solve .. uc_lp_wait) of the
device-resident instance: device transpose, scaling and power iteration,
then restarted-Halpern PDHG with FP32 iterates and FP64 KKT checks every 64
iterations.  `value` is the solve's own time from its start to the first
check with relative KKT error <= 1e-4 (t_to_eps_s); the solve then goes on
until the FP64 duality gap is <= 1e-7 as well, and the wall time to that
returned point is reported beside it.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import resource
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, public figure

WORKLOADS = {
    "large": ("6049-bus-shaped DC-UC LP relaxation: 6,049 buses, 8,500 branches, 700 units, "
              "48 hourly periods, 3 line-outage copies"),
    "large_kc0": "6049-bus-shaped DC-UC LP relaxation without contingency copies (48 periods)",
    "medium": "500-bus DC-UC LP relaxation, 120 units, 48 half-hour periods",
    "tiny": "30-bus DC-UC LP relaxation, 10 units, 24 hourly periods",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_unit_bytes(rows, cols, nnz, vb=4):
    """Algorithmic bytes of one SpMV over a CSR matrix of `rows` rows: values
    and column indices, row pointers, each gathered element once, the output."""
    return nnz * (vb + 4) + 4 * (rows + 1) + vb * cols + vb * rows


def primal_bytes(n, m, nnz, vb=4):
    # upper bound of the library's figure (no block reads its c, l, u from
    # the flags): A^T values + column indices, row pointers, one read of y per
    # row of A, per column: c, l, u, x, x0 read and x, xbar written
    return nnz * (vb + 4) + 4 * (n + 1) + vb * m + 7 * vb * n


def dual_bytes(n, m, nnz, vb=4):
    # upper bound, as above: A values + column indices, row pointers, one
    # read of xbar per column,
    # per row: b, y, y0 read and y written
    return nnz * (vb + 4) + 4 * (m + 1) + vb * n + 4 * vb * m


# the device code and the launch shape it is compiled for
KERNEL_SOURCES = ("kernels.hip", "uclp_dev.h")


def measured_traffic(kernel="k_primal"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "k_primal_large_traffic.json")
    csrc = os.path.join(ROOT, "paper_2607_03627_amd", "csrc")
    try:
        with open(path) as f:
            rec = json.load(f)
        h = hashlib.sha256()
        for name in KERNEL_SOURCES:
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(f.read())
        digest = h.hexdigest()
    except OSError:
        return None
    if rec.get("kernel_sources_sha256") != digest:
        return None
    return rec.get(kernel, {}).get("traffic_bytes")


def _cpu_baseline_child(workload, seed, time_limit_s, q, kw=None):
    """Child process of cpu_baseline: builds the workload and runs the oracle
    on it, then reports status, wall and CPU seconds of the solve."""
    from oracle.reference import highs_solve
    from paper_2607_03627_amd.instances import make_instance

    lp = make_instance(workload, seed, **(kw or {}))
    q.put(("start", time.perf_counter()))
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    st = highs_solve(lp, "highs-ipm", time_limit=time_limit_s)[0]
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    q.put(("done", int(st), wall, (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)))


def host_threads() -> int:
    """CPU threads this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(lp, workload, seed, time_limit_s=25.0, hard_limit_s=60.0, kw=None):
    """The oracle (HiGHS interior point through oracle/reference.py) on the
    workload itself, in a child process: the measured time if it finishes,
    else a lower bound.  HiGHS checks its own time limit only between
    iterations, so the child is also stopped at a hard wall-clock limit.
    kw: extra arguments of make_instance for the workload."""
    import multiprocessing as mp
    import queue as _queue

    ctx = mp.get_context("spawn")
    q = ctx.Queue()
    ru0 = resource.getrusage(resource.RUSAGE_CHILDREN)
    proc = ctx.Process(target=_cpu_baseline_child, args=(workload, seed, time_limit_s, q, kw), daemon=True)
    proc.start()
    t_start, res = None, None
    t_spawn = time.perf_counter()
    last_log = t_spawn
    while True:
        try:
            msg = q.get(timeout=1.0)
            if msg[0] == "start":
                t_start = time.perf_counter()
            else:
                res = msg
                break
        except _queue.Empty:
            pass
        now = time.perf_counter()
        if now - last_log >= 15.0:
            log(f"[bench] cpu_baseline: oracle running for {now - (t_start or t_spawn):.0f} s")
            last_log = now
        if t_start is not None and now - t_start >= hard_limit_s:
            break
        if not proc.is_alive() and q.empty():
            break
    stopped = res is None
    if stopped and proc.is_alive():
        proc.kill()
    proc.join(30)
    if res is not None:
        st, wall, cpu = res[1], res[2], res[3]
    else:
        st = None
        wall = time.perf_counter() - (t_start or t_spawn)
        ru1 = resource.getrusage(resource.RUSAGE_CHILDREN)
        cpu = (ru1.ru_utime - ru0.ru_utime) + (ru1.ru_stime - ru0.ru_stime)
    done = st == 0
    how = ("finished" if done else
           f"stopped at the {hard_limit_s:.0f} s wall-clock limit, value is a lower bound" if stopped else
           f"status {st}, not finished, value is a lower bound")
    return {
        "value": wall, "unit": "s", "cores": max(1, round(cpu / max(wall, 1e-9))), "kind": "oracle",
        "bound": "measured" if done else "lower",
        "host_cores": host_threads(),
        "sample": (f"HiGHS interior point with crossover (oracle/reference.py) on the workload itself "
                   f"({lp.m} rows, {lp.n} cols, {lp.nnz} nnz), model set-up included, HiGHS time limit "
                   f"{time_limit_s:.0f} s, hard limit {hard_limit_s:.0f} s: {how}; {wall:.1f} s wall, "
                   f"{cpu:.1f} s CPU ({host_threads()} host cores available)"),
    }


# Concurrent instances in the batched serving legs.  The 200 GB budget
# admits all 64 requests at once; capping the engine at 32 resident
# instances gave lower p50 and p99 and at least the same solves per second on
# the refinement stream (seed 0, and the held-out seeds 1 and 2) than 16 or
# 64, since half the stream's matrices and vectors stay in the 256 MB
# Infinity Cache.
SERVING_SLOTS = 32


def serving_leg(seed=0, n_requests=64, eps=1e-8, iter_limit=400000, extra_streams=0, slots=SERVING_SLOTS):
    """Poisson stream of differently sized UC LPs (Exp(50 ms) gaps, 300-2000 buses,
    24 or 48 periods): continuous batching on one engine, FP32 + FP64 polish
    and FP32 + iterative refinement, against plain FP64 PDHG one request at
    a time (FIFO), same tolerance.
    extra_streams > 0 serves that many more streams (seeds 1, 2, ...) batched
    with refinement and pools their latencies with the first refinement
    stream for p50 / p99."""
    from paper_2607_03627_amd import serving, uclp
    from paper_2607_03627_amd.instances import make_instance, serving_stream

    reqs = serving_stream(seed, n_requests)
    lps = [make_instance(r.shape, r.seed) for r in reqs]
    arr = [r.arrival_s for r in reqs]
    out = {"requests": n_requests, "stream_seed": seed, "rel_kkt_target": eps, "slots": slots,
           "rows": [lp.m for lp in lps], "nnz_total": int(sum(lp.nnz for lp in lps))}
    ob = uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_MIXED_POLISH, eps_rel=1e-4, eps_polish=eps,
                                 iter_limit=iter_limit)
    rb = serving.run_stream(lps, arr, ob, max_slots=slots, hbm_budget_bytes=200 << 30,
                            progress=lambda m: log(f"[bench] serving batched: {m}"))
    out["batched_fp32_polish"] = rb.stats
    log(f"[bench] serving batched: {rb.stats}")
    # the same stream, batched, FP32 with iterative refinement to the same target
    orf = uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_REFINE, eps_rel=1e-4, eps_polish=eps,
                                  iter_limit=iter_limit)
    rr = serving.run_stream(lps, arr, orf, max_slots=slots, hbm_budget_bytes=200 << 30,
                            progress=lambda m: log(f"[bench] serving batched refine: {m}"))
    out["batched_fp32_refine"] = rr.stats
    log(f"[bench] serving batched refine: {rr.stats}")
    if extra_streams > 0:
        more = [rr]
        for sd in range(seed + 1, seed + 1 + extra_streams):
            rq = serving_stream(sd, n_requests)
            r = serving.run_stream([make_instance(q.shape, q.seed) for q in rq], [q.arrival_s for q in rq], orf,
                                   max_slots=slots, hbm_budget_bytes=200 << 30,
                                   progress=lambda m: log(f"[bench] serving stream {sd}: {m}"))
            log(f"[bench] serving batched refine stream {sd}: {r.stats}")
            more.append(r)
        out["batched_refine_pooled"] = serving.pooled_latency(more)
        out["batched_refine_pooled"]["streams"] = len(more)
        out["batched_refine_pooled"]["solves_per_s_by_stream"] = [r.stats["solves_per_s"] for r in more]
    of = uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP64, eps_rel=eps, iter_limit=iter_limit)
    rf = serving.run_stream(lps, arr, of, max_slots=1, hbm_budget_bytes=200 << 30,
                            progress=lambda m: log(f"[bench] serving fp64 fifo: {m}"))
    out["fp64_one_at_a_time"] = rf.stats
    log(f"[bench] serving fp64 fifo: {rf.stats}")
    out["throughput_ratio"] = rb.stats["solves_per_s"] / rf.stats["solves_per_s"]
    out["throughput_ratio_refine"] = rr.stats["solves_per_s"] / rf.stats["solves_per_s"]
    out["worst_rel_kkt"] = {"batched": max(s.info["rel_kkt"] for s in rb.served),
                            "batched_refine": max(s.info["rel_kkt"] for s in rr.served),
                            "fp64": max(s.info["rel_kkt"] for s in rf.served)}
    return out


def scenario_leg(base_lp, n_scen=16, full=False):
    """Scenario batch over the shared matrix (load x U[0.85,1.15] per bus, cost
    x U[0.95,1.05] per unit), warm-started from the nominal solution, against
    sequential plain FP64 solves of the same scenarios, all to 1e-4 with the
    duality gap closed to 1e-7.  full=True adds the cold batch and sequential
    single-LP FP32 solves."""
    import numpy as np

    from paper_2607_03627_amd import uclp
    from paper_2607_03627_amd.instances import scenario_data

    data = [scenario_data(base_lp, s) for s in range(1, n_scen + 1)]
    c, b, lb, ub = (np.stack([d[k] for d in data]) for k in range(4))
    out = {"scenarios": n_scen}
    h = uclp.uc_lp_create(base_lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_MIXED, eps_rel=1e-4))
    try:
        t = time.perf_counter()
        uclp.uc_lp_solve(h)
        uclp.uc_lp_wait(h, 600)
        xn, yn = uclp.uc_lp_get_solution(h, base_lp.n, base_lp.m)
        out["nominal_s"] = time.perf_counter() - t
        t = time.perf_counter()
        x, y, infos = uclp.uc_lp_solve_scenarios(h, base_lp.n, base_lp.m, c, b, lb, ub, xn, yn)
        out["batch_warm_s"] = time.perf_counter() - t
        out["batch_iters"] = [i.iters for i in infos]
        out["batch_status"] = [uclp.STATUS_NAMES[i.status] for i in infos]
        out["batch_rel_kkt_max"] = max(i.rel_kkt for i in infos)
        out["batch_iters_fp64"] = [i.iters_fp64 for i in infos]
        out["batch_t_to_eps_s_max"] = max(i.t_to_eps_s for i in infos)
        if full:
            t = time.perf_counter()
            _, _, infos = uclp.uc_lp_solve_scenarios(h, base_lp.n, base_lp.m, c, b, lb, ub)
            out["batch_cold_s"] = time.perf_counter() - t
            out["batch_cold_iters"] = [i.iters for i in infos]
            out["batch_cold_status"] = [uclp.STATUS_NAMES[i.status] for i in infos]
    finally:
        uclp.uc_lp_destroy(h)
    log(f"[bench] scenarios batch: {out}")
    seq = 0.0
    its = []
    for k in range(n_scen):
        lp_k = base_lp.with_data(c=c[k], b=b[k], lb=lb[k], ub=ub[k])
        t = time.perf_counter()
        _, _, info = uclp.solve(lp_k, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP64, eps_rel=1e-4),
                                timeout_s=600)
        seq += info["t_total_s"]
        its.append(info["iters"])
    out["sequential_fp64_cold_s"] = seq
    out["sequential_iters"] = its
    out["speedup_vs_sequential"] = seq / out["batch_warm_s"]
    log(f"[bench] scenarios sequential: {seq:.2f}s")
    if not full:
        return out
    # the same scenarios one at a time on the single-LP FP32 path
    seq32 = 0.0
    its32 = []
    for k in range(n_scen):
        lp_k = base_lp.with_data(c=c[k], b=b[k], lb=lb[k], ub=ub[k])
        _, _, info = uclp.solve(lp_k, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_MIXED, eps_rel=1e-4),
                                timeout_s=600)
        seq32 += info["t_total_s"]
        its32.append(info["iters"])
    out["sequential_fp32_cold_s"] = seq32
    out["sequential_fp32_iters"] = its32
    out["speedup_vs_sequential_fp32"] = seq32 / out["batch_warm_s"]
    out["cold_batch_speedup_vs_sequential_fp32"] = seq32 / out["batch_cold_s"]
    log(f"[bench] scenarios sequential fp32: {seq32:.2f}s")
    return out


def race_leg(large_lp):
    """Algorithm 1 on synthetic UC LPs of several sizes: this library's GPU
    PDHG (FP32, 1e-4) against HiGHS interior point on the host cores, checked
    every 0.5 s; the first to finish wins and the other is stopped."""
    from paper_2607_03627_amd import uclp
    from paper_2607_03627_amd.instances import make_instance
    from paper_2607_03627_amd.race import race

    cases = [("tiny/0", make_instance("tiny", 0)), ("medium/0", make_instance("medium", 0)),
             ("medium/1", make_instance("medium", 1)), ("large_kc0/0", make_instance("large_kc0", 0)),
             ("large/0", large_lp)]
    rows = []
    for name, lp in cases:
        r = race(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_MIXED, eps_rel=1e-4), poll_s=0.5,
                 cpu_method="highs-ipm", timeout_s=600)
        rows.append({"case": name, "rows": lp.m, "winner": r.winner, "seconds": round(r.seconds, 3),
                     "polls": r.polls,
                     "legs": {x.name: {"status": x.status, "seconds": round(x.seconds, 3),
                                       "solve_s": x.info.get("t_total_s", x.info.get("highs_seconds"))}
                              for x in r.results}})
        log(f"[bench] race {name}: {rows[-1]}")
    wins = {}
    for row in rows:
        wins[row["winner"]] = wins.get(row["winner"], 0) + 1
    return {"poll_s": 0.5, "cases": rows, "wins": wins}


def size_sweep_leg(time_limit_s=45.0):
    """GPU PDHG against the CPU oracle leg across problem sizes: where does the
    GPU stop paying off?  Each LP is solved by the library (FP32 to 1e-4, and
    FP32 + FP64 polish to 1e-8) and by HiGHS interior point with crossover on
    the host cores (stopped at a time limit)."""
    from paper_2607_03627_amd import uclp
    from paper_2607_03627_amd.instances import make_instance

    cases = [("tiny", 0, {}), ("medium", 0, {"n_periods": 12}), ("medium", 0, {}), ("large_kc0", 0, {}),
             ("large", 0, {})]
    rows = []
    for shape, seed, kw in cases:
        lp = make_instance(shape, seed, **kw)
        r = {"case": f"{shape}/{seed}" + ("" if not kw else f" {kw}"), "rows": lp.m, "cols": lp.n, "nnz": lp.nnz}
        for label, o in (("gpu_fp32_1e-4", dict(precision=uclp.UC_LP_FP32_MIXED, eps_rel=1e-4)),
                         ("gpu_polish_1e-8", dict(precision=uclp.UC_LP_FP32_MIXED_POLISH, eps_rel=1e-4,
                                                  eps_polish=1e-8))):
            t = time.perf_counter()
            _, _, info = uclp.solve(lp, uclp.uc_lp_opts_default(**o), timeout_s=600)
            r[label] = {"create_to_done_s": time.perf_counter() - t, "solve_s": info["t_total_s"],
                        "status": info["status_name"], "iters": info["iters"], "pobj": info["pobj"]}
        cb = cpu_baseline(lp, shape, seed, time_limit_s=time_limit_s, hard_limit_s=time_limit_s + 30.0, kw=kw)
        r["cpu_highs_ipm"] = {"s": cb["value"], "finished": cb["bound"] == "measured", "cores": cb["cores"],
                              "host_cores": host_threads()}
        log(f"[bench] size sweep {r}")
        rows.append(r)
    return {"time_limit_s": time_limit_s, "cases": rows}


def dual_form_leg():
    """The same library on the LP and on its dual (paper_2607_03627_amd/
    dual_form.py): time, iterations and objective of each form."""
    from paper_2607_03627_amd import uclp
    from paper_2607_03627_amd.dual_form import dual_form
    from paper_2607_03627_amd.instances import make_instance

    rows = []
    for shape, seed in (("medium", 0), ("large_kc0", 0)):
        lp = make_instance(shape, seed)
        df = dual_form(lp)
        r = {"case": f"{shape}/{seed}", "primal_size": [lp.m, lp.n, lp.nnz],
             "dual_size": [df.lp.m, df.lp.n, df.lp.nnz], "oracle_obj": golden_objective(f"{shape}/{seed}")}
        for form, L, sgn in (("primal", lp, 1.0), ("dual", df.lp, -1.0)):
            for label, o in (("fp32_1e-4", dict(precision=uclp.UC_LP_FP32_MIXED, eps_rel=1e-4)),
                             ("polish_1e-8", dict(precision=uclp.UC_LP_FP32_MIXED_POLISH, eps_rel=1e-4,
                                                  eps_polish=1e-8))):
                _, _, info = uclp.solve(L, uclp.uc_lp_opts_default(**o), timeout_s=600)
                r[f"{form}_{label}"] = {"solve_s": info["t_total_s"], "t_to_1e-4_s": info["t_to_eps_s"],
                                        "status": info["status_name"], "iters": info["iters"],
                                        "objective": sgn * info["pobj"]}
        log(f"[bench] dual form {r}")
        rows.append(r)
    return {"cases": rows}


def golden_objective(key):
    """The oracle's optimum of a seeded instance as stored by
    tests/golden/make_golden.py (None when not stored)."""
    try:
        with open(os.path.join(ROOT, "tests", "golden", "objectives.json")) as f:
            return json.load(f).get(key, {}).get("obj")
    except OSError:
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--iter-limit", type=int, default=100000,
                    help="iteration limit of each solve (short runs for hardware counters)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream leg")
    ap.add_argument("--no-scenarios", action="store_true", help="skip the 16-scenario batch leg")
    ap.add_argument("--scenarios-full", action="store_true",
                    help="scenario leg with the cold batch and sequential FP32 solves")
    ap.add_argument("--no-race", action="store_true", help="skip the GPU-CPU race on five LPs")
    ap.add_argument("--size-sweep", action="store_true", help="GPU vs CPU oracle across problem sizes")
    ap.add_argument("--dual-form", action="store_true", help="the LP and its dual on the same library")
    ap.add_argument("--serving-streams", type=int, default=5,
                    help="batched refinement serving over this many request streams (latencies pooled for "
                         "p50 / p99; 5 streams = 320 requests)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    from paper_2607_03627_amd import uclp
    from paper_2607_03627_amd.instances import make_instance

    uclp.load()
    t0 = time.time()
    lp = make_instance(args.workload, args.seed)
    log(f"[bench] instance {args.workload}/{args.seed}: m={lp.m} n={lp.n} nnz={lp.nnz} ({time.time() - t0:.1f}s)")

    def run(h, n_steps, label):
        walls, infos = [], []
        for i in range(n_steps):
            t = time.perf_counter()
            uclp.uc_lp_solve(h)
            uclp.uc_lp_wait(h, 1200)
            walls.append(time.perf_counter() - t)
            info = uclp.uc_lp_status(h).as_dict()
            infos.append(info)
            log(f"[bench] {label} step {i}: {walls[-1]:.3f}s status {info['status_name']} iters {info['iters']} "
                f"restarts {info['restarts']} t_eps {info['t_to_eps_s']:.3f}s (iters {info['iters_at_eps']}) "
                f"setup {info['t_setup_s']:.3f}s kkt {info['rel_kkt']:.2e} gap {info['rel_gap']:.2e} "
                f"pobj {info['pobj']:.10g} at_eps {info['pobj_at_eps']:.10g} primal_us {info['primal_kernel_us']:.1f} "
                f"dual_us {info['dual_kernel_us']:.1f} iters_fp64 {info['iters_fp64']}")
        return walls, infos

    opts = uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_MIXED, eps_rel=1e-4, timing=1,
                                   iter_limit=args.iter_limit)
    t0 = time.time()
    h = uclp.uc_lp_create(lp, opts)
    log(f"[bench] create+upload {time.time() - t0:.2f}s")
    try:
        run(h, args.warmup, "warmup")
        walls, infos = run(h, args.steps, "timed")
    finally:
        uclp.uc_lp_destroy(h)
    ok = all(i["status"] == uclp.UC_LP_OPTIMAL and i["t_to_eps_s"] > 0 for i in infos) or args.iter_limit < 100000
    value = statistics.median(i["t_to_eps_s"] for i in infos)
    last = infos[-1]
    n_i, m_i, z_i = last["n_presolved"], last["m_presolved"], last["nnz_presolved"]
    pb = last["primal_bytes"]
    db = last["dual_bytes"]
    assert pb <= primal_bytes(n_i, m_i, z_i) and db <= dual_bytes(n_i, m_i, z_i)
    p_us = statistics.median(i["primal_kernel_us"] for i in infos)
    d_us = statistics.median(i["dual_kernel_us"] for i in infos)
    # the primal half-step is an SpMV over A^T (n rows gathering the m-vector y)
    pu = spmv_unit_bytes(n_i, m_i, z_i)
    du = spmv_unit_bytes(m_i, n_i, z_i)
    achieved = pu / (p_us * 1e-6) / 1e9 if p_us > 0 else None
    zstar = golden_objective(f"{args.workload}/{args.seed}")
    out = {
        "metric": "time-to-1e-4 rel KKT (s) on 6049-bus UC LP",
        "value": value if ok else None,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * value,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "shape": args.workload, "seed": args.seed,
                   "rows": lp.m, "cols": lp.n, "nnz": lp.nnz, "precision": "FP32 iterates, FP64 KKT/restart/gap",
                   "eps_rel": 1e-4, "eps_gap_rel": opts.eps_gap_rel, "kkt_every": 64,
                   "value_is": "solve start -> first check at rel. KKT <= 1e-4 (library clock), where the "
                               "solve ends; extra.wall_s_returned is the host wall time to the returned point",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": "k_primal<float> (A^T SpMV + projection + Halpern)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": measured_traffic("k_primal") if args.workload == "large" else None,
                     "bytes_per_launch": pu, "bytes_unit": "one SpMV of A^T: 8 nnz + 4 (n+1) + 4 m + 4 n",
                     "us_per_launch": p_us,
                     "impl_bytes_per_launch": pb,
                     "achieved_impl": pb / (p_us * 1e-6) / 1e9 if p_us > 0 else None,
                     "frac_impl": pb / (p_us * 1e-6) / 1e9 / HBM_PEAK_GBS if p_us > 0 else None},
        "extra": {
            "status": [i["status_name"] for i in infos], "iters": [i["iters"] for i in infos],
            "iters_at_eps": [i["iters_at_eps"] for i in infos],
            "restarts": [i["restarts"] for i in infos], "t_to_eps_s": [i["t_to_eps_s"] for i in infos],
            "wall_s_returned": walls, "t_setup_s": [i["t_setup_s"] for i in infos],
            "rel_kkt": [i["rel_kkt"] for i in infos], "rel_gap": [i["rel_gap"] for i in infos],
            "rel_gap_at_eps": [i["rel_gap_at_eps"] for i in infos],
            "pobj": [i["pobj"] for i in infos], "pobj_at_eps": [i["pobj_at_eps"] for i in infos],
            "oracle_obj": zstar,
            "obj_err_at_eps_vs_oracle": (abs(last["pobj_at_eps"] - zstar) / abs(zstar)) if zstar else None,
            "obj_err_returned_vs_oracle": (abs(last["pobj"] - zstar) / abs(zstar)) if zstar else None,
            "norm_a_est": last["norm_a_est"], "norm_a_bound": last["norm_a_bound"], "eta": last["eta"],
            "dual_kernel": {"bytes_per_launch": du, "us_per_launch": d_us,
                            "achieved_gbs": du / (d_us * 1e-6) / 1e9 if d_us > 0 else None,
                            "impl_bytes_per_launch": db,
                            "achieved_impl_gbs": db / (d_us * 1e-6) / 1e9 if d_us > 0 else None},
            "us_per_iter": 1e6 * statistics.median(i["t_to_eps_s"] - i["t_setup_s"] for i in infos) /
                           max(1, statistics.median(i["iters_at_eps"] for i in infos)),
            "context": ("paper (A800 + Xeon W9-3495X, Gurobi 13.0.1 beta, end-to-end MILP): max runtime "
                        "42.12 -> 5.77 min, average speed-up 2.14-5.61x over 45 GO Challenge 3 cases"),
        },
    }
    if not args.no_extra:
        ex = out["extra"]
        try:
            ex["copy_gbs"] = uclp.uc_copy_bench(1 << 30, 20)
            out["roofline"]["frac_of_copy"] = achieved / ex["copy_gbs"] if achieved else None
            # the production half-step kernels over 4 rotating device copies of
            # the instance (working set > the 256 MB Infinity Cache)
            h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_MIXED))
            try:
                hs = uclp.uc_lp_bench_half_steps(h, uclp.UC_LP_FP32_MIXED, copies=4, reps=64)
            finally:
                uclp.uc_lp_destroy(h)
            hs["copies"] = 4
            hs["primal_gbs"] = pu / (hs["primal_us"] * 1e-6) / 1e9
            hs["dual_gbs"] = du / (hs["dual_us"] * 1e-6) / 1e9
            hs["primal_impl_gbs"] = hs["primal_bytes"] / (hs["primal_us"] * 1e-6) / 1e9
            hs["dual_impl_gbs"] = hs["dual_bytes"] / (hs["dual_us"] * 1e-6) / 1e9
            ex["spmv_hbm_4copies"] = hs
            out["roofline"]["spmv_hbm_gbs_4copies"] = hs["primal_gbs"]
            A = lp
            sb = spmv_unit_bytes(A.m, A.n, A.nnz)
            # 4 rotating copies defeat the Infinity Cache; 1 copy is the matrix
            # resident as in a solve, which keeps multiplying the same matrix
            for algo, name in ((uclp.UC_LP_SPMV_ROWSPLIT, "rowsplit"), (uclp.UC_LP_SPMV_MERGEPATH, "mergepath")):
                for copies, tag in ((4, ""), (1, "_1copy")):
                    us = uclp.uc_spmv_bench(A.m, A.n, A.row_ptr, A.col_idx, A.val, uclp.UC_LP_FP32_MIXED, algo,
                                            copies=copies, reps=40)
                    ex[f"spmv_{name}_fp32{tag}"] = {"us": us, "gbs": sb / (us * 1e-6) / 1e9, "bytes": sb,
                                                   "copies": copies}
        except Exception as e:  # extras never hide the main line
            ex["extra_error_bandwidth"] = repr(e)
        try:
            # plain FP64 PDHG to the same targets on the same instance
            h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP64, eps_rel=1e-4, timing=1))
            try:
                w64, i64 = run(h, 1, "fp64")
            finally:
                uclp.uc_lp_destroy(h)
            ex["fp64_plain"] = {"wall_s": w64[0], "t_to_eps_s": i64[0]["t_to_eps_s"], "iters": i64[0]["iters"],
                                "iters_at_eps": i64[0]["iters_at_eps"], "status": i64[0]["status_name"],
                                "pobj": i64[0]["pobj"], "primal_us": i64[0]["primal_kernel_us"],
                                "dual_us": i64[0]["dual_kernel_us"],
                                "obj_err_vs_oracle": abs(i64[0]["pobj"] - zstar) / abs(zstar) if zstar else None}
            # FP32 to 1e-4, then FP64 to 5e-6: the returned point whose objective
            # matches the oracle's optimum within 1e-6
            h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_MIXED_POLISH,
                                                               eps_rel=1e-4, eps_polish=5e-6))
            try:
                wq, iq = run(h, 1, "polish5e-6")
            finally:
                uclp.uc_lp_destroy(h)
            ex["returned_point_polish_5e-6"] = {
                "wall_s": wq[0], "t_to_1e-4_s": iq[0]["t_to_eps_s"], "solve_s": iq[0]["t_total_s"],
                "iters": iq[0]["iters"], "iters_fp64": iq[0]["iters_fp64"], "status": iq[0]["status_name"],
                "rel_kkt": iq[0]["rel_kkt"], "pobj": iq[0]["pobj"],
                "obj_err_vs_oracle": abs(iq[0]["pobj"] - zstar) / abs(zstar) if zstar else None}
            # FP32 + FP64 polish to 1e-8
            h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_MIXED_POLISH,
                                                               eps_rel=1e-4, eps_polish=1e-8))
            try:
                wp, ip_ = run(h, 1, "polish")
            finally:
                uclp.uc_lp_destroy(h)
            ex["fp32_polish_1e-8"] = {"wall_s": wp[0], "iters": ip_[0]["iters"], "iters_fp64": ip_[0]["iters_fp64"],
                                      "status": ip_[0]["status_name"], "pobj": ip_[0]["pobj"],
                                      "rel_kkt": ip_[0]["rel_kkt"],
                                      "obj_err_vs_oracle": abs(ip_[0]["pobj"] - zstar) / abs(zstar) if zstar else None}
            # FP32 to 1e-4, then iterative refinement with FP32 inner solves to 1e-8
            h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_REFINE,
                                                               eps_rel=1e-4, eps_polish=1e-8))
            try:
                wr, ir = run(h, 1, "refine")
            finally:
                uclp.uc_lp_destroy(h)
            ex["fp32_refine_1e-8"] = {"wall_s": wr[0], "solve_s": ir[0]["t_total_s"], "t_to_1e-4_s": ir[0]["t_to_eps_s"],
                                      "iters": ir[0]["iters"], "rounds": ir[0]["refine_rounds"],
                                      "status": ir[0]["status_name"], "pobj": ir[0]["pobj"],
                                      "rel_kkt": ir[0]["rel_kkt"],
                                      "obj_err_vs_oracle": abs(ir[0]["pobj"] - zstar) / abs(zstar) if zstar else None}
        except Exception as e:
            ex["extra_error_modes"] = repr(e)
        if args.workload == "large" and args.seed == 0:
            # seeds the default parameters were not chosen on
            held = []
            try:
                for sd in (1, 2, 3, 4):
                    lp_s = make_instance("large", sd)
                    h = uclp.uc_lp_create(lp_s, opts)
                    try:
                        _, inf_s = run(h, 1, f"seed{sd}")
                    finally:
                        uclp.uc_lp_destroy(h)
                    held.append({"seed": sd, "t_to_eps_s": inf_s[0]["t_to_eps_s"], "iters_at_eps": inf_s[0]["iters_at_eps"],
                                 "iters": inf_s[0]["iters"], "status": inf_s[0]["status_name"],
                                 "t_total_s": inf_s[0]["t_total_s"]})
                    del lp_s
            except Exception as e:
                held.append({"error": repr(e)})
            ex["heldout_seeds"] = held
    if not args.no_serving:
        try:
            out["serving"] = serving_leg(extra_streams=max(0, args.serving_streams - 1))
        except Exception as e:
            out["serving"] = {"error": repr(e)}
    if not args.no_scenarios and args.workload == "large":
        try:
            out["scenarios"] = scenario_leg(lp, full=args.scenarios_full)
        except Exception as e:
            out["scenarios"] = {"error": repr(e)}
    if args.size_sweep:
        try:
            out["size_sweep"] = size_sweep_leg()
        except Exception as e:
            out["size_sweep"] = {"error": repr(e)}
    if args.dual_form:
        try:
            out["dual_form"] = dual_form_leg()
        except Exception as e:
            out["dual_form"] = {"error": repr(e)}
    if not args.no_race:
        try:
            out["race"] = race_leg(lp)
        except Exception as e:
            out["race"] = {"error": repr(e)}
    if not args.no_cpu:
        try:
            out["cpu_baseline"] = cpu_baseline(lp, args.workload, args.seed)
        except Exception as e:
            out["cpu_baseline"] = {"value": None, "error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
