"""Concurrent GPU–CPU race (the paper's Algorithm 1) over the C ABI.

Algorithm 1 runs two solvers on the same LP at once, checks both on a fixed
interval (0.5 s in the paper), returns the first that finishes and terminates
the other.  Here:

- the GPU leg is this library's restarted-PDHG solve (`uc_lp_solve` is
  asynchronous, `uc_lp_status` polls it, `uc_lp_cancel` terminates it);
- the CPU leg is an interior-point solve of the same LP by HiGHS through
  SciPy, in a child process started before the GPU handle exists, so that it
  can be terminated at once.  It stands in for the paper's CPU barrier leg.

The race is a driver on top of the library: it never feeds a result of one
leg into the other, and the library's own entry points never call the CPU
leg.
"""

from __future__ import annotations

import multiprocessing as mp
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import uclp


@dataclass
class LegResult:
    name: str
    finished: bool
    seconds: float
    status: str
    obj: Optional[float] = None
    x: Optional[np.ndarray] = None
    y: Optional[np.ndarray] = None
    info: dict = field(default_factory=dict)


class Leg:
    """One solver of the race: start(), poll() -> LegResult | None, stop()."""

    name = "leg"

    def start(self) -> None:
        raise NotImplementedError

    def poll(self) -> Optional[LegResult]:
        raise NotImplementedError

    def stop(self) -> None:
        raise NotImplementedError


class GpuLeg(Leg):
    name = "gpu-pdhg"

    def __init__(self, lp, opts: Optional[uclp.uc_lp_opts] = None):
        self.lp = lp
        self.h = uclp.uc_lp_create(lp, opts)  # validated, presolved and uploaded here
        self.t0 = None

    def start(self):
        self.t0 = time.perf_counter()
        uclp.uc_lp_solve(self.h)

    def poll(self):
        info = uclp.uc_lp_status(self.h)
        if info.status not in uclp.TERMINAL:
            return None
        d = info.as_dict()
        ok = info.status == uclp.UC_LP_OPTIMAL
        x = y = None
        if info.status not in (uclp.UC_LP_INFEASIBLE, uclp.UC_LP_FAILED):
            x, y = uclp.uc_lp_get_solution(self.h, self.lp.n, self.lp.m)
        return LegResult(self.name, ok, time.perf_counter() - self.t0, d["status_name"], d["pobj"], x, y, d)

    def stop(self):
        uclp.uc_lp_cancel(self.h)
        uclp.uc_lp_wait(self.h, 60)

    def close(self):
        uclp.uc_lp_destroy(self.h)
        self.h = None


def _cpu_child(conn, method, time_limit):
    """Child process: receive the LP arrays, solve with HiGHS, send the result."""
    import scipy.sparse as sp
    from scipy.optimize import linprog

    msg = conn.recv()
    if msg is None:
        return
    A = sp.csr_matrix((msg["val"], msg["col_idx"], msg["row_ptr"]), shape=(msg["m"], msg["n"]))
    sense = msg["sense"]
    E = np.flatnonzero(sense == ord("E"))
    G = np.flatnonzero(sense == ord("G"))
    Lr = np.flatnonzero(sense == ord("L"))
    A_ub = sp.vstack([-A[G], A[Lr]]).tocsr()
    b_ub = np.concatenate([-msg["b"][G], msg["b"][Lr]])
    conn.send(("go", time.perf_counter()))
    t0 = time.perf_counter()
    res = linprog(msg["c"], A_ub=A_ub if A_ub.shape[0] else None, b_ub=b_ub if A_ub.shape[0] else None,
                  A_eq=A[E] if len(E) else None, b_eq=msg["b"][E] if len(E) else None,
                  bounds=np.c_[msg["lb"], msg["ub"]], method=method,
                  options={"time_limit": float(time_limit)})
    dt = time.perf_counter() - t0
    y = np.zeros(msg["m"])
    if res.status == 0:
        if len(E):
            y[E] = res.eqlin.marginals
        ub_rows = np.concatenate([G, Lr])
        if len(ub_rows):
            mu = res.ineqlin.marginals
            y[G] = -mu[:len(G)]
            y[Lr] = mu[len(G):]
    conn.send(("done", res.status, float(res.fun) if res.status == 0 else None,
               res.x if res.status == 0 else None, y, dt))


class CpuLeg(Leg):
    name = "cpu-highs-ipm"

    def __init__(self, lp, method: str = "highs-ipm", time_limit: float = 3600.0):
        self.lp = lp
        ctx = mp.get_context("spawn")
        self.conn, child = ctx.Pipe()
        self.proc = ctx.Process(target=_cpu_child, args=(child, method, time_limit), daemon=True)
        self.proc.start()
        self.t0 = None

    def start(self):
        lp = self.lp
        self.conn.send(dict(m=int(lp.m), n=int(lp.n), row_ptr=np.asarray(lp.row_ptr), col_idx=np.asarray(lp.col_idx),
                            val=np.asarray(lp.val), c=np.asarray(lp.c), b=np.asarray(lp.b),
                            sense=np.asarray(lp.sense), lb=np.asarray(lp.lb), ub=np.asarray(lp.ub)))
        self.t0 = time.perf_counter()
        self.conn.recv()  # the child has its matrices and starts now

    def poll(self):
        if not self.conn.poll():
            if not self.proc.is_alive():
                return LegResult(self.name, False, time.perf_counter() - self.t0, "DIED")
            return None
        msg = self.conn.recv()
        _, status, obj, x, y, dt = msg
        return LegResult(self.name, status == 0, time.perf_counter() - self.t0,
                         "OPTIMAL" if status == 0 else f"HIGHS_STATUS_{status}", obj, x, y, {"highs_seconds": dt})

    def stop(self):
        if self.proc.is_alive():
            self.proc.terminate()
        self.proc.join(10)

    def close(self):
        self.stop()


@dataclass
class RaceResult:
    winner: Optional[str]
    seconds: float
    polls: int
    results: List[LegResult]


def run_race(legs: List[Leg], poll_s: float = 0.5, timeout_s: float = 3600.0) -> RaceResult:
    """Start every leg, check them every poll_s seconds, return the first that
    finished with a solution and stop the others (Algorithm 1)."""
    for leg in legs:
        leg.start()
    t0 = time.perf_counter()
    polls = 0
    done: dict = {}
    winner = None
    while winner is None:
        time.sleep(poll_s)
        polls += 1
        for i, leg in enumerate(legs):
            if i in done:
                continue
            r = leg.poll()
            if r is not None:
                done[i] = r
                if r.finished and winner is None:
                    winner = i
        if len(done) == len(legs) or time.perf_counter() - t0 > timeout_s:
            break
    for i, leg in enumerate(legs):
        if i not in done:
            leg.stop()
            done[i] = LegResult(leg.name, False, time.perf_counter() - t0, "TERMINATED")
    return RaceResult(legs[winner].name if winner is not None else None, time.perf_counter() - t0, polls,
                      [done[i] for i in range(len(legs))])


def race(lp, opts: Optional[uclp.uc_lp_opts] = None, poll_s: float = 0.5, cpu_method: str = "highs-ipm",
         timeout_s: float = 3600.0) -> RaceResult:
    """Race this library's GPU PDHG against HiGHS on the CPU for one LP."""
    cpu = CpuLeg(lp, cpu_method, timeout_s)  # started before the GPU is touched
    gpu = GpuLeg(lp, opts)
    try:
        return run_race([gpu, cpu], poll_s, timeout_s)
    finally:
        gpu.close()
        cpu.close()
