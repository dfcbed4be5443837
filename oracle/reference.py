"""Oracle: the LP optimum through SciPy's HiGHS interface (a library call).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module.

The simplex in simplex.py keeps a sparse LU of a basis of the full row count
and prices every column each pivot, which is practical up to a few thousand
rows.  For larger instances the optimum of the same relaxation (Sec. II-C)
comes from `scipy.optimize.linprog` with the HiGHS dual simplex or interior
point method; tests pin this call against simplex.py on the small sizes.
"""

from __future__ import annotations

import os
import time

import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog


def highs_solve(lp, method: str = "highs-ipm", time_limit: float = None, disp: bool = False):
    """Return (status, obj, x, y, seconds).  y uses the Lagrangian sign
    convention of kkt.py (y >= 0 on 'G' rows).  disp: HiGHS prints its
    progress log."""
    A = sp.csr_matrix((np.asarray(lp.val, float), np.asarray(lp.col_idx, np.int64),
                       np.asarray(lp.row_ptr, np.int64)), shape=(lp.m, lp.n))
    sense = np.asarray(lp.sense)
    E = np.flatnonzero(sense == ord("E"))
    G = np.flatnonzero(sense == ord("G"))
    L = np.flatnonzero(sense == ord("L"))
    ub_rows = np.concatenate([G, L])
    A_ub = sp.vstack([-A[G], A[L]]).tocsr()
    b_ub = np.concatenate([-np.asarray(lp.b)[G], np.asarray(lp.b)[L]])
    opts = {"presolve": True, "disp": bool(disp)}
    if time_limit is not None:
        opts["time_limit"] = float(time_limit)
    t0 = time.perf_counter()
    res = linprog(np.asarray(lp.c, float), A_ub=A_ub if len(ub_rows) else None,
                  b_ub=b_ub if len(ub_rows) else None,
                  A_eq=A[E] if len(E) else None, b_eq=np.asarray(lp.b)[E] if len(E) else None,
                  bounds=np.c_[lp.lb, lp.ub], method=method, options=opts)
    dt = time.perf_counter() - t0
    y = np.zeros(lp.m)
    if res.status == 0:
        if len(E):
            y[E] = res.eqlin.marginals
        if len(ub_rows):
            mu = res.ineqlin.marginals       # <= 0 for A_ub x <= b_ub in a min problem
            y[G] = -mu[:len(G)]
            y[L] = mu[len(G):]
    return res.status, (float(res.fun) if res.status == 0 else float("nan")), \
        (res.x if res.status == 0 else None), y, dt


def host_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1
