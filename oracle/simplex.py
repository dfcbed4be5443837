"""Oracle: the LP optimum by a plain two-phase bounded revised primal simplex (FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module.

What it computes is the plain definition of the result the GPU path
approximates: the optimum of the continuous relaxation that both legs of the
paper's concurrent solver solve (Sec. II-C; Sec. III-C says PDHG replaces the
barrier solve of that same relaxation),

    z* = min { c'x : a_i'x = b_i (E rows), a_i'x >= b_i (G rows),
                     a_i'x <= b_i (L rows), lb <= x <= ub },

together with one optimal primal-dual pair (x*, y*).  The sign convention of
y is that of the Lagrangian c'x - y'(Ax - b): y_i >= 0 on G rows, y_i <= 0 on
L rows, free on E rows.

Method (textbook bounded-variable simplex, e.g. Chvatal, "Linear Programming",
ch. 8, and Bixby's description of the revised method):
  * one surplus column per G row (a'x - s = b, s >= 0) and one slack column
    per L row (a'x + s = b, s >= 0), so all rows become equalities;
  * every non-basic column sits at a finite bound, or at 0 if it is free;
  * phase 1: one artificial column per row, signed so its start value is
    non-negative, and the sum of artificials is minimised;
  * phase 2: artificials are frozen at 0 and c'x is minimised;
  * pricing: Dantzig's most violating reduced cost; after a run of
    degenerate pivots, Bland's smallest-index rule until progress resumes;
  * ratio test: bounded, including the entering column's own bound flip;
  * linear algebra: a sparse LU of the basis from SciPy (a library
    primitive), refactored every `refactor_every` pivots, with product-form
    eta updates in between.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

AT_LB, AT_UB, AT_ZERO, BASIC = 0, 1, 2, 3


@dataclass
class SimplexResult:
    status: str            # "optimal", "infeasible", "unbounded", "iteration_limit"
    x: np.ndarray          # structural primal values, length n
    y: np.ndarray          # row duals, length m
    obj: float
    iterations: int
    phase1_iterations: int


def _csr(lp):
    return sp.csr_matrix((np.asarray(lp.val, dtype=np.float64),
                          np.asarray(lp.col_idx, dtype=np.int64),
                          np.asarray(lp.row_ptr, dtype=np.int64)), shape=(lp.m, lp.n))


class _Basis:
    """LU of the basis matrix plus a product-form eta file."""

    def __init__(self, Acsc: sp.csc_matrix, basis: np.ndarray):
        B = Acsc[:, basis].tocsc()
        self.lu = spla.splu(B, permc_spec="COLAMD", diag_pivot_thresh=0.1)
        self.etas = []  # list of (r, alpha)

    def ftran(self, a: np.ndarray) -> np.ndarray:
        v = self.lu.solve(a)
        for r, al in self.etas:
            vr = v[r] / al[r]
            v -= al * vr
            v[r] = vr
        return v

    def btran(self, w: np.ndarray) -> np.ndarray:
        w = w.copy()
        for r, al in reversed(self.etas):
            wr = w[r]
            w[r] = (wr - (al @ w - al[r] * wr)) / al[r]
        return self.lu.solve(w, trans="T")

    def update(self, r: int, alpha: np.ndarray):
        self.etas.append((r, alpha.copy()))


def simplex_solve(lp, tol: float = 1e-9, max_iter: Optional[int] = None,
                  refactor_every: int = 64, degenerate_switch: int = 50,
                  verbose: bool = False) -> SimplexResult:
    m, n = lp.m, lp.n
    A = _csr(lp)
    sense = np.asarray(lp.sense)
    b = np.asarray(lp.b, dtype=np.float64)
    c = np.asarray(lp.c, dtype=np.float64)
    lb = np.asarray(lp.lb, dtype=np.float64)
    ub = np.asarray(lp.ub, dtype=np.float64)

    # ---- equality standard form: [A | slack/surplus | artificials] ----
    g_rows = np.flatnonzero(sense == ord("G"))
    l_rows = np.flatnonzero(sense == ord("L"))
    n_sl = len(g_rows) + len(l_rows)
    sl_rows = np.concatenate([g_rows, l_rows])
    sl_coef = np.concatenate([-np.ones(len(g_rows)), np.ones(len(l_rows))])
    S = sp.csc_matrix((sl_coef, (sl_rows, np.arange(n_sl))), shape=(m, n_sl))

    # start: every structural / slack column at a finite bound (0 if free)
    ntot0 = n + n_sl
    lo = np.concatenate([lb, np.zeros(n_sl)])
    hi = np.concatenate([ub, np.full(n_sl, np.inf)])
    xN = np.where(np.isfinite(lo), lo, np.where(np.isfinite(hi), hi, 0.0))
    status0 = np.where(np.isfinite(lo), AT_LB, np.where(np.isfinite(hi), AT_UB, AT_ZERO))
    AS = sp.hstack([A.tocsc(), S], format="csc")
    resid = b - AS @ xN
    art_sign = np.where(resid >= 0, 1.0, -1.0)
    Art = sp.csc_matrix((art_sign, (np.arange(m), np.arange(m))), shape=(m, m))
    Afull = sp.hstack([AS, Art], format="csc")
    AfullT = Afull.T.tocsr()
    ntot = ntot0 + m

    lo = np.concatenate([lo, np.zeros(m)])
    hi = np.concatenate([hi, np.full(m, np.inf)])
    x = np.concatenate([xN, np.abs(resid)])
    stat = np.concatenate([status0, np.full(m, BASIC)])
    basis = np.arange(ntot0, ntot)
    pos_in_basis = np.full(ntot, -1)
    pos_in_basis[basis] = np.arange(m)

    bscale = 1.0 + np.max(np.abs(b), initial=0.0)
    feas_tol = tol * bscale
    if max_iter is None:
        max_iter = 50 * (m + n) + 10000

    it = 0
    p1_iters = 0

    def run_phase(cost: np.ndarray, dtol: float):
        nonlocal it, x, stat, basis
        fact = _Basis(Afull, basis)
        since_refactor = 0
        degenerate_run = 0
        bland = False
        while True:
            if it >= max_iter:
                return "iteration_limit"
            if since_refactor >= refactor_every:
                fact = _Basis(Afull, basis)
                since_refactor = 0
                # recompute basic values from the non-basic ones to remove drift
                nb = stat != BASIC
                rhs = b - Afull[:, nb] @ x[nb]
                x[basis] = fact.ftran(rhs)
            yv = fact.btran(cost[basis])
            d = cost - AfullT @ yv
            movable = (stat != BASIC) & (hi > lo)
            inc = movable & (((stat == AT_LB) | (stat == AT_ZERO)) & (d < -dtol))
            dec = movable & (((stat == AT_UB) | (stat == AT_ZERO)) & (d > dtol))
            cand = np.flatnonzero(inc | dec)
            if cand.size == 0:
                return "optimal"
            if bland:
                q = int(cand[0])
            else:
                q = int(cand[np.argmax(np.abs(d[cand]))])
            direction = 1.0 if inc[q] else -1.0
            aq = Afull[:, q].toarray().ravel()
            alpha = fact.ftran(aq)
            delta = direction * alpha
            xb = x[basis]
            lob = lo[basis]
            hib = hi[basis]
            piv_tol = 1e-9
            t_best = np.inf
            r = -1
            to_upper = False
            # basic variables that decrease hit their lower bound
            dn = np.flatnonzero((delta > piv_tol) & np.isfinite(lob))
            up = np.flatnonzero((delta < -piv_tol) & np.isfinite(hib))
            ratios_dn = np.maximum(xb[dn] - lob[dn], 0.0) / delta[dn]
            ratios_up = np.maximum(hib[up] - xb[up], 0.0) / (-delta[up])
            idx = np.concatenate([dn, up])
            ratios = np.concatenate([ratios_dn, ratios_up])
            hits_up = np.concatenate([np.zeros(len(dn), bool), np.ones(len(up), bool)])
            if idx.size:
                if bland:
                    tmin = ratios.min()
                    ties = np.flatnonzero(ratios <= tmin + 1e-12)
                    # smallest column index among the tied leaving candidates
                    k = ties[np.argmin(basis[idx[ties]])]
                else:
                    # Harris two-pass: relax bounds by the feasibility tolerance,
                    # then take the largest pivot among the admissible rows
                    relax_dn = (np.maximum(xb[dn] - lob[dn], 0.0) + feas_tol) / delta[dn]
                    relax_up = (np.maximum(hib[up] - xb[up], 0.0) + feas_tol) / (-delta[up])
                    tmax = np.concatenate([relax_dn, relax_up]).min()
                    adm = np.flatnonzero(ratios <= tmax)
                    k = adm[np.argmax(np.abs(delta[idx[adm]]))]
                t_best = ratios[k]
                r = int(idx[k])
                to_upper = bool(hits_up[k])
            flip = hi[q] - lo[q]
            if np.isfinite(flip) and flip <= t_best:
                # bound flip of the entering column: no basis change
                t = flip
                x[basis] = xb - t * delta
                x[q] = hi[q] if direction > 0 else lo[q]
                stat[q] = AT_UB if direction > 0 else AT_LB
                it += 1
                degenerate_run = 0
                bland = False
                continue
            if r < 0:
                return "unbounded"
            t = t_best
            x[basis] = xb - t * delta
            x[q] = x[q] + direction * t
            leave = int(basis[r])
            x[leave] = hi[leave] if to_upper else lo[leave]
            stat[leave] = AT_UB if to_upper else AT_LB
            stat[q] = BASIC
            basis[r] = q
            fact.update(r, alpha)
            since_refactor += 1
            it += 1
            if t <= 1e-12:
                degenerate_run += 1
                if degenerate_run >= degenerate_switch:
                    bland = True
            else:
                degenerate_run = 0
                bland = False
            if verbose and it % 500 == 0:
                print(f"  simplex it {it}  obj {cost @ x:.10g}  bland={bland}")

    # ---- phase 1 ----
    c1 = np.zeros(ntot)
    c1[ntot0:] = 1.0
    st = run_phase(c1, tol)
    p1_iters = it
    infeas = float(np.sum(x[ntot0:]))
    if st == "iteration_limit":
        return SimplexResult(st, x[:n].copy(), np.zeros(m), np.nan, it, p1_iters)
    if infeas > 1e-9 * bscale:
        return SimplexResult("infeasible", x[:n].copy(), np.zeros(m), np.nan, it, p1_iters)
    # freeze artificials at zero
    hi[ntot0:] = 0.0
    x[ntot0:][stat[ntot0:] != BASIC] = 0.0

    # ---- phase 2 ----
    c2 = np.zeros(ntot)
    c2[:n] = c
    cscale = 1.0 + np.max(np.abs(c), initial=0.0)
    st = run_phase(c2, tol * cscale)
    fact = _Basis(Afull, basis)
    nb = stat != BASIC
    x[basis] = fact.ftran(b - Afull[:, nb] @ x[nb])
    y = fact.btran(c2[basis])
    xs = x[:n].copy()
    # clip round-off outside the bounds
    xs = np.minimum(np.maximum(xs, lb), ub)
    return SimplexResult(st, xs, y, float(c @ xs), it, p1_iters)
