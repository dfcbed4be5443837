"""Crossover: from an approximate primal-dual point of the LP relaxation to an
optimal vertex (basic solution) with its basis.

In the paper's GPU pipeline the first-order solve is followed by crossover
before simplex clean-up and branch-and-bound (Sec. II-C, Algorithm 1; Sec.
III-C times "relaxation and crossover" as one stage).  This module does that
step on the host for a point returned by the PDHG library:

1. Standard form.  Every row gets a logical column: a_i'x - s_i = b_i with
   s_i in [0, 0] ('E'), [0, inf) ('G'), (-inf, 0] ('L'), so the system is
   [A, -I] z = b with bounds on every column of z = (x, s).
2. Basis identification.  A column whose value lies well inside its bounds
   must be basic in any nearby vertex; a column at a bound with a reduced
   cost of the right sign can stay nonbasic there.  Columns are ranked by
   how far inside their bounds they sit (then by how small their reduced
   cost is), and m linearly independent columns are taken in that order by
   an LU with partial pivoting of the weighted, transposed candidate matrix
   (the logical columns complete any rank deficit).
3. Basic solution.  Nonbasic columns go to their nearer bound (free ones to
   0); the basic values follow from B z_B = b - N z_N.
4. Clean-up.  A bounded primal simplex from that basis: while some basic
   value violates its bounds, it minimises the sum of violations (a step
   stops where a violating variable reaches its bound); then it minimises
   c'x with the bounded ratio test.  Dantzig pricing, Bland's rule after a
   run of degenerate steps.

Host code (NumPy / SciPy); it does not use the CPU oracle.
"""

from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import scipy.linalg as la
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .instances import SENSE_E, SENSE_G, SENSE_L

AT_LOWER, AT_UPPER, AT_ZERO, BASIC = 0, 1, 2, 3


@dataclass
class CrossoverResult:
    status: str          # "optimal", "pivot_limit", "unbounded", "singular"
    x: np.ndarray        # vertex, original columns
    y: np.ndarray        # row duals (Lagrangian c'x - y'(Ax - b))
    obj: float
    basis: np.ndarray    # basic columns of [A, -I] (n structural, then one logical per row)
    pivots: int          # simplex pivots after the basis was identified
    phase1_pivots: int
    seconds: float
    candidates: int      # columns strictly inside their bounds at the input point


def _standard_form(lp):
    m, n = lp.m, lp.n
    A = sp.csr_matrix((np.asarray(lp.val, float), np.asarray(lp.col_idx), np.asarray(lp.row_ptr)), shape=(m, n))
    M = sp.hstack([A, -sp.identity(m, format="csr")]).tocsc()
    sense = np.asarray(lp.sense)
    slo = np.where(sense == SENSE_L, -np.inf, 0.0)
    shi = np.where(sense == SENSE_G, np.inf, 0.0)
    lo = np.concatenate([np.asarray(lp.lb, float), slo])
    hi = np.concatenate([np.asarray(lp.ub, float), shi])
    cost = np.concatenate([np.asarray(lp.c, float), np.zeros(m)])
    return A, M, lo, hi, cost


def _independent(D, w, m):
    """Rows of D (one per column of M) in pivot order of an LU with partial
    pivoting of D scaled by w; a pivot counts if it keeps a fair part of its
    row's own size (1e-9), i.e. the row is not a combination of earlier ones."""
    p, _, U = la.lu(D * w[:, None], p_indices=True)
    order = np.argsort(p)          # D*w = L[p] U: the k-th pivot is row order[k]
    k = min(m, U.shape[0])
    diag = np.abs(np.diag(U))[:k]
    return [int(r) for r, d in zip(order[:k], diag) if d > 1e-9 * w[r]]


def _pick_basis(M, order_weight, m):
    """m independent columns of M, preferring large weights: an LU with
    partial (row) pivoting of the transposed, row-normalised matrix whose
    rows are scaled by the weights, so each pivot goes to the heaviest column
    still independent of those chosen before it.  Logical columns complete
    any deficit in a second, smaller pass."""
    D = M.toarray().T
    norms = np.abs(D).max(axis=1)
    norms[norms == 0] = 1.0
    D /= norms[:, None]
    chosen = _independent(D, order_weight, m)
    if len(chosen) < m:
        n = M.shape[1] - m
        rows = chosen + [n + i for i in range(m)]
        w2 = np.concatenate([np.full(len(chosen), 1e6), np.ones(m)])
        sub = _independent(D[rows], w2, m)
        chosen = [rows[r] for r in sub]
    return np.array(chosen[:m], dtype=np.int64)


class _Basis:
    """LU of the basis matrix, refactored after every pivot."""

    def __init__(self, M, idx):
        self.idx = np.array(idx)
        self.lu = spla.splu(M[:, self.idx].tocsc())

    def solve(self, v):
        return self.lu.solve(v)

    def solve_t(self, v):
        return self.lu.solve(v, trans="T")


def crossover(lp, x, y, tol=1e-9, max_pivots=None, verbose=False) -> CrossoverResult:
    t0 = time.perf_counter()
    m, n = lp.m, lp.n
    A, M, lo, hi, cost = _standard_form(lp)
    N = n + m
    b = np.asarray(lp.b, float)
    x = np.clip(np.asarray(x, float), lo[:n], hi[:n])
    s = np.clip(A @ x - b, lo[n:], hi[n:])
    z = np.concatenate([x, s])
    d = cost - M.T @ np.asarray(y, float)
    scale = 1.0 + np.abs(z)
    dist = np.minimum(z - lo, hi - z)                 # inf for free columns
    inside = dist > 1e-7 * scale
    candidates = int(np.sum(inside))
    # weights: inside columns first (farther inside first), then columns at a
    # bound with a small reduced cost, then the rest
    dn = np.abs(d) / (1.0 + np.abs(cost).max())
    w = np.where(inside, 1e8 * (1.0 + np.minimum(dist / scale, 1.0)), 1e4 / (1.0 + 1e6 * dn))
    w[lo == hi] = 1e-3                                # fixed columns only to complete the rank
    basis = list(_pick_basis(M, w, m))
    if len(basis) < m:
        return CrossoverResult("singular", x, np.asarray(y, float), float(np.dot(lp.c, x)), np.array(basis), 0, 0,
                               time.perf_counter() - t0, candidates)
    status = np.full(N, AT_LOWER, dtype=np.int8)
    finite_lo, finite_hi = np.isfinite(lo), np.isfinite(hi)
    up = finite_hi & (~finite_lo | (hi - z < z - lo))
    status[up] = AT_UPPER
    status[~finite_lo & ~finite_hi] = AT_ZERO
    status[basis] = BASIC

    def nonbasic_value(j):
        return lo[j] if status[j] == AT_LOWER else hi[j] if status[j] == AT_UPPER else 0.0

    max_pivots = max_pivots or 20 * (m + n)
    pivots = phase1 = degenerate = 0
    result = "optimal"
    while True:
        B = _Basis(M, basis)
        nb = np.flatnonzero(status != BASIC)
        zN = np.array([nonbasic_value(j) for j in nb])
        zB = B.solve(b - M[:, nb] @ zN)
        lB, hB = lo[basis], hi[basis]
        ftol = tol * (1.0 + np.abs(zB))
        below, above = zB < lB - ftol, zB > hB + ftol
        infeasible = below.any() or above.any()
        cB = np.where(below, -1.0, np.where(above, 1.0, 0.0)) if infeasible else cost[basis]
        pi = B.solve_t(cB)
        dN = (0.0 if infeasible else cost[nb]) - M[:, nb].T @ pi
        dtol = tol * (1.0 + np.abs(cost).max())
        st = status[nb]
        can_up = ((st == AT_LOWER) | (st == AT_ZERO)) & (dN < -dtol) & (lo[nb] < hi[nb])
        can_dn = ((st == AT_UPPER) | (st == AT_ZERO)) & (dN > dtol) & (lo[nb] < hi[nb])
        elig = np.flatnonzero(can_up | can_dn)
        if elig.size == 0:
            if infeasible:
                result = "infeasible"
            break
        if pivots >= max_pivots:
            result = "pivot_limit"
            break
        k = elig[0] if degenerate > 50 else elig[np.argmax(np.abs(dN[elig]))]   # Bland / Dantzig
        q = nb[k]
        dirn = 1.0 if can_up[k] else -1.0
        alpha = B.solve(M[:, q].toarray().ravel())
        dz = -dirn * alpha                           # change of z_B per unit step of z_q
        # ratio test
        theta = hi[q] - lo[q] if np.isfinite(hi[q] - lo[q]) else np.inf
        leave, leave_to = -1, None
        ptol = 1e-12
        for i in np.flatnonzero(np.abs(dz) > ptol):
            if infeasible and below[i]:
                if dz[i] > 0:
                    t = (lB[i] - zB[i]) / dz[i]
                    bound = AT_LOWER
                else:
                    continue
            elif infeasible and above[i]:
                if dz[i] < 0:
                    t = (hB[i] - zB[i]) / dz[i]
                    bound = AT_UPPER
                else:
                    continue
            elif dz[i] > 0:
                if not np.isfinite(hB[i]):
                    continue
                t = (hB[i] - zB[i]) / dz[i]
                bound = AT_UPPER
            else:
                if not np.isfinite(lB[i]):
                    continue
                t = (lB[i] - zB[i]) / dz[i]
                bound = AT_LOWER
            t = max(t, 0.0)
            if t < theta - 1e-12 or (leave >= 0 and abs(t - theta) <= 1e-12 and abs(dz[i]) > abs(dz[leave])):
                theta, leave, leave_to = t, i, bound
        if not np.isfinite(theta):
            result = "unbounded"
            break
        degenerate = degenerate + 1 if theta <= 1e-12 else 0
        pivots += 1
        phase1 += int(infeasible)
        if leave < 0:
            # bound flip of the entering column, no basis change
            status[q] = AT_UPPER if dirn > 0 else AT_LOWER
            continue
        out = basis[leave]
        basis[leave] = q
        status[q] = BASIC
        status[out] = AT_LOWER if leave_to == AT_LOWER else AT_UPPER
        if lo[out] == -np.inf and hi[out] == np.inf:
            status[out] = AT_ZERO
        if verbose and pivots % 100 == 0:
            print(f"[crossover] pivot {pivots} phase {'1' if infeasible else '2'}", flush=True)
    zfull = np.zeros(N)
    zfull[basis] = zB
    nbm = status != BASIC
    zfull[nbm] = [nonbasic_value(j) for j in np.flatnonzero(nbm)]
    xv = zfull[:n]
    return CrossoverResult(result, xv, pi if not infeasible else np.asarray(y, float), float(np.dot(lp.c, xv)),
                           np.array(basis), pivots, phase1, time.perf_counter() - t0, candidates)
