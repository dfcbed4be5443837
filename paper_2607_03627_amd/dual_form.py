"""The dual LP of a unit-commitment LP relaxation, in the same input form.

The paper's aggressive presolve may hand the solver the dual formulation
(Sec. II-D lists the dual form among the tuned settings) and shrinks the
6,049-bus problems to a few 10^4 rows, after which the CPU leg wins every
case (Sec. III-E).  This module builds that dual on the host so that the
same PDHG library can solve it and the two forms can be timed side by side.

For  min c'x  s.t.  A_E x = b_E,  A_G x >= b_G,  A_L x <= b_L,  l <= x <= u
the Lagrangian dual is

    max  b'y + sum_j l_j p_j - sum_j u_j q_j
    s.t. A'y + p - q = c,   y_G >= 0,  y_L <= 0,  p >= 0,  q >= 0,

with p_j only where l_j is finite and q_j only where u_j is finite.  It is
returned as a minimisation (objective negated) with n equality rows and the
columns (y, p, q); its optimal value is minus the primal optimum, and the
duals of its rows (in the sign convention of include/uc_lp.h) are -x.

Host-side data preparation only: no solver arithmetic.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .instances import LP, SENSE_E, SENSE_G, SENSE_L


@dataclass
class DualForm:
    lp: LP                 # the dual as a minimisation in LP form
    m_primal: int
    n_primal: int
    p_cols: np.ndarray     # primal column of each p column
    q_cols: np.ndarray     # primal column of each q column


def dual_form(lp: LP) -> DualForm:
    m, n = lp.m, lp.n
    A = sp.csr_matrix((np.asarray(lp.val, float), np.asarray(lp.col_idx), np.asarray(lp.row_ptr)), shape=(m, n))
    sense = np.asarray(lp.sense)
    lb, ub = np.asarray(lp.lb, float), np.asarray(lp.ub, float)
    pc = np.flatnonzero(np.isfinite(lb))
    qc = np.flatnonzero(np.isfinite(ub))
    # rows j = primal columns: A'_j y + p_j - q_j = c_j
    P = sp.csr_matrix((np.ones(len(pc)), (pc, np.arange(len(pc)))), shape=(n, len(pc)))
    Q = sp.csr_matrix((-np.ones(len(qc)), (qc, np.arange(len(qc)))), shape=(n, len(qc)))
    M = sp.hstack([A.T.tocsr(), P, Q]).tocsr()
    M.sort_indices()
    nd = m + len(pc) + len(qc)
    cost = np.concatenate([-np.asarray(lp.b, float), -lb[pc], ub[qc]])
    lo = np.concatenate([np.where(sense == SENSE_G, 0.0, -np.inf), np.zeros(len(pc) + len(qc))])
    hi = np.concatenate([np.where(sense == SENSE_L, 0.0, np.inf), np.full(len(pc) + len(qc), np.inf)])
    d = LP(m=n, n=nd, row_ptr=M.indptr.astype(np.int32), col_idx=M.indices.astype(np.int32),
           val=M.data.astype(np.float64), c=cost, b=np.asarray(lp.c, float).copy(),
           sense=np.full(n, SENSE_E, np.uint8), lb=lo, ub=hi,
           meta=dict(dual_of=lp.meta.get("shape"), seed=lp.meta.get("seed")))
    return DualForm(d, m, n, pc, qc)


def primal_objective(df: DualForm, dual_obj: float) -> float:
    """The primal optimum from the dual form's (minimised) optimum."""
    return -dual_obj
