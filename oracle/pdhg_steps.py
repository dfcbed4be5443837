"""Oracle: single steps of the restarted-PDHG method, written out plainly (FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module.

The paper names PDHG as the GPU leg's method for the LP relaxation (Sec.
II-B, II-C, III-C) and fixes its iteration limit and tolerances (Sec. II-D)
but gives no equations.  The steps below are the published ones this build
follows; each function restates one of them, without any blocking or fusion:

  * minimal presolve (removal of fixed columns and empty rows, 'L' rows
    negated, equality rows first): `internal_problem`;
  * CSR transpose with entries of each transposed row in increasing row
    order: `csr_transpose`;
  * plain sparse products: `csr_matvec`;
  * diagonal preconditioning, Ruiz equilibration in the inf-norm (D. Ruiz,
    "A scaling algorithm to equilibrate both rows and columns norms in
    matrices", RAL-TR-2001-034) followed by the Pock-Chambolle alpha = 1
    scaling (Pock & Chambolle, ICCV 2011, Lemma 2): `ruiz_pc_scaling`;
  * the operator norm ||A_hat||_2 (largest singular value): `spectral_norm`;
  * one PDHG step for the saddle problem min_x max_y c'x - y'(Ax - b) with
    x in [l, u] and y_G >= 0 (Chambolle & Pock, JMIV 2011, Algorithm 1 with
    theta = 1): `pdhg_step`;
  * the reflected Halpern update toward an anchor point (Lu & Yang,
    "Restarted Halpern PDHG for linear programming", 2024):
    `halpern_update`;
  * the fixed-point residual in the PDHG metric used by the restart test:
    `fixed_point_residual`.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclass
class InternalProblem:
    """min c'x s.t. A[:mE] x = b[:mE], A[mE:] x >= b[mE:], l <= x <= u."""

    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    c: np.ndarray
    b: np.ndarray
    l: np.ndarray
    u: np.ndarray
    m_eq: int
    row_map: np.ndarray   # original row; -(row+1) for a negated 'L' row
    col_map: np.ndarray   # original column
    obj_offset: float

    @property
    def m(self):
        return len(self.b)

    @property
    def n(self):
        return len(self.c)

    def matrix(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.m, self.n))


def internal_problem(lp) -> InternalProblem:
    """Minimal presolve.

    Fixed columns (lb == ub) leave the problem: their value times their
    column moves to the right-hand side and c_j lb_j to the objective
    offset.  Rows without entries afterwards leave the problem (their
    feasibility is a property of b alone).  'L' rows are multiplied by -1 so
    that every inequality reads a'x >= b.  Equality rows come first, each
    group in original order.
    """
    A = sp.csr_matrix((np.asarray(lp.val, float), np.asarray(lp.col_idx, np.int64),
                       np.asarray(lp.row_ptr, np.int64)), shape=(lp.m, lp.n))
    lb = np.asarray(lp.lb, float)
    ub = np.asarray(lp.ub, float)
    fixed = lb == ub
    keep_c = np.flatnonzero(~fixed)
    b = np.asarray(lp.b, float) - A[:, fixed] @ lb[fixed]
    offset = float(np.asarray(lp.c, float)[fixed] @ lb[fixed])
    Ak = A[:, keep_c].tocsr()
    nz = np.diff(Ak.indptr) > 0
    sense = np.asarray(lp.sense)
    sign = np.where(sense == ord("L"), -1.0, 1.0)
    eq = np.flatnonzero((sense == ord("E")) & nz)
    ineq = np.flatnonzero((sense != ord("E")) & nz)
    order = np.concatenate([eq, ineq])
    Ai = (sp.diags(sign) @ Ak)[order].tocsr()
    Ai.sort_indices()
    row_map = np.where(sign[order] < 0, -(order + 1), order)
    return InternalProblem(
        row_ptr=Ai.indptr.astype(np.int64), col_idx=Ai.indices.astype(np.int64),
        val=Ai.data.astype(float), c=np.asarray(lp.c, float)[keep_c], b=(sign * b)[order],
        l=lb[keep_c], u=ub[keep_c], m_eq=len(eq), row_map=row_map, col_map=keep_c,
        obj_offset=offset)


def csr_transpose(row_ptr, col_idx, val, n_cols):
    """Transpose of a CSR matrix; within a transposed row, entries follow
    increasing original row index (a stable counting sort by column)."""
    row_ptr = np.asarray(row_ptr, np.int64)
    col_idx = np.asarray(col_idx, np.int64)
    m = len(row_ptr) - 1
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    order = np.argsort(col_idx, kind="stable")
    t_ptr = np.zeros(n_cols + 1, np.int64)
    np.cumsum(np.bincount(col_idx, minlength=n_cols), out=t_ptr[1:])
    return t_ptr, rows[order], np.asarray(val)[order]


def csr_matvec(row_ptr, col_idx, val, x):
    """y_i = sum_k val[k] x[col[k]] over the entries k of row i."""
    row_ptr = np.asarray(row_ptr, np.int64)
    m = len(row_ptr) - 1
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    prod = np.asarray(val, float) * np.asarray(x, float)[np.asarray(col_idx, np.int64)]
    return np.bincount(rows, weights=prod, minlength=m)


def ruiz_pc_scaling(A: sp.csr_matrix, ruiz_iters: int = 10, pock_chambolle: bool = True):
    """Diagonal scalings D_r, D_c with A_hat = diag(D_r) A diag(D_c).

    Each Ruiz pass divides every row and every column of the current matrix
    by the square root of its largest absolute entry (both factors taken
    from the same matrix, then applied together); an all-zero row or column
    keeps factor 1.  The Pock-Chambolle pass with alpha = 1 then divides
    each row and column by the square root of its absolute sum.
    """
    M = sp.csr_matrix(A, dtype=float, copy=True)
    m, n = M.shape
    Dr = np.ones(m)
    Dc = np.ones(n)
    for _ in range(ruiz_iters):
        Aa = abs(M)
        rmax = Aa.max(axis=1).toarray().ravel()
        cmax = Aa.max(axis=0).toarray().ravel()
        r = np.where(rmax > 0, 1.0 / np.sqrt(np.where(rmax > 0, rmax, 1.0)), 1.0)
        s = np.where(cmax > 0, 1.0 / np.sqrt(np.where(cmax > 0, cmax, 1.0)), 1.0)
        M = (sp.diags(r) @ M @ sp.diags(s)).tocsr()
        Dr *= r
        Dc *= s
    if pock_chambolle:
        Aa = abs(M)
        rs = np.asarray(Aa.sum(axis=1)).ravel()
        cs = np.asarray(Aa.sum(axis=0)).ravel()
        r = np.where(rs > 0, 1.0 / np.sqrt(np.where(rs > 0, rs, 1.0)), 1.0)
        s = np.where(cs > 0, 1.0 / np.sqrt(np.where(cs > 0, cs, 1.0)), 1.0)
        M = (sp.diags(r) @ M @ sp.diags(s)).tocsr()
        Dr *= r
        Dc *= s
    return Dr, Dc, M


def spectral_norm(A: sp.spmatrix) -> float:
    """Largest singular value (dense SVD for small matrices, ARPACK otherwise)."""
    m, n = A.shape
    if min(m, n) <= 600:
        return float(np.linalg.svd(A.toarray(), compute_uv=False)[0])
    s = spla.svds(A.astype(float), k=1, return_singular_vectors=False, tol=1e-10,
                  random_state=0)
    return float(s[0])


def project_box(x, l, u):
    return np.minimum(np.maximum(x, l), u)


def project_dual(y, m_eq):
    out = np.array(y, dtype=float, copy=True)
    out[m_eq:] = np.maximum(out[m_eq:], 0.0)
    return out


def pdhg_step(A: sp.csr_matrix, c, b, l, u, m_eq, x, y, tau, sigma):
    """x_hat = P_X(x - tau (c - A'y)),  y_hat = P_Y(y + sigma (b - A(2 x_hat - x)))."""
    x_hat = project_box(x - tau * (c - A.T @ y), l, u)
    y_hat = project_dual(y + sigma * (b - A @ (2.0 * x_hat - x)), m_eq)
    return x_hat, y_hat


def halpern_update(z, z_hat, z_anchor, k, gamma=1.0):
    """z_next = w ((1 + gamma) z_hat - gamma z) + (1 - w) z_anchor with
    w = (k + 1)/(k + 2): the Halpern step on the reflected operator
    (1 + gamma) T - gamma I; gamma = 1 is the reflected form, 0 plain Halpern."""
    w = (k + 1.0) / (k + 2.0)
    return w * ((1.0 + gamma) * z_hat - gamma * z) + (1.0 - w) * z_anchor


def fixed_point_residual(A, x, y, x_hat, y_hat, tau, sigma):
    """||z - T(z)||_P with P = [[I/tau, A'], [A, I/sigma]].

    P is the metric in which the step of pdhg_step is a proximal-point step
    for the Lagrangian c'x - y'(Ax - b): writing the optimality conditions of
    the two projections as 0 in F(z+) + P (z+ - z), with F the (monotone)
    saddle operator, gives the off-diagonal blocks +A' and +A (the primal
    step uses the old y, the dual step the extrapolated 2 x_hat - x).  T is
    firmly nonexpansive in this norm when tau sigma ||A||_2^2 < 1."""
    dx = x_hat - x
    dy = y_hat - y
    q = dx @ dx / tau + dy @ dy / sigma + 2.0 * dy @ (A @ dx)
    return math.sqrt(max(q, 0.0))
