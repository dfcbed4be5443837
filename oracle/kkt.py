"""Oracle: KKT residuals of a primal-dual pair for the LP relaxation (FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module.

The paper stops its first-order solve on an absolute feasibility tolerance
and a convergence tolerance (Sec. II-D, the PDHG parameter paragraph); it
does not define the residuals.  This module writes out the standard
definitions used for first-order LP solvers (the relative KKT error of
Applegate et al., "Practical large-scale LP with PDHG", NeurIPS 2021), for

    min c'x  s.t.  a_i'x = b_i (E),  a_i'x >= b_i (G),  a_i'x <= b_i (L),
                   lb <= x <= ub,

with the Lagrangian sign convention c'x - y'(Ax - b):

  primal residual  r_i = b_i - a_i'x on E rows, max(0, b_i - a_i'x) on G rows,
                   min(0, b_i - a_i'x) on L rows;            rho_p = ||r||_2
  reduced costs    d = c - A'y
  bound multiplier lam_j = d_j (both bounds finite), max(d_j, 0) (only lb
                   finite), min(d_j, 0) (only ub finite), 0 (free)
  dual residual    rho_d = || [d - lam ; min(y_G, 0) ; max(y_L, 0)] ||_2
  objectives       pobj = c'x,
                   dobj = b'y + sum_j (lb_j max(lam_j, 0) + ub_j min(lam_j, 0))
  relative KKT     max( rho_p / (1 + ||b||_2), rho_d / (1 + ||c||_2),
                        |pobj - dobj| / (1 + |pobj| + |dobj|) )

Every sum is a plain NumPy/SciPy reduction in float64; `math.fsum` variants
are used where a test needs an exactly rounded reference.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class KKT:
    rho_p: float
    rho_d: float
    pobj: float
    dobj: float
    rel_p: float
    rel_d: float
    rel_gap: float
    rel_kkt: float
    max_primal_violation: float  # inf-norm of row violations and bound violations


def csr_matrix(lp) -> sp.csr_matrix:
    return sp.csr_matrix((np.asarray(lp.val, dtype=np.float64),
                          np.asarray(lp.col_idx, dtype=np.int64),
                          np.asarray(lp.row_ptr, dtype=np.int64)), shape=(lp.m, lp.n))


def bound_multiplier(d: np.ndarray, lb: np.ndarray, ub: np.ndarray) -> np.ndarray:
    fl = np.isfinite(lb)
    fu = np.isfinite(ub)
    lam = np.zeros_like(d)
    both = fl & fu
    lam[both] = d[both]
    only_l = fl & ~fu
    lam[only_l] = np.maximum(d[only_l], 0.0)
    only_u = fu & ~fl
    lam[only_u] = np.minimum(d[only_u], 0.0)
    return lam


def kkt(lp, x: np.ndarray, y: np.ndarray) -> KKT:
    A = csr_matrix(lp)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    b = np.asarray(lp.b, dtype=np.float64)
    c = np.asarray(lp.c, dtype=np.float64)
    lb = np.asarray(lp.lb, dtype=np.float64)
    ub = np.asarray(lp.ub, dtype=np.float64)
    sense = np.asarray(lp.sense)
    isE = sense == ord("E")
    isG = sense == ord("G")
    isL = sense == ord("L")

    ax = A @ x
    r = b - ax
    r = np.where(isG, np.maximum(r, 0.0), np.where(isL, np.minimum(r, 0.0), r))
    rho_p = float(np.linalg.norm(r))

    d = c - A.T @ y
    lam = bound_multiplier(d, lb, ub)
    dres = np.concatenate([d - lam, np.minimum(y[isG], 0.0), np.maximum(y[isL], 0.0)])
    rho_d = float(np.linalg.norm(dres))

    pobj = float(c @ x)
    lam_pos = np.maximum(lam, 0.0)
    lam_neg = np.minimum(lam, 0.0)
    lterm = np.zeros_like(lam)
    uterm = np.zeros_like(lam)
    mp = lam_pos > 0
    mn = lam_neg < 0
    lterm[mp] = lb[mp] * lam_pos[mp]
    uterm[mn] = ub[mn] * lam_neg[mn]
    dobj = float(b @ y + lterm.sum() + uterm.sum())

    rel_p = rho_p / (1.0 + float(np.linalg.norm(b)))
    rel_d = rho_d / (1.0 + float(np.linalg.norm(c)))
    rel_gap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
    bviol = np.maximum(np.maximum(lb - x, x - ub), 0.0)
    maxviol = float(max(np.max(np.abs(r), initial=0.0), np.max(bviol, initial=0.0)))
    return KKT(rho_p, rho_d, pobj, dobj, rel_p, rel_d, rel_gap,
               max(rel_p, rel_d, rel_gap), maxviol)
