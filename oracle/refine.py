"""Oracle: one round of iterative refinement for the LP, written out plainly (FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module.

The paper asks for PDHG solutions of the relaxation at tight tolerances
(Sec. II-D) and runs its first-order solve on GPU arithmetic; it gives no
refinement scheme.  Iterative refinement for LP (Gleixner, Steffy & Wolter,
"Iterative refinement for linear programming", INFORMS J. Computing 28(3),
2016) reaches such tolerances with a low-precision inner solver: the error of
a primal-dual point (x*, y*) is itself the solution of an LP of the same
matrix, the "correction LP", whose data are the residuals of (x*, y*) scaled
up so that its solution is of order one; solving it to the inner solver's
relative accuracy and adding the scaled-back correction shrinks the error by
about that accuracy per round.

For min c'x, A_E x = b_E, A_G x >= b_G, l <= x <= u with the Lagrangian
c'x - y'(Ax - b), y_G >= 0, substituting x = x* + x~/D_P and y = y* + y~/D_D
and multiplying the Lagrangian by D_P D_D gives

    c~'x~ - y~'(A x~ - b~),
    c~ = D_D (c - A'y*),          b~ = D_P (b - A x*),
    l~ = D_P (l - x*),            u~ = D_P (u - x*),
    y~_E free,                    y~_G >= ylo_G = -D_D y*_G.

So the correction problem is the same saddle problem with shifted data and a
shifted lower bound on the inequality duals: a PDHG solver takes it as it
is, with the projection y~_G >= ylo_G.  Its primal form is an LP with the
objective (c~ - A_G' ylo_G)'x~ + ylo_G'b~_G, because the supremum over
y~_G >= ylo_G of -y~_G'(A_G x~ - b~_G) is -ylo_G'(A_G x~ - b~_G) on the
feasible set (`standard_form`).

Scale factors (the reading this build takes; the 2016 paper uses inf-norms
and a simplex, whose points are exactly complementary):
    delta_P = || primal violation of x* ||_2   (E rows: r, G rows: max(r, 0))
    delta_D = || dual residual of y* ||_2      (d - lam(d), as in kkt.py)
    D_P = min(1 / delta_P, growth * D_P_prev)  (growth * D_P_prev if delta_P = 0)
    D_D = min(1 / delta_D, growth * D_D_prev)
and the primal weight carries over from the solve that produced the
correction: PDHG on data whose primal part is scaled by D_P and dual part by
D_D takes the same steps as on the unscaled error when its primal weight is
multiplied by D_D / D_P, so a round starts at
omega_prev * (D_D / D_P) / (D_D_prev / D_P_prev).

The new point of a round is x* <- proj_[l,u](x* + x~ / D_P),
y* <- y* + y~ / D_D with y*_G projected to >= 0 (the first round takes the
first solve's point as x~, y~ with x* = 0, y* = 0, D = 1).

The correction data go to FP32 for the inner solve; the bounds are rounded
outward-safe: l~ and ylo upward, u~ downward, so every FP32-feasible
correction maps back into the FP64 box and onto y_G >= 0.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .kkt import bound_multiplier


def round_up32(v):
    """Smallest float32 >= v, elementwise (infinities and NaN pass through)."""
    v = np.asarray(v, dtype=np.float64)
    f = v.astype(np.float32)
    low = f.astype(np.float64) < v
    return np.where(low, np.nextafter(f, np.float32(np.inf)), f).astype(np.float32)


def round_down32(v):
    """Largest float32 <= v, elementwise."""
    v = np.asarray(v, dtype=np.float64)
    f = v.astype(np.float32)
    high = f.astype(np.float64) > v
    return np.where(high, np.nextafter(f, np.float32(-np.inf)), f).astype(np.float32)


@dataclass
class Round:
    x: np.ndarray          # new x* (FP64, in [l, u])
    y: np.ndarray          # new y* (FP64, y_G >= 0)
    r: np.ndarray          # b - A x*
    d: np.ndarray          # c - A' y*
    viol: np.ndarray       # primal violation of each row
    dres: np.ndarray       # d - lam(d)
    delta_p: float         # D_P
    delta_d: float         # D_D
    omega: float           # starting primal weight of the next correction solve
    c_t: np.ndarray        # correction data, FP64
    b_t: np.ndarray
    l_t: np.ndarray
    u_t: np.ndarray
    ylo: np.ndarray        # lower bound of y~ on G rows (-inf on E rows)

    def fp32(self):
        """The correction data as the inner FP32 solve receives them:
        c~, b~ to nearest; l~, ylo rounded up, u~ rounded down (a box that
        the rounding would empty collapses to the rounded midpoint)."""
        lo = round_up32(self.l_t)
        hi = round_down32(self.u_t)
        bad = lo > hi
        mid = ((self.l_t + self.u_t) / 2).astype(np.float32)
        lo = np.where(bad, mid, lo)
        hi = np.where(bad, mid, hi)
        return dict(c=self.c_t.astype(np.float32), b=self.b_t.astype(np.float32), l=lo, u=hi,
                    ylo=round_up32(self.ylo))


def refine_round(A: sp.csr_matrix, c, b, l, u, m_eq: int, x_star, y_star, x_corr, y_corr,
                 inv_dp: float, inv_dd: float, first: bool, dp_prev: float, dd_prev: float,
                 growth: float, omega_prev: float) -> Round:
    """One refinement round: fold the correction (x_corr, y_corr) of the
    previous round into (x*, y*), then form the next correction problem."""
    c, b, l, u = (np.asarray(v, dtype=np.float64) for v in (c, b, l, u))
    m = len(b)
    isG = np.arange(m) >= m_eq
    base_x = np.zeros_like(c) if first else np.asarray(x_star, dtype=np.float64)
    base_y = np.zeros_like(b) if first else np.asarray(y_star, dtype=np.float64)
    x = np.minimum(np.maximum(base_x + np.asarray(x_corr, dtype=np.float64) * inv_dp, l), u)
    y = base_y + np.asarray(y_corr, dtype=np.float64) * inv_dd
    y = np.where(isG, np.maximum(y, 0.0), y)
    r = b - A @ x
    viol = np.where(isG, np.maximum(r, 0.0), r)
    d = c - A.T @ y
    dres = d - bound_multiplier(d, l, u)
    delta_p_err = float(np.linalg.norm(viol))
    delta_d_err = float(np.linalg.norm(dres))
    dp = min(1.0 / delta_p_err, growth * dp_prev) if delta_p_err > 0 else growth * dp_prev
    dd = min(1.0 / delta_d_err, growth * dd_prev) if delta_d_err > 0 else growth * dd_prev
    omega = omega_prev * (dd / dp) / (dd_prev / dp_prev)
    ylo = np.where(isG, -dd * y, -np.inf)
    return Round(x=x, y=y, r=r, d=d, viol=viol, dres=dres, delta_p=dp, delta_d=dd, omega=omega,
                 c_t=dd * d, b_t=dp * r, l_t=dp * (l - x), u_t=dp * (u - x), ylo=ylo)


def standard_form(A: sp.csr_matrix, m_eq: int, rnd: Round):
    """The correction problem as a plain LP: (objective vector, constant).
    Constraints: A_E x~ = b~_E, A_G x~ >= b~_G, l~ <= x~ <= u~.  A G-row dual
    mu >= 0 of this LP is y~_G - ylo_G."""
    G = slice(m_eq, None)
    AG = A[G]
    cobj = rnd.c_t - AG.T @ rnd.ylo[G]
    const = float(rnd.ylo[G] @ rnd.b_t[G])
    return cobj, const


def map_back(rnd: Round, m_eq: int, x_t, mu):
    """Point of the original problem from a solution (x~, mu) of the standard
    form: y~_E = mu_E, y~_G = ylo_G + mu_G."""
    y_t = np.asarray(mu, dtype=np.float64).copy()
    y_t[m_eq:] += rnd.ylo[m_eq:]
    return rnd.x + np.asarray(x_t) / rnd.delta_p, rnd.y + y_t / rnd.delta_d
