"""The dual-form transformation (paper_2607_03627_amd/dual_form.py) against
strong duality, with both LPs solved by the CPU oracle."""

import numpy as np

from oracle.kkt import kkt
from oracle.simplex import simplex_solve
from paper_2607_03627_amd.dual_form import dual_form
from paper_2607_03627_amd.instances import make_instance


def with_one_sided_columns(lp):
    """Line flows keep one limit (alternating), unit outputs lose their lower
    bound 0: columns bounded below only and above only."""
    lb, ub = lp.lb.copy(), lp.ub.copy()
    off, nt, L, G = lp.meta["col_off"], lp.meta["ncol_t"], lp.meta["L"], lp.meta["G"]
    for t in range(lp.meta["T"]):
        f0 = t * nt + off["f"]
        ub[f0:f0 + L:2] = np.inf
        lb[f0 + 1:f0 + L:2] = -np.inf
        lb[t * nt + off["p"]:t * nt + off["p"] + G] = -np.inf
    return lp.with_data(lb=lb, ub=ub)


def test_dual_form_has_the_primal_optimum():
    # strong duality: minus the dual form's optimum is the primal optimum; its
    # row duals, negated, are a primal optimum
    for lp in (make_instance("tiny", 5, n_periods=2), with_one_sided_columns(make_instance("tiny", 5, n_periods=2))):
        res = simplex_solve(lp)
        df = dual_form(lp)
        assert df.lp.m == lp.n and df.lp.n == lp.m + len(df.p_cols) + len(df.q_cols)
        rd = simplex_solve(df.lp)
        assert res.status == rd.status == "optimal"
        assert abs(-rd.obj - res.obj) <= 1e-9 * (1 + abs(res.obj))
        k = kkt(lp, np.clip(-rd.y, lp.lb, lp.ub), res.y)
        assert abs(k.pobj - res.obj) <= 1e-7 * (1 + abs(res.obj))
        assert k.rel_p <= 1e-9
