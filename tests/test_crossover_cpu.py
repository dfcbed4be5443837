"""Crossover (paper_2607_03627_amd/crossover.py) from approximate points to an
optimal vertex, checked against the CPU oracle's optimum and KKT evaluator."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.kkt import kkt
from oracle.simplex import simplex_solve
from paper_2607_03627_amd.crossover import crossover
from paper_2607_03627_amd.instances import make_instance


def one_sided(lp):
    lb, ub = lp.lb.copy(), lp.ub.copy()
    off, nt, L = lp.meta["col_off"], lp.meta["ncol_t"], lp.meta["L"]
    for t in range(lp.meta["T"]):
        f0 = t * nt + off["f"]
        ub[f0:f0 + L:2] = np.inf
        lb[f0 + 1:f0 + L:2] = -np.inf
    return lp.with_data(lb=lb, ub=ub)


def check_vertex(lp, r, z):
    """An optimal basic solution: objective, KKT, bounds, and at most m
    columns of [A, -I] strictly inside their bounds, all of them basic."""
    assert r.status == "optimal"
    assert abs(r.obj - z) <= 1e-9 * (1 + abs(z))
    k = kkt(lp, r.x, r.y)
    assert k.rel_kkt <= 1e-9
    assert np.all(r.x >= lp.lb - 1e-9) and np.all(r.x <= lp.ub + 1e-9)
    A = sp.csr_matrix((lp.val, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))
    tol = 1e-7 * (1 + np.abs(r.x))
    inside = np.flatnonzero((r.x > lp.lb + tol) & (r.x < lp.ub - tol))
    assert len(r.basis) == lp.m and set(inside) <= set(int(j) for j in r.basis if j < lp.n)
    B = sp.hstack([A, -sp.identity(lp.m)]).tocsc()[:, r.basis].toarray()
    assert np.linalg.matrix_rank(B) == lp.m


@pytest.mark.parametrize("noise", [0.0, 1e-6, 1e-3])
@pytest.mark.parametrize("variant", ["plain", "one_sided"])
def test_crossover_from_perturbed_optimum(noise, variant):
    lp = make_instance("tiny", 3, n_periods=6)
    if variant == "one_sided":
        lp = one_sided(lp)
    ref = simplex_solve(lp)
    rng = np.random.default_rng(1)
    x = ref.x + noise * rng.normal(size=lp.n) * (1 + np.abs(ref.x))
    y = ref.y + noise * rng.normal(size=lp.m) * (1 + np.abs(ref.y))
    r = crossover(lp, x, y)
    check_vertex(lp, r, ref.obj)


def test_crossover_from_an_interior_point():
    # a point far from any vertex (the average of the optimum and the box
    # centre): the clean-up simplex still ends at an optimal vertex
    lp = make_instance("tiny", 4, n_periods=3)
    ref = simplex_solve(lp)
    box = np.isfinite(lp.lb) & np.isfinite(lp.ub)
    mid = np.zeros(lp.n)
    mid[box] = 0.5 * (lp.lb[box] + lp.ub[box])
    r = crossover(lp, 0.5 * (ref.x + mid), 0.5 * ref.y)
    check_vertex(lp, r, ref.obj)
