"""Pins of the iterative-refinement oracle (oracle/refine.py) against facts
that do not come from it: a one-dimensional round computed by hand, the
optimum of the original LP recovered from a simplex solve of the correction
LP (on the unscaled and on the Ruiz/Pock-Chambolle-scaled internal
problem), the exact optimum being a fixed point, a planted sign mistake
that the recovery test catches, and directed FP32 rounding checked against
neighbouring floats."""

import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import pdhg_steps as ps
from oracle import refine as rf
from oracle.kkt import kkt
from oracle.simplex import simplex_solve
from paper_2607_03627_amd.instances import LP, make_instance


def lp_from(A, b, m_eq, c, l, u):
    A = sp.csr_matrix(A)
    A.sort_indices()
    m = A.shape[0]
    sense = np.array([ord("E")] * m_eq + [ord("G")] * (m - m_eq), np.uint8)
    return LP(m=m, n=A.shape[1], row_ptr=A.indptr.astype(np.int32), col_idx=A.indices.astype(np.int32),
              val=A.data.astype(float), c=np.asarray(c, float), b=np.asarray(b, float), sense=sense,
              lb=np.asarray(l, float), ub=np.asarray(u, float))


def test_round_by_hand_one_dimensional():
    # min x  s.t.  x >= 1 (G row),  0 <= x <= 5;  optimum x = 1, y = 1.
    A = sp.csr_matrix(np.array([[1.0]]))
    r = rf.refine_round(A, [1.0], [1.0], [0.0], [5.0], 0, None, None, [0.9], [1.2], 1.0, 1.0, True,
                        1.0, 1.0, 1e4, 3.0)
    assert r.x[0] == 0.9 and r.y[0] == 1.2
    assert math.isclose(r.r[0], 0.1, rel_tol=1e-15) and math.isclose(r.viol[0], 0.1, rel_tol=1e-15)
    assert math.isclose(r.d[0], -0.2, rel_tol=1e-15)
    assert r.dres[0] == 0.0                      # boxed column: lam = d
    assert math.isclose(r.delta_p, 10.0, rel_tol=1e-14)
    assert r.delta_d == 1e4                      # no dual residual: growth cap
    assert math.isclose(r.omega, 3.0 * 1e4 / 10.0, rel_tol=1e-14)   # weight 3 carried over
    assert math.isclose(r.c_t[0], -2000.0, rel_tol=1e-14)
    assert math.isclose(r.b_t[0], 1.0, rel_tol=1e-14)
    assert math.isclose(r.l_t[0], -9.0, rel_tol=1e-14) and math.isclose(r.u_t[0], 41.0, rel_tol=1e-14)
    assert math.isclose(r.ylo[0], -12000.0, rel_tol=1e-14)
    cobj, const = rf.standard_form(A, 0, r)
    assert math.isclose(cobj[0], 10000.0, rel_tol=1e-14) and math.isclose(const, -12000.0, rel_tol=1e-14)
    # the correction LP: min 1e4 x~ - 12000, x~ >= 1, x~ in [-9, 41] -> x~ = 1, mu = 1e4
    x, y = rf.map_back(r, 0, [1.0], [1e4])
    assert math.isclose(x[0], 1.0, rel_tol=1e-15) and math.isclose(y[0], 1.0, rel_tol=1e-15)


def test_first_round_projects_and_later_rounds_accumulate():
    A = sp.csr_matrix(np.array([[1.0, 1.0], [1.0, -1.0]]))
    c, b, l, u = [1.0, 2.0], [1.0, 0.0], [0.0, -np.inf], [1.0, np.inf]
    r = rf.refine_round(A, c, b, l, u, 1, None, None, [1.5, 0.25], [0.5, -0.5], 1.0, 1.0, True,
                        1.0, 1.0, 1e4, 1.0)
    assert r.x.tolist() == [1.0, 0.25]          # clamped to u = 1
    assert r.y.tolist() == [0.5, 0.0]            # G-row dual projected to >= 0
    r2 = rf.refine_round(A, c, b, l, u, 1, r.x, r.y, [-2.0, 4.0], [1.0, 3.0], 0.5, 0.25, False,
                         r.delta_p, r.delta_d, 1e4, r.omega)
    assert r2.x.tolist() == [0.0, 2.25] and r2.y.tolist() == [0.75, 0.75]
    # one-sided column 1 (free): its whole reduced cost is dual residual
    assert r2.dres[1] == r2.d[1] and r2.dres[0] == 0.0


def perturbed_optimum(lp, rng, scale):
    res = simplex_solve(lp)
    assert res.status == "optimal"
    x = res.x + scale * rng.normal(size=lp.n) * (1 + np.abs(res.x))
    y = res.y + scale * rng.normal(size=lp.m) * (1 + np.abs(res.y))
    return res, x, y


def solve_correction(A, m_eq, rnd):
    cobj, const = rf.standard_form(A, m_eq, rnd)
    sub = lp_from(A, rnd.b_t, m_eq, cobj, rnd.l_t, rnd.u_t)
    res = simplex_solve(sub)
    assert res.status == "optimal"
    return res, const


def internal_lp(ip, Dr=None, Dc=None):
    A = ip.matrix()
    if Dr is None:
        return A, lp_from(A, ip.b, ip.m_eq, ip.c, ip.l, ip.u), ip.c, ip.b, ip.l, ip.u
    Ah = sp.diags(Dr) @ A @ sp.diags(Dc)
    c, b, l, u = ip.c * Dc, ip.b * Dr, ip.l / Dc, ip.u / Dc
    return sp.csr_matrix(Ah), lp_from(Ah, b, ip.m_eq, c, l, u), c, b, l, u


@pytest.mark.parametrize("scaled", [False, True])
@pytest.mark.parametrize("seed", [0, 3])
def test_correction_lp_recovers_the_optimum(scaled, seed):
    """Solving the correction LP exactly and mapping back gives an optimal
    primal-dual pair of the original LP: objective equal to the simplex
    optimum and KKT error at rounding level."""
    lp = make_instance("tiny", seed, n_periods=4)
    ip = ps.internal_problem(lp)
    if scaled:
        Dr, Dc, _ = ps.ruiz_pc_scaling(ip.matrix())
        A, ilp, c, b, l, u = internal_lp(ip, Dr, Dc)
    else:
        A, ilp, c, b, l, u = internal_lp(ip)
    rng = np.random.default_rng(seed)
    opt, x0, y0 = perturbed_optimum(ilp, rng, 1e-3)
    rnd = rf.refine_round(A, c, b, l, u, ip.m_eq, None, None, x0, y0, 1.0, 1.0, True, 1.0, 1.0, 1e4, 1.0)
    assert rnd.delta_p > 0 and rnd.delta_d > 0
    corr, const = solve_correction(A, ip.m_eq, rnd)
    x, y = rf.map_back(rnd, ip.m_eq, corr.x, corr.y)
    k = kkt(ilp, x, y)
    assert abs(k.pobj - opt.obj) <= 1e-9 * (1 + abs(opt.obj))
    assert k.rel_kkt <= 1e-9


def test_correction_value_is_the_scaled_lagrangian_gap():
    """At the correction optimum x~, c~'x~ - ylo_G'(A_G x~ - b~_G) equals
    D_P D_D (c'x - L(x*)), with x the mapped-back optimum and
    L(x*) = c'x* - y*'(A x* - b) the Lagrangian at the start point (the
    E-row terms vanish because x satisfies the E rows)."""
    lp = make_instance("tiny", 1, n_periods=4)
    ip = ps.internal_problem(lp)
    A, ilp, c, b, l, u = internal_lp(ip)
    rng = np.random.default_rng(7)
    opt, x0, y0 = perturbed_optimum(ilp, rng, 1e-3)
    rnd = rf.refine_round(A, c, b, l, u, ip.m_eq, None, None, x0, y0, 1.0, 1.0, True, 1.0, 1.0, 1e4, 1.0)
    corr, const = solve_correction(A, ip.m_eq, rnd)
    x, y = rf.map_back(rnd, ip.m_eq, corr.x, corr.y)
    lag_start = float(c @ rnd.x - rnd.y @ (A @ rnd.x - b))
    # the G-row term of the standard form is the sup over y~_G >= ylo_G at the optimum
    G = slice(ip.m_eq, None)
    value = float(rnd.c_t @ corr.x - rnd.ylo[G] @ (A[G] @ corr.x - rnd.b_t[G]))
    assert math.isclose(value, corr.obj + const, rel_tol=1e-9, abs_tol=1e-9)
    assert math.isclose(value, rnd.delta_p * rnd.delta_d * (float(c @ x) - lag_start), rel_tol=1e-7, abs_tol=1e-7)


def test_exact_optimum_is_a_fixed_point():
    lp = make_instance("tiny", 2, n_periods=3)
    ip = ps.internal_problem(lp)
    A, ilp, c, b, l, u = internal_lp(ip)
    opt = simplex_solve(ilp)
    rnd = rf.refine_round(A, c, b, l, u, ip.m_eq, None, None, opt.x, opt.y, 1.0, 1.0, True, 1.0, 1.0, 1e4, 1.0)
    scale_r = 1 + np.abs(b).max()
    assert np.linalg.norm(rnd.viol) <= 1e-9 * scale_r
    assert np.linalg.norm(rnd.dres) <= 1e-9 * (1 + np.abs(c).max())
    # the point does not move: the correction LP's solution maps back to an
    # optimal point with the same objective
    corr, const = solve_correction(A, ip.m_eq, rnd)
    x, y = rf.map_back(rnd, ip.m_eq, corr.x, corr.y)
    assert abs(float(c @ x) - opt.obj) <= 1e-9 * (1 + abs(opt.obj))
    assert kkt(ilp, x, y).rel_kkt <= 1e-9


def test_planted_shift_sign_is_caught():
    """With the dual shift of the G rows taken with the wrong sign the
    mapped-back point is no longer optimal."""
    lp = make_instance("tiny", 0, n_periods=4)
    ip = ps.internal_problem(lp)
    A, ilp, c, b, l, u = internal_lp(ip)
    rng = np.random.default_rng(0)
    opt, x0, y0 = perturbed_optimum(ilp, rng, 1e-3)
    rnd = rf.refine_round(A, c, b, l, u, ip.m_eq, None, None, x0, y0, 1.0, 1.0, True, 1.0, 1.0, 1e4, 1.0)
    bad = rf.Round(**{**rnd.__dict__, "ylo": -rnd.ylo})
    bad.ylo[: ip.m_eq] = -np.inf
    corr, const = solve_correction(A, ip.m_eq, bad)
    x, y = rf.map_back(bad, ip.m_eq, corr.x, corr.y)
    k = kkt(ilp, x, y)
    assert k.rel_kkt > 1e-6 or abs(k.pobj - opt.obj) > 1e-6 * (1 + abs(opt.obj))


def test_scaled_correction_step_is_the_scaled_error_step():
    """The weight carried over: one PDHG step on the correction data scaled
    by (D_P, D_D) with primal weight omega * D_D / D_P is the step on the
    unscaled error (D = 1, weight omega), scaled by D_P and D_D."""
    lp = make_instance("tiny", 1, n_periods=3)
    ip = ps.internal_problem(lp)
    A, ilp, c, b, l, u = internal_lp(ip)
    m = ip.m
    rng = np.random.default_rng(5)
    x0 = np.clip(rng.normal(size=ip.n), l, u)
    y0 = 100.0 * rng.normal(size=m)
    # a growth cap below every 1 / delta gives D_P = D_D = 1e-6; without it
    # D_P = 1 / delta_P and D_D = 1 / delta_D differ
    one = rf.refine_round(A, c, b, l, u, m, None, None, x0, y0, 1.0, 1.0, True, 1.0, 1.0, 1e-6, 1.0)
    big = rf.refine_round(A, c, b, l, u, m, None, None, x0, y0, 1.0, 1.0, True, 1.0, 1.0, 1e4, 1.0)
    assert one.delta_p == 1e-6 and one.delta_d == 1e-6
    assert abs((big.delta_d / big.delta_p) / (one.delta_d / one.delta_p) - 1) > 0.1
    ex, ey = rng.normal(size=ip.n) * 1e-3, rng.normal(size=m) * 1e-3
    eta, omega = 0.9, 2.5
    dp1, dd1 = one.delta_p, one.delta_d
    w1 = omega * (dd1 / dp1)
    xs1, ys1 = ps.pdhg_step(A, one.c_t, one.b_t, one.l_t, one.u_t, m, dp1 * ex, dd1 * ey, eta / w1, eta * w1)
    wb = w1 * (big.delta_d / big.delta_p) / (dd1 / dp1)
    xsb, ysb = ps.pdhg_step(A, big.c_t, big.b_t, big.l_t, big.u_t, m, big.delta_p * ex, big.delta_d * ey,
                            eta / wb, eta * wb)
    assert np.allclose(xsb / big.delta_p, xs1 / dp1, rtol=1e-9, atol=1e-12)
    assert np.allclose(ysb / big.delta_d, ys1 / dd1, rtol=1e-9, atol=1e-12)
    # a weight that does not carry the change of D_D / D_P takes another step
    xsw, _ = ps.pdhg_step(A, big.c_t, big.b_t, big.l_t, big.u_t, m, big.delta_p * ex, big.delta_d * ey,
                          eta / w1, eta * w1)
    assert not np.allclose(xsw / big.delta_p, xs1 / dp1, rtol=1e-6, atol=1e-9)


def test_directed_rounding_against_neighbouring_floats():
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-30, 30, 2000),
                        [0.0, -0.0, 0.1, -0.1, 1.0, np.inf, -np.inf, 3.4e38, -3.4e38]])
    up, dn = rf.round_up32(v), rf.round_down32(v)
    fin = np.isfinite(v)
    assert np.all(up[fin].astype(np.float64) >= v[fin]) and np.all(dn[fin].astype(np.float64) <= v[fin])
    below = np.nextafter(up, np.float32(-np.inf)).astype(np.float64)
    above = np.nextafter(dn, np.float32(np.inf)).astype(np.float64)
    assert np.all(below[fin] < v[fin]) and np.all(above[fin] > v[fin])
    # known neighbours of 0.1
    assert rf.round_up32(0.1) == np.float32(0.1) and float(np.float32(0.1)) > 0.1
    assert rf.round_down32(0.1) == np.nextafter(np.float32(0.1), np.float32(0))
    assert rf.round_up32(np.inf) == np.inf and rf.round_down32(-np.inf) == -np.inf
