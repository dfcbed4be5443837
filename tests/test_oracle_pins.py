"""Pins of the CPU oracle against facts that do not come from the oracle itself:
brute-force vertex enumeration, LP strong duality, closed forms of economic
dispatch and of DC network flows, hand-computed KKT values, an independent
library solve, and algebraic properties of the single PDHG steps."""

import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import pdhg_steps as ps
from oracle.kkt import kkt
from oracle.reference import highs_solve
from oracle.simplex import simplex_solve
from paper_2607_03627_amd.instances import (LP, Grid, Units, build_uc_lp, make_instance,
                                            SENSE_E, SENSE_G, SENSE_L)


def dense_lp(A, b, sense, c, lb, ub):
    A = np.asarray(A, float)
    M = sp.csr_matrix(A)
    M.sort_indices()
    return LP(m=A.shape[0], n=A.shape[1], row_ptr=M.indptr.astype(np.int32),
              col_idx=M.indices.astype(np.int32), val=M.data.astype(float),
              c=np.asarray(c, float), b=np.asarray(b, float),
              sense=np.asarray([ord(s) for s in sense], np.uint8),
              lb=np.asarray(lb, float), ub=np.asarray(ub, float))


def random_tiny_lp(rng, n, mE, mG, mL=0):
    m = mE + mG + mL
    A = rng.normal(size=(m, n)) * (rng.random((m, n)) < 0.8)
    lb = rng.uniform(-2, 0, n)
    ub = lb + rng.uniform(0.5, 3, n)
    xf = lb + rng.random(n) * (ub - lb)
    b = A @ xf
    b[mE:mE + mG] -= rng.uniform(0, 1, mG)
    b[mE + mG:] += rng.uniform(0, 1, mL)
    c = rng.normal(size=n)
    return dense_lp(A, b, "E" * mE + "G" * mG + "L" * mL, c, lb, ub), A


def brute_force_min(A, b, sense, c, lb, ub, tol=1e-9):
    """Minimum of c'x over the vertices of a bounded polytope."""
    m, n = A.shape
    eq = [i for i in range(m) if sense[i] == "E"]
    ineq = [i for i in range(m) if sense[i] != "E"]
    # candidate active constraints: inequality rows and the 2n bounds
    cands = [("row", i) for i in ineq] + [("lb", j) for j in range(n)] + [("ub", j) for j in range(n)]
    best = math.inf
    need = n - len(eq)
    if need < 0:
        raise ValueError
    for subset in itertools.combinations(cands, need):
        M = [A[i] for i in eq]
        r = [b[i] for i in eq]
        for kind, idx in subset:
            if kind == "row":
                M.append(A[idx]); r.append(b[idx])
            else:
                e = np.zeros(n); e[idx] = 1.0
                M.append(e); r.append(lb[idx] if kind == "lb" else ub[idx])
        M = np.array(M)
        if abs(np.linalg.det(M)) < 1e-10:
            continue
        x = np.linalg.solve(M, np.array(r))
        ax = A @ x
        ok = np.all(x >= lb - tol) and np.all(x <= ub + tol)
        for i in range(m):
            if sense[i] == "E":
                ok &= abs(ax[i] - b[i]) <= tol
            elif sense[i] == "G":
                ok &= ax[i] >= b[i] - tol
            else:
                ok &= ax[i] <= b[i] + tol
        if ok:
            best = min(best, float(c @ x))
    return best


# ---------------------------------------------------------------------------
# simplex: brute force, duality, certificate, library agreement
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_simplex_matches_vertex_enumeration(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 6))
    mE = int(rng.integers(0, min(2, n - 1) + 1))
    mG = int(rng.integers(0, 4))
    mL = int(rng.integers(0, 2))
    lp, A = random_tiny_lp(rng, n, mE, mG, mL)
    sense = "".join(chr(s) for s in lp.sense)
    ref = brute_force_min(A, lp.b, sense, lp.c, lp.lb, lp.ub)
    res = simplex_solve(lp)
    assert res.status == "optimal"
    assert abs(res.obj - ref) <= 1e-9 * (1 + abs(ref))


def explicit_dual(lp):
    """The dual LP written as a minimisation in the same E/G/bounds form.

    Dual variables: y_E free, y_G >= 0, y_L <= 0, and lam+ >= 0 / lam- >= 0 for
    the finite lower / upper bounds.  One equality row per primal column:
    A'y + lam+ - lam- = c.  Objective: min -(b'y + l'lam+ - u'lam-).
    """
    A = sp.csr_matrix((lp.val, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n)).toarray()
    cols, cost, lo, hi = [], [], [], []
    for i in range(lp.m):
        cols.append(A[i]); cost.append(-lp.b[i])
        s = chr(lp.sense[i])
        lo.append(-np.inf if s in "EL" else 0.0)
        hi.append(np.inf if s in "EG" else 0.0)
    for j in range(lp.n):
        e = np.zeros(lp.n); e[j] = 1.0
        if np.isfinite(lp.lb[j]):
            cols.append(e); cost.append(-lp.lb[j]); lo.append(0.0); hi.append(np.inf)
        if np.isfinite(lp.ub[j]):
            cols.append(-e); cost.append(lp.ub[j]); lo.append(0.0); hi.append(np.inf)
    D = np.array(cols).T
    return dense_lp(D, lp.c, "E" * lp.n, cost, lo, hi)


@pytest.mark.parametrize("seed", range(8))
def test_strong_duality(seed):
    rng = np.random.default_rng(200 + seed)
    lp, _ = random_tiny_lp(rng, int(rng.integers(3, 7)), 1, int(rng.integers(1, 4)), 1)
    # make one variable free to exercise the free-column paths
    lp.lb[0], lp.ub[0] = -np.inf, np.inf
    p = simplex_solve(lp)
    d = simplex_solve(explicit_dual(lp))
    assert p.status == "optimal" and d.status == "optimal"
    assert abs(p.obj + d.obj) <= 1e-9 * (1 + abs(p.obj))


@pytest.mark.parametrize("periods", [4, 12])
def test_simplex_certificate_on_uc(periods):
    lp = make_instance("tiny", 3, n_periods=periods)
    res = simplex_solve(lp)
    assert res.status == "optimal"
    k = kkt(lp, res.x, res.y)
    assert k.rel_kkt <= 1e-9
    assert k.max_primal_violation <= 1e-8


@pytest.mark.slow
def test_simplex_agrees_with_highs_on_tiny_grid():
    lp = make_instance("tiny", 0)
    res = simplex_solve(lp)
    st, obj, x, y, _ = highs_solve(lp, "highs-ds")
    assert res.status == "optimal" and st == 0
    assert abs(res.obj - obj) <= 1e-9 * abs(obj)
    assert kkt(lp, res.x, res.y).rel_kkt <= 1e-9


# ---------------------------------------------------------------------------
# closed forms: merit order and DC network flows
# ---------------------------------------------------------------------------

def single_bus_lp(rng, G, T, su_zero=False):
    pmax = rng.uniform(0.5, 3.0, G)
    units = Units(bus=np.zeros(G, np.int64), pmin=rng.uniform(0.1, 0.4, G) * pmax, pmax=pmax,
                  cost=rng.uniform(10, 60, G), noload=rng.uniform(50, 200, G),
                  startup=np.zeros(G) if su_zero else rng.uniform(100, 500, G), ramp=0.5 * pmax)
    grid = Grid(1, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0), np.zeros(0), 0)
    loads = rng.uniform(0.15, 0.85, (T, 1)) * pmax.sum()
    return units, build_uc_lp(grid, units, loads, 1.0, include_ramp=False), loads


def merit_order(units, demand, dt):
    """Fill Pmax in ascending order of kappa = 100 c dt + (NL dt + SU)/Pmax."""
    kappa = 100.0 * units.cost * dt + (units.noload * dt + units.startup) / units.pmax
    order = np.argsort(kappa)
    left = demand
    obj = 0.0
    price = None
    for g in order:
        take = min(units.pmax[g], left)
        obj += kappa[g] * take
        left -= take
        if left <= 0:
            price = kappa[g]
            break
    return obj, price


@pytest.mark.parametrize("seed", range(6))
def test_single_period_dispatch_is_merit_order(seed):
    rng = np.random.default_rng(300 + seed)
    units, lp, loads = single_bus_lp(rng, int(rng.integers(3, 9)), 1)
    obj, price = merit_order(units, loads[0, 0], 1.0)
    res = simplex_solve(lp)
    assert res.status == "optimal"
    assert abs(res.obj - obj) <= 1e-10 * obj
    bal = lp.meta["period_row_base"][0] + lp.meta["row_off"]["bal"]
    assert abs(res.y[bal] - price) <= 1e-9 * price


@pytest.mark.parametrize("seed", range(3))
def test_multi_period_dispatch_without_startup_cost(seed):
    rng = np.random.default_rng(400 + seed)
    units, lp, loads = single_bus_lp(rng, 5, 4, su_zero=True)
    total = sum(merit_order(units, loads[t, 0], 1.0)[0] for t in range(4))
    res = simplex_solve(lp)
    assert abs(res.obj - total) <= 1e-10 * total


@pytest.mark.parametrize("seed", range(4))
def test_dc_flows_solve_reduced_laplacian(seed):
    rng = np.random.default_rng(500 + seed)
    N = 9
    # spanning tree + two chords, huge thermal limits so no line binds
    frm = [int(rng.integers(0, i)) for i in range(1, N)]
    to = list(range(1, N))
    frm += [0, 3]; to += [5, 8]
    L = len(frm)
    grid = Grid(N, np.array(frm), np.array(to), rng.uniform(5, 20, L), np.full(L, 1e3), N - 1)
    d = rng.uniform(0.1, 0.5, (1, N))
    units = Units(bus=np.array([0]), pmin=np.array([0.1]), pmax=np.array([50.0]),
                  cost=np.array([20.0]), noload=np.array([100.0]), startup=np.array([200.0]),
                  ramp=np.array([25.0]))
    lp = build_uc_lp(grid, units, d, 1.0, include_ramp=False)
    res = simplex_solve(lp)
    assert res.status == "optimal"
    Lap = np.zeros((N, N))
    for l in range(L):
        i, j, B = frm[l], to[l], grid.line_b[l]
        Lap[i, i] += B; Lap[j, j] += B; Lap[i, j] -= B; Lap[j, i] -= B
    theta = np.zeros(N)
    theta[1:] = np.linalg.solve(Lap[1:, 1:], -d[0, 1:])
    flows = grid.line_b * (theta[np.array(frm)] - theta[np.array(to)])
    off = lp.meta["col_off"]
    assert np.allclose(res.x[off["f"]:off["f"] + L], flows, rtol=0, atol=1e-9)
    assert np.allclose(res.x[off["th"]:off["th"] + N], theta, rtol=0, atol=1e-9)
    kappa = 100 * 20.0 + (100.0 + 200.0) / 50.0
    assert abs(res.obj - kappa * d.sum()) <= 1e-10 * res.obj


# ---------------------------------------------------------------------------
# KKT evaluator: hand-computed values
# ---------------------------------------------------------------------------

def test_kkt_hand_values_equality_row():
    lp = dense_lp([[1.0, 1.0]], [1.0], "E", [1.0, 2.0], [0, 0], [1, 1])
    k = kkt(lp, [1.0, 0.0], [1.0])
    assert k.rho_p == 0 and k.rho_d == 0 and k.pobj == 1.0 and k.dobj == 1.0
    k = kkt(lp, [0.5, 0.25], [0.5])
    assert math.isclose(k.rho_p, 0.25) and k.rho_d == 0.0
    assert math.isclose(k.pobj, 1.0) and math.isclose(k.dobj, 0.5)
    assert math.isclose(k.rel_p, 0.25 / 2.0) and math.isclose(k.rel_gap, 0.5 / 2.5)


def test_kkt_hand_values_inequality_and_free():
    lp = dense_lp([[1.0]], [2.0], "G", [1.0], [-np.inf], [np.inf])
    k = kkt(lp, [2.0], [1.0])
    assert k.rel_kkt == 0.0 and k.pobj == 2.0 and k.dobj == 2.0
    k = kkt(lp, [2.0], [-1.0])
    assert math.isclose(k.rho_d, math.sqrt(5.0))
    k = kkt(lp, [1.5], [1.0])
    assert math.isclose(k.rho_p, 0.5)
    # an 'L' row: y <= 0 is dual feasible
    lp = dense_lp([[1.0]], [3.0], "L", [-1.0], [-np.inf], [np.inf])
    k = kkt(lp, [3.0], [-1.0])
    assert k.rel_kkt == 0.0


def test_bound_multiplier_one_sided_hand_values():
    from oracle.kkt import bound_multiplier
    d = np.array([-1.0, 2.0, -3.0, 4.0, 5.0, -6.0, 7.0])
    lb = np.array([0.0, 0.0, -np.inf, -np.inf, -np.inf, 1.0, 1.0])
    ub = np.array([np.inf, np.inf, 5.0, 5.0, np.inf, 2.0, 2.0])
    # only lb finite: max(d, 0); only ub finite: min(d, 0); free: 0; boxed: d
    assert list(bound_multiplier(d, lb, ub)) == [0.0, 2.0, -3.0, 0.0, 0.0, -6.0, 7.0]


def test_kkt_hand_values_one_sided_bounds():
    # min -x1 + x2  s.t.  x1 + x2 = 1,  x1 <= 2 (no lower bound),  x2 >= 0 (no upper
    # bound): optimum x = (1, 0), objective -1, y = -1, reduced costs d = (0, 2)
    lp = dense_lp([[1.0, 1.0]], [1.0], "E", [-1.0, 1.0], [-np.inf, 0.0], [2.0, np.inf])
    k = kkt(lp, [1.0, 0.0], [-1.0])
    assert k.rel_kkt == 0.0 and k.pobj == -1.0 and k.dobj == -1.0
    # y = 0: d = (-1, 1); x1 has only an upper bound, so lam1 = min(-1, 0) = -1
    # enters the dual objective as ub1 * lam1 = -2; x2's lam2 = 1 adds lb2 * 1 = 0
    k = kkt(lp, [1.0, 0.0], [0.0])
    assert k.rho_d == 0.0 and k.dobj == -2.0
    assert math.isclose(k.rel_gap, 1.0 / 4.0)
    # y = -2: d = (1, 3); lam1 = min(1, 0) = 0 leaves a dual residual of 1
    k = kkt(lp, [1.0, 0.0], [-2.0])
    assert k.rho_d == 1.0 and k.dobj == -2.0
    assert math.isclose(k.rel_d, 1.0 / (1.0 + math.sqrt(2.0)))


def one_sided_uc(seed, periods=4):
    """A small UC grid whose line flows lose one of their limits (lower or
    upper, alternating over the lines) and whose units lose the lower bound
    0 of their output (the rows p - Pmin u >= 0 keep p >= 0)."""
    lp = make_instance("tiny", seed, n_periods=periods)
    lb, ub = lp.lb.copy(), lp.ub.copy()
    off, nt, L, G = lp.meta["col_off"], lp.meta["ncol_t"], lp.meta["L"], lp.meta["G"]
    for t in range(lp.meta["T"]):
        f0 = t * nt + off["f"]
        ub[f0:f0 + L:2] = np.inf
        lb[f0 + 1:f0 + L:2] = -np.inf
        p0 = t * nt + off["p"]
        lb[p0:p0 + G] = -np.inf
    return lp.with_data(lb=lb, ub=ub)


def test_simplex_on_one_sided_columns_agrees_with_highs():
    # columns bounded on one side only are negated or kept by the simplex's
    # set-up; HiGHS (a separate library) must find the same optimum, and the
    # KKT evaluator's one-sided branches must certify the simplex point
    lp = one_sided_uc(3)
    res = simplex_solve(lp)
    assert res.status == "optimal"
    st, obj, x, y, _ = highs_solve(lp, "highs-ds")
    assert st == 0
    assert abs(res.obj - obj) <= 1e-9 * (1 + abs(obj))
    k = kkt(lp, res.x, res.y)
    assert k.rel_kkt <= 1e-9
    lbo, ubo = np.isfinite(lp.lb) & ~np.isfinite(lp.ub), np.isfinite(lp.ub) & ~np.isfinite(lp.lb)
    assert lbo.sum() > 0 and ubo.sum() > 0
    # relaxing limits cannot raise the optimum
    base = simplex_solve(make_instance("tiny", 3, n_periods=4))
    assert res.obj <= base.obj + 1e-9 * abs(base.obj)


def test_kkt_detects_flipped_dual_sign():
    lp = make_instance("tiny", 1, n_periods=3)
    res = simplex_solve(lp)
    assert kkt(lp, res.x, res.y).rel_kkt < 1e-9
    assert kkt(lp, res.x, -res.y).rel_kkt > 1e-2


# ---------------------------------------------------------------------------
# single steps of the method
# ---------------------------------------------------------------------------

def random_csr(rng, m, n, density=0.3, empty_rows=()):
    A = sp.random(m, n, density=density, random_state=rng, format="csr")
    A.data = rng.normal(size=A.data.shape)
    A = A.tolil()
    for r in empty_rows:
        A[r, :] = 0
    A = A.tocsr()
    A.eliminate_zeros()
    A.sort_indices()
    return A


def test_transpose_matches_dense_and_is_row_stable():
    rng = np.random.default_rng(7)
    A = random_csr(rng, 40, 23, 0.2, empty_rows=(3, 17))
    tp, tc, tv = ps.csr_transpose(A.indptr, A.indices, A.data, 23)
    T = sp.csr_matrix((tv, tc, tp), shape=(23, 40)).toarray()
    assert np.array_equal(T, A.toarray().T)
    for j in range(23):
        seg = tc[tp[j]:tp[j + 1]]
        assert np.all(np.diff(seg) > 0)


def test_matvec_matches_dense_and_exact_sum():
    rng = np.random.default_rng(8)
    A = random_csr(rng, 50, 31, 0.3, empty_rows=(0, 49))
    x = rng.normal(size=31)
    y = ps.csr_matvec(A.indptr, A.indices, A.data, x)
    assert np.allclose(y, A.toarray() @ x, rtol=1e-14, atol=1e-14)
    for i in (1, 10, 25):
        ks = range(A.indptr[i], A.indptr[i + 1])
        exact = math.fsum(A.data[k] * x[A.indices[k]] for k in ks)
        assert abs(y[i] - exact) <= 4 * np.finfo(float).eps * sum(abs(A.data[k] * x[A.indices[k]]) for k in ks)


def test_ruiz_equilibrates_diagonal_in_one_pass():
    d = np.array([4.0, 0.25, 9.0, 1e-4])
    Dr, Dc, M = ps.ruiz_pc_scaling(sp.csr_matrix(np.diag(d)), ruiz_iters=1, pock_chambolle=False)
    assert np.allclose(M.toarray(), np.eye(4), rtol=1e-15)


def test_ruiz_converges_and_pc_bounds_norm():
    rng = np.random.default_rng(9)
    A = random_csr(rng, 60, 45, 0.15) * 100.0
    A = sp.diags(rng.uniform(0.01, 100, 60)) @ A
    Dr, Dc, M = ps.ruiz_pc_scaling(A, ruiz_iters=30, pock_chambolle=False)
    Ma = abs(M)
    rmax = Ma.max(axis=1).toarray().ravel()
    cmax = Ma.max(axis=0).toarray().ravel()
    assert np.allclose(rmax[rmax > 0], 1.0, atol=1e-3) and np.allclose(cmax[cmax > 0], 1.0, atol=1e-3)
    Dr, Dc, M = ps.ruiz_pc_scaling(A, ruiz_iters=10, pock_chambolle=True)
    assert ps.spectral_norm(M) <= 1.0 + 1e-12
    # the scaled matrix is D_r A D_c
    assert np.allclose(M.toarray(), np.diag(Dr) @ A.toarray() @ np.diag(Dc), rtol=1e-13, atol=0)
    # a constant matrix reaches the Pock-Chambolle bound exactly
    Dr, Dc, M = ps.ruiz_pc_scaling(sp.csr_matrix(np.full((5, 7), 3.0)), 0, True)
    assert math.isclose(ps.spectral_norm(M), 1.0, rel_tol=1e-12)


def test_spectral_norm_known_values():
    rng = np.random.default_rng(10)
    Q1, _ = np.linalg.qr(rng.normal(size=(8, 8)))
    Q2, _ = np.linalg.qr(rng.normal(size=(6, 6)))
    S = np.zeros((8, 6)); S[:6, :6] = np.diag([3.5, 2, 1, 0.5, 0.1, 0.01])
    assert math.isclose(ps.spectral_norm(sp.csr_matrix(Q1 @ S @ Q2.T)), 3.5, rel_tol=1e-12)
    big = sp.random(900, 700, density=0.01, random_state=3, format="csr")
    assert math.isclose(ps.spectral_norm(big), np.linalg.norm(big.toarray(), 2), rel_tol=1e-8)


def scaled_internal_optimum(lp):
    res = simplex_solve(lp)
    ip = ps.internal_problem(lp)
    A = ip.matrix()
    Dr, Dc, Ah = ps.ruiz_pc_scaling(A)
    x = res.x[ip.col_map] / Dc
    y = np.array([res.y[r] if r >= 0 else -res.y[-r - 1] for r in ip.row_map]) / Dr
    return ip, Dr, Dc, Ah, x, y


def test_pdhg_step_fixed_point_at_lp_optimum():
    lp = make_instance("tiny", 2, n_periods=3)
    ip, Dr, Dc, Ah, x, y = scaled_internal_optimum(lp)
    c, b, l, u = ip.c * Dc, ip.b * Dr, ip.l / Dc, ip.u / Dc
    for tau, sigma in ((0.3, 2.0), (1e-3, 50.0)):
        xh, yh = ps.pdhg_step(Ah, c, b, l, u, ip.m_eq, x, y, tau, sigma)
        assert np.max(np.abs(xh - x)) <= 1e-8 * (1 + np.max(np.abs(x)))
        assert np.max(np.abs(yh - y)) <= 1e-8 * (1 + np.max(np.abs(y)))
        assert ps.fixed_point_residual(Ah, x, y, xh, yh, tau, sigma) <= 1e-6
    # a perturbed point is not fixed and moves toward feasibility of its bounds
    xp = x + 0.1
    xh, yh = ps.pdhg_step(Ah, c, b, l, u, ip.m_eq, xp, y, 0.3, 2.0)
    assert np.all(xh >= l) and np.all(xh <= u) and np.all(yh[ip.m_eq:] >= 0)
    assert np.max(np.abs(xh - xp)) > 1e-3


def test_pdhg_step_one_dimensional_hand_values():
    # min 2x s.t. x >= 1 (G), 0 <= x <= 5; from x = 3, y = 0.5, tau = 0.5, sigma = 2
    A = sp.csr_matrix(np.array([[1.0]]))
    xh, yh = ps.pdhg_step(A, np.array([2.0]), np.array([1.0]), np.array([0.0]), np.array([5.0]),
                          0, np.array([3.0]), np.array([0.5]), 0.5, 2.0)
    # x_hat = 3 - 0.5 (2 - 0.5) = 2.25 ; y_hat = max(0, 0.5 + 2 (1 - (4.5 - 3))) = 0
    assert xh[0] == 2.25 and yh[0] == 0.0
    z = ps.halpern_update(np.array([3.0]), np.array([2.25]), np.array([1.0]), 0)
    assert z[0] == 0.5 * (4.5 - 3.0) + 0.5 * 1.0


@pytest.mark.parametrize("gamma", [0.0, 0.5, 1.0])
def test_halpern_iteration_converges_to_anchor_projection(gamma):
    # T = projection onto a box is firmly nonexpansive, so (1 + gamma) T - gamma I
    # is nonexpansive for gamma in [0, 1] with the same fixed points (the box);
    # Halpern's iteration anchored at z0 then tends to the point of the box
    # nearest z0, at rate O(1/k) in the residual.
    rng = np.random.default_rng(int(gamma * 10))
    lo, hi = -np.ones(40), np.ones(40)
    z0 = 3 * rng.normal(size=40)
    z = z0.copy()
    for k in range(4000):
        z = ps.halpern_update(z, np.clip(z, lo, hi), z0, k, gamma)
    assert np.max(np.abs(z - np.clip(z0, lo, hi))) < 2e-2
    assert np.max(np.abs(z - np.clip(z, lo, hi))) < 5e-3
    # a dropped anchor term ends at a different point
    z = z0.copy()
    for k in range(4000):
        w = (k + 1.0) / (k + 2.0)
        z = w * ((1 + gamma) * np.clip(z, lo, hi) - gamma * z)
    assert np.max(np.abs(z - np.clip(z0, lo, hi))) > 0.1


def test_internal_problem_maps_and_offsets():
    lp = dense_lp([[1, 2, 0], [0, 0, 0], [3, 0, 1], [1, 1, 1]], [4, 0, 2, 9], "GEEL",
                  [1, 1, 1], [0, 2, -np.inf], [5, 2, np.inf])
    ip = ps.internal_problem(lp)
    assert list(ip.col_map) == [0, 2]
    assert list(ip.row_map) == [2, 0, -4]          # E rows first, then G, then negated L
    assert ip.m_eq == 1
    assert np.allclose(ip.b, [2 - 0, 4 - 4, -(9 - 2)])
    assert ip.obj_offset == 2.0
    assert np.allclose(ip.matrix().toarray(), [[3, 1], [1, 0], [-1, -1]])


def p_norm(A, ux, uy, tau, sigma):
    """||(ux, uy)||_P through the oracle's residual with z = 0, T(z) = u."""
    return ps.fixed_point_residual(A, np.zeros_like(ux), np.zeros_like(uy), ux, uy, tau, sigma)


def test_fixed_point_residual_hand_values_with_cross_term():
    # A = [[2]], dz = (1, 3), tau = 1/2, sigma = 1/4:
    # 1/0.5 + 9/0.25 + 2 * 3 * (2 * 1) = 2 + 36 + 12 = 50
    A = sp.csr_matrix(np.array([[2.0]]))
    assert math.isclose(p_norm(A, np.array([1.0]), np.array([3.0]), 0.5, 0.25), math.sqrt(50.0))
    # A = [[1, 0, 2], [0, -1, 1]], dx = (1, 2, -1), dy = (0.5, -1): A dx = (-1, -3),
    # dy'A dx = 2.5; tau = 2, sigma = 1/2: 6/2 + 1.25/0.5 + 2 * 2.5 = 10.5
    A = sp.csr_matrix(np.array([[1.0, 0.0, 2.0], [0.0, -1.0, 1.0]]))
    r = ps.fixed_point_residual(A, np.array([1.0, 1.0, 1.0]), np.array([0.0, 1.0]),
                                np.array([2.0, 3.0, 0.0]), np.array([0.5, 0.0]), 2.0, 0.5)
    assert math.isclose(r, math.sqrt(10.5))


def firm_nonexpansiveness_excess(residual, trials=200, seed=0):
    """Largest relative excess of ||Tz - Tz'||^2 + ||(I-T)z - (I-T)z'||^2 over
    ||z - z'||^2 in the norm `residual` measures, over random small LPs, step
    pairs with tau sigma ||A||^2 < 1, and point pairs."""
    rng = np.random.default_rng(seed)
    worst = -np.inf
    for _ in range(trials):
        m, n, meq = 4, 5, 2
        A = sp.csr_matrix(rng.normal(size=(m, n)))
        nrm = np.linalg.svd(A.toarray(), compute_uv=False)[0]
        tau = 0.9 / nrm * rng.uniform(0.3, 3.0)
        sigma = 0.9 / (nrm * nrm * tau)
        c, b = rng.normal(size=n), rng.normal(size=m)
        l, u = -rng.uniform(0, 1, n), rng.uniform(0, 1, n)
        z = [(rng.normal(size=n), rng.normal(size=m)) for _ in range(2)]
        T = [ps.pdhg_step(A, c, b, l, u, meq, x, y, tau, sigma) for x, y in z]

        def nsq(ux, uy):
            return residual(A, np.zeros(n), np.zeros(m), ux, uy, tau, sigma) ** 2

        lhs = nsq(T[0][0] - T[1][0], T[0][1] - T[1][1]) + \
            nsq((z[0][0] - T[0][0]) - (z[1][0] - T[1][0]), (z[0][1] - T[0][1]) - (z[1][1] - T[1][1]))
        rhs = nsq(z[0][0] - z[1][0], z[0][1] - z[1][1])
        worst = max(worst, (lhs - rhs) / rhs)
    return worst


def test_fixed_point_residual_is_the_metric_of_the_step():
    # the PDHG step is a proximal-point step, hence firmly nonexpansive, in the
    # metric the residual measures; the restart test relies on that
    assert firm_nonexpansiveness_excess(ps.fixed_point_residual) <= 1e-12


# ---------------------------------------------------------------------------
# planted mistakes in the oracle are caught by the pins above
# ---------------------------------------------------------------------------

def test_planted_step_mistakes_break_the_fixed_point():
    lp = make_instance("tiny", 2, n_periods=3)
    ip, Dr, Dc, Ah, x, y = scaled_internal_optimum(lp)
    c, b, l, u = ip.c * Dc, ip.b * Dr, ip.l / Dc, ip.u / Dc

    def no_extrapolation(x, y, tau, sigma):
        xh = ps.project_box(x - tau * (c - Ah.T @ y), l, u)
        return xh, ps.project_dual(y + sigma * (b - Ah @ xh) + 0.0 * x.sum(), ip.m_eq)

    def wrong_sign(x, y, tau, sigma):
        xh = ps.project_box(x - tau * (c + Ah.T @ y), l, u)
        return xh, ps.project_dual(y + sigma * (b - Ah @ (2 * xh - x)), ip.m_eq)

    # extrapolation alone does not move the fixed point; the sign does
    xh, yh = no_extrapolation(x, y, 0.3, 2.0)
    assert np.max(np.abs(xh - x)) <= 1e-8 * (1 + np.max(np.abs(x)))
    xh, yh = wrong_sign(x, y, 0.3, 2.0)
    assert np.max(np.abs(xh - x)) > 1e-3


def test_planted_sign_of_the_residual_cross_term_is_caught():
    # the residual with the cross term's sign flipped is still a norm (for
    # tau sigma ||A||^2 < 1) but the step is not nonexpansive in it, and the
    # hand values differ
    def flipped(A, x, y, x_hat, y_hat, tau, sigma):
        dx, dy = x_hat - x, y_hat - y
        return math.sqrt(max(dx @ dx / tau + dy @ dy / sigma - 2.0 * dy @ (A @ dx), 0.0))

    assert firm_nonexpansiveness_excess(flipped) > 1e-2
    A = sp.csr_matrix(np.array([[2.0]]))
    assert not math.isclose(flipped(A, np.zeros(1), np.zeros(1), np.ones(1), np.full(1, 3.0), 0.5, 0.25),
                            math.sqrt(50.0))

