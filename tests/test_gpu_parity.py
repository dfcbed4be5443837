"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every input is a seeded synthetic instance; every expected value comes from
oracle/ (at run time, or stored in tests/golden/objectives.json by
tests/golden/make_golden.py)."""

import json
import math
import os
import sys
import time

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import pdhg_steps as ps
from oracle.kkt import kkt
from oracle.simplex import simplex_solve
from paper_2607_03627_amd import uclp
from paper_2607_03627_amd.instances import LP, make_instance

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "objectives.json")))
U32 = np.finfo(np.float32).eps / 2
U64 = np.finfo(np.float64).eps / 2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _lib():
    uclp.load()


class Handle:
    def __init__(self, lp, **opts):
        self.lp = lp
        self.h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(**opts))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        uclp.uc_lp_destroy(self.h)


def internal_oracle(lp):
    ip = ps.internal_problem(lp)
    A = ip.matrix()
    Dr, Dc, Ah = ps.ruiz_pc_scaling(A)
    return ip, A, Dr, Dc, Ah


_FULL = {}


def full_size_case():
    """The 6,049-bus-shaped LP the benchmark times, with the oracle's internal
    problem and scaling, built once per test session."""
    if not _FULL:
        lp = make_instance("large", 0)
        _FULL["lp"] = lp
        _FULL["oracle"] = internal_oracle(lp)
    return _FULL["lp"], _FULL["oracle"]


def ragged_instance(seed):
    """The 30-bus LP with one dense row (sum of all columns <= 1e6) and one
    dense column (0.01 in every row, cost 50, bounds [0, 1]): a row of A and a
    row of A^T longer than one LDS tile, next to the short UC rows."""
    base = make_instance("tiny", seed)
    m, n = base.m, base.n
    rows = [base.col_idx[base.row_ptr[i]:base.row_ptr[i + 1]] for i in range(m)]
    vals = [base.val[base.row_ptr[i]:base.row_ptr[i + 1]] for i in range(m)]
    cols = [np.append(r, n) for r in rows] + [np.arange(n + 1)]
    vs = [np.append(v, 0.01) for v in vals] + [np.append(np.ones(n), 0.01)]
    rp = np.zeros(m + 2, np.int32)
    rp[1:] = np.cumsum([len(r) for r in cols])
    return LP(m=m + 1, n=n + 1, row_ptr=rp, col_idx=np.concatenate(cols).astype(np.int32),
              val=np.concatenate(vs), c=np.append(base.c, 50.0), b=np.append(base.b, 1e6),
              sense=np.append(base.sense, np.uint8(ord("L"))), lb=np.append(base.lb, 0.0),
              ub=np.append(base.ub, 1.0))


def one_sided_instance(seed, periods=24):
    """The 30-bus LP whose line flows keep only one limit (upper or lower,
    alternating over the lines) and whose unit outputs lose their lower bound
    0 (the rows p - Pmin u >= 0 still keep p >= 0): columns with only a lower
    bound and columns with only an upper bound, next to boxed and free ones."""
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


def instance_and_oracle(shape, seed):
    if shape == "large":
        assert seed == 0
        return full_size_case()
    if shape == "ragged":
        lp = ragged_instance(seed)
    elif shape == "one_sided":
        lp = one_sided_instance(seed)
    else:
        lp = make_instance(shape, seed)
    return lp, internal_oracle(lp)


# ---------------------------------------------------------------------------
# a1 presolve + transpose, a2 scaling, a3 operator norm
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape,seed", [("tiny", 0), ("medium", 1), ("large", 0)])
def test_presolve_and_transpose_bit_exact(shape, seed):
    say("case", shape, seed)
    lp, (ip, _, _, _, _) = instance_and_oracle(shape, seed)
    with Handle(lp) as H:
        d = uclp.uc_lp_internal_dims(H.h)
        assert (d["m"], d["n"], d["nnz"], d["m_eq"]) == (ip.m, ip.n, len(ip.col_idx), ip.m_eq)
        assert np.array_equal(d["row_map"], ip.row_map) and np.array_equal(d["col_map"], ip.col_map)
        tp, tc, tv = uclp.uc_lp_get_transpose(H.h, d["n"], d["nnz"])
    rp, rc, rv = ps.csr_transpose(ip.row_ptr, ip.col_idx, ip.val, ip.n)
    assert np.array_equal(tp, rp) and np.array_equal(tc, rc)
    assert np.array_equal(tv, rv)


@pytest.mark.parametrize("shape,seed", [("tiny", 0), ("medium", 0)])
def test_scaling_and_operator_norm(shape, seed):
    lp = make_instance(shape, seed)
    say("case", shape, seed)
    ip, A, Dr, Dc, Ah = internal_oracle(lp)
    with Handle(lp) as H:
        dr, dc, nrm = uclp.uc_lp_get_scaling(H.h, ip.m, ip.n)
    assert np.max(np.abs(dr / Dr - 1)) <= 1e-12
    assert np.max(np.abs(dc / Dc - 1)) <= 1e-12
    true = ps.spectral_norm(Ah)
    # power iteration approaches the largest singular value from below
    assert nrm <= true * (1 + 1e-10)
    assert nrm >= 0.97 * true
    assert true <= 1 + 1e-12      # the Pock-Chambolle bound
    check_step_bound(lp, true)


def check_step_bound(lp, sigma1):
    """The step comes from an upper bound on ||A_hat||_2: tau sigma sigma1^2 < 1."""
    x, y, info = solve(lp, precision=uclp.UC_LP_FP64, iter_limit=64, eps_rel=1e-12)
    bound, eta, est = info["norm_a_bound"], info["eta"], info["norm_a_est"]
    say("  sigma1", sigma1, "estimate", est, "bound", bound, "eta", eta)
    assert bound >= sigma1 * (1 - 1e-12) and bound <= 1 + 1e-12
    assert est <= bound
    tau, sigma = eta / info["omega"], eta * info["omega"]
    assert tau * sigma * sigma1 ** 2 < 1.0
    assert math.isclose(eta, 0.99 / bound, rel_tol=1e-15)


# ---------------------------------------------------------------------------
# a4-a6: one PDHG step with the Halpern update
# ---------------------------------------------------------------------------

def step_inputs(ip, Dc, Dr, seed):
    rng = np.random.default_rng(seed)
    l, u = ip.l / Dc, ip.u / Dc
    x = np.clip(rng.normal(0, 1, ip.n), l, u)
    x0 = np.clip(rng.normal(0, 1, ip.n), l, u)
    y = rng.normal(0, 1, ip.m)
    y[ip.m_eq:] = np.abs(y[ip.m_eq:])
    y0 = rng.normal(0, 1, ip.m)
    y0[ip.m_eq:] = np.abs(y0[ip.m_eq:])
    return x, y, x0, y0


@pytest.mark.parametrize("shape,seed,gamma", [("tiny", 1, 1.0), ("medium", 2, 1.0), ("tiny", 3, 0.5), ("ragged", 0, 1.0),
                                              ("large", 0, 1.0)])
@pytest.mark.parametrize("prec", [uclp.UC_LP_FP64, uclp.UC_LP_FP32_MIXED])
def test_pdhg_step_elementwise(shape, seed, gamma, prec):
    # ("large", 0) is the benchmark's full-size LP: every one of its 3.2M + 3.0M
    # step outputs is compared with the oracle's
    say("case", shape, seed, gamma, prec)
    lp, (ip, A, Dr, Dc, Ah) = instance_and_oracle(shape, seed)
    c, b, l, u = ip.c * Dc, ip.b * Dr, ip.l / Dc, ip.u / Dc
    x, y, x0, y0 = step_inputs(ip, Dc, Dr, seed)
    tau, sigma, k = 0.37, 1.9, 5
    with Handle(lp, halpern_gamma=gamma) as H:
        xh, yh, xn, yn = uclp.uc_lp_debug_step(H.h, prec, x, y, x0, y0, k, tau, sigma)
        _, gdc, _ = uclp.uc_lp_get_scaling(H.h, ip.m, ip.n)
    # the kernels project onto their own scaled bounds l / D_c, u / D_c
    gl, gu = ip.l / gdc, ip.u / gdc
    if prec == uclp.UC_LP_FP32_MIXED:
        gl, gu = gl.astype(np.float32).astype(float), gu.astype(np.float32).astype(float)
    if prec == uclp.UC_LP_FP32_MIXED:
        # the FP32 path works on FP32-rounded inputs and data
        f = lambda v: v.astype(np.float32).astype(np.float64)
        x, y, x0, y0, c, b, l, u = map(f, (x, y, x0, y0, c, b, l, u))
        Ah = sp.csr_matrix((f(Ah.data), Ah.indices, Ah.indptr), shape=Ah.shape)
    rx, ry = ps.pdhg_step(Ah, c, b, l, u, ip.m_eq, x, y, tau, sigma)
    rxn = ps.halpern_update(x, rx, x0, k, gamma)
    ryn = ps.halpern_update(y, ry, y0, k, gamma)
    absA = abs(Ah)
    rowlen = np.diff(Ah.indptr).max()
    if prec == uclp.UC_LP_FP64:
        # scaled data differ from the oracle's in the last bits of D_r, D_c
        ex = 1e-12 * (np.abs(x) + tau * (np.abs(c) + absA.T @ np.abs(y)) + 1)
        ey = 1e-12 * (np.abs(y) + sigma * (np.abs(b) + absA @ (2 * np.abs(rx) + np.abs(x))) + 1)
    else:
        g = (rowlen + 4) * U32
        ex = 4 * g * (np.abs(x) + tau * (np.abs(c) + absA.T @ np.abs(y))) + 1e-30
        exb = 2 * ex + U32 * (2 * np.abs(rx) + np.abs(x))
        ey = 4 * g * (np.abs(y) + sigma * (np.abs(b) + absA @ (2 * np.abs(rx) + np.abs(x)))) \
            + sigma * (absA @ exb) + 1e-30
    assert np.all(np.abs(xh - rx) <= ex)
    assert np.all(np.abs(yh - ry) <= ey)
    w = (k + 1) / (k + 2)
    assert np.all(np.abs(xn - rxn) <= 2 * w * ex + 4 * U32 * (np.abs(rxn) + np.abs(x) + np.abs(x0)) + 1e-30)
    assert np.all(np.abs(yn - ryn) <= 2 * w * ey + 4 * U32 * (np.abs(ryn) + np.abs(y) + np.abs(y0)) + 1e-30)
    # projections hold exactly
    assert np.all(xh >= gl) and np.all(xh <= gu) and np.all(yh[ip.m_eq:] >= 0)


def step_with_bounds(Ah, absA, c, b, l, u, m_eq, x, y, x0, y0, k, tau, sigma, gamma, fp32, dx, dy):
    """One oracle step (pdhg_step, then the Halpern update toward the anchor)
    from (x, y), with elementwise bounds on how far an implementation may be
    from it when its own input is within (dx, dy) of (x, y) and it rounds
    within the forward-error bounds of test_pdhg_step_elementwise: the input
    error carried through the step (projections are 1-Lipschitz elementwise,
    products are bounded by |A|) plus the step's own rounding."""
    rowlen = np.diff(Ah.indptr).max()
    xh, yh = ps.pdhg_step(Ah, c, b, l, u, m_eq, x, y, tau, sigma)
    ax, ay = np.abs(x) + dx, np.abs(y) + dy
    if fp32:
        g = (rowlen + 4) * U32
        lx = 4 * g * (ax + tau * (np.abs(c) + absA.T @ ay)) + 1e-30
        ly = 4 * g * (ay + sigma * (np.abs(b) + absA @ (2 * np.abs(xh) + ax))) \
            + sigma * (absA @ (U32 * (2 * np.abs(xh) + ax))) + 1e-30
        uh = 8 * U32
    else:
        lx = 1e-12 * (ax + tau * (np.abs(c) + absA.T @ ay) + 1)
        ly = 1e-12 * (ay + sigma * (np.abs(b) + absA @ (2 * np.abs(xh) + ax)) + 1)
        uh = 1e-13
    exh = dx + tau * (absA.T @ dy) + lx
    eyh = dy + sigma * (absA @ (2 * exh + dx)) + ly
    w = (k + 1.0) / (k + 2.0)
    xn = ps.halpern_update(x, xh, x0, k, gamma)
    yn = ps.halpern_update(y, yh, y0, k, gamma)
    exn = w * ((1 + gamma) * exh + gamma * dx) + uh * (2 * np.abs(xh) + ax + np.abs(x0) + np.abs(xn))
    eyn = w * ((1 + gamma) * eyh + gamma * dy) + uh * (2 * np.abs(yh) + ay + np.abs(y0) + np.abs(yn))
    return dict(xh=xh, yh=yh, exh=exh, eyh=eyh, xn=xn, yn=yn, exn=exn, eyn=eyn)


@pytest.mark.parametrize("shape,seed,gamma,threads", [
    ("tiny", 1, 1.0, 256), ("tiny", 1, 1.0, 512), ("tiny", 3, 0.5, 256), ("tiny", 3, 0.5, 512),
    ("ragged", 0, 1.0, 256), ("ragged", 0, 1.0, 512), ("ragged", 0, 0.5, 512),
    ("medium", 2, 1.0, 256), ("medium", 2, 1.0, 512), ("medium", 2, 0.5, 256),
    ("large", 0, 1.0, 256), ("large", 0, 1.0, 512)])
@pytest.mark.parametrize("prec", [uclp.UC_LP_FP64, uclp.UC_LP_FP32_MIXED])
def test_consecutive_iterations_elementwise(shape, seed, gamma, threads, prec):
    # Runs of J = 1..4 iterations launched as one check interval launches
    # them: J - 1 non-check iterations (the Halpern step inside the half-step
    # kernels; with gamma = 1 the primal iterate rebuilt from x_bar and the
    # anchor), then a check iteration, the FP64 check kernels and the finish
    # kernel.  Run J's check iteration sees the iterate the non-check kernels
    # produced at step J - 1; run J - 1's finish kernel produced the same
    # iterate by another code path.  Each run is compared element by element
    # with one oracle step from run J - 1's iterate (the inputs for J = 1),
    # allowing a few ulps between the two paths, in both workgroup shapes;
    # so is the fixed-point residual of the restart test.
    say("case iterate", shape, seed, gamma, threads, prec)
    lp, (ip, A, Dr, Dc, Ah) = instance_and_oracle(shape, seed)
    c, b, l, u = ip.c * Dc, ip.b * Dr, ip.l / Dc, ip.u / Dc
    x, y, x0, y0 = step_inputs(ip, Dc, Dr, seed)
    tau, sigma, k = 0.37, 1.9, 3
    fp32 = prec == uclp.UC_LP_FP32_MIXED
    f = (lambda v: v.astype(np.float32).astype(np.float64)) if fp32 else (lambda v: v)
    runs = []
    with Handle(lp, halpern_gamma=gamma) as H:
        for J in range(1, 5):
            runs.append(uclp.uc_lp_debug_iterate(H.h, prec, J, x, y, x0, y0, k, tau, sigma,
                                                 block_threads=threads))
    x, y, x0, y0, c, b, l, u = map(f, (x, y, x0, y0, c, b, l, u))
    Ah = sp.csr_matrix((f(Ah.data), Ah.indices, Ah.indptr), shape=Ah.shape)
    absA = abs(Ah)
    uu = 4 * U32 if fp32 else 4 * U64
    zx, zy = x, y
    dx, dy = np.zeros_like(x), np.zeros_like(y)
    for J, (xh, yh, xn, yn, rfp) in enumerate(runs, start=1):
        r = step_with_bounds(Ah, absA, c, b, l, u, ip.m_eq, zx, zy, x0, y0, k + J - 1, tau, sigma, gamma, fp32,
                             dx, dy)
        assert np.all(np.abs(xh - r["xh"]) <= r["exh"]), J
        assert np.all(np.abs(yh - r["yh"]) <= r["eyh"]), J
        assert np.all(np.abs(xn - r["xn"]) <= r["exn"]), J
        assert np.all(np.abs(yn - r["yn"]) <= r["eyn"]), J
        # the residual is a norm of T(z) - z: it moves by at most the norm of
        # the bounds on T(z) and z (|e_y'A e_x| <= e_y'|A| e_x)
        ro = ps.fixed_point_residual(Ah, zx, zy, r["xh"], r["yh"], tau, sigma)
        ex, ey = r["exh"] + dx, r["eyh"] + dy
        tol = math.sqrt(ex @ ex / tau + ey @ ey / sigma + 2 * ey @ (absA @ ex)) + 1e-12 * ro
        assert abs(rfp - ro) <= tol, (J, rfp, ro, tol)
        # a Halpern weight taken one step late is outside the bounds
        p = step_with_bounds(Ah, absA, c, b, l, u, ip.m_eq, zx, zy, x0, y0, k + J, tau, sigma, gamma, fp32,
                             dx, dy)
        assert np.any(np.abs(xn - p["xn"]) > p["exn"]) or np.any(np.abs(yn - p["yn"]) > p["eyn"]), J
        # the next run's check iteration starts from the non-check kernels'
        # own Halpern step: the same formula in the same precision, so the two
        # paths differ by a few ulps at most
        zx, zy = xn, yn
        dx = uu * (np.abs(xn) + np.abs(xh) + np.abs(x0))
        dy = uu * (np.abs(yn) + np.abs(yh) + np.abs(y0))


# ---------------------------------------------------------------------------
# a7: the FP64 KKT check kernels
# ---------------------------------------------------------------------------

def test_full_size_scaling():
    # D_r, D_c of the benchmark's LP against the oracle's; the power-iteration
    # estimate stays below the Pock-Chambolle bound of the scaled matrix
    lp, (ip, A, Dr, Dc, Ah) = full_size_case()
    say("case large 0 scaling")
    with Handle(lp) as H:
        dr, dc, nrm = uclp.uc_lp_get_scaling(H.h, ip.m, ip.n)
    assert np.max(np.abs(dr / Dr - 1)) <= 1e-12
    assert np.max(np.abs(dc / Dc - 1)) <= 1e-12
    assert 0.5 < nrm <= 1 + 1e-12
    true = ps.spectral_norm(Ah)
    say("  ARPACK sigma1", true)
    assert nrm <= true * (1 + 1e-8)
    check_step_bound(lp, true)


def test_full_size_solve_in_the_benchmark_configuration():
    # the benchmark's solve (FP32 iterates, FP64 checks, stop at 1e-4, event
    # timing on); the oracle recomputes the KKT error of the returned point
    lp, _ = full_size_case()
    say("case large 0 solve")
    x, y, info = solve(lp, precision=uclp.UC_LP_FP32_MIXED, eps_rel=1e-4, timing=1)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    k = kkt(lp, x, y)
    say("large rel_kkt", k.rel_kkt, info["rel_kkt"], k.pobj, "iters", info["iters"])
    assert k.rel_kkt <= 1e-4 * 1.001
    assert abs(k.rel_kkt - info["rel_kkt"]) <= 1e-6
    assert np.all(x >= lp.lb) and np.all(x <= lp.ub)
    assert info["primal_kernel_us"] > 0 and info["dual_kernel_us"] > 0


def test_full_size_objective_matches_oracle():
    # The 1e-4 point of the benchmark is ~2e-5 away from the optimum in
    # objective, and at 1e-5 relative KKT the FP64 iterates of this LP were
    # still 5e-7 - 2e-6 away; FP32 to 1e-4 followed by FP64 to 5e-6 returns a
    # point whose objective matches the oracle's optimum within 1e-6 (inside
    # the paper's 100,000-iteration limit)
    lp, _ = full_size_case()
    if "large/0" not in GOLDEN:
        pytest.skip("no stored oracle objective for the 6,049-bus LP (tests/golden/make_golden.py --large)")
    z = GOLDEN["large/0"]["obj"]
    say("case large 0 objective")
    x, y, info = solve(lp, precision=uclp.UC_LP_FP32_MIXED_POLISH, eps_rel=1e-4, eps_polish=5e-6)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    k = kkt(lp, x, y)
    say("  oracle", z, "returned", k.pobj, abs(k.pobj - z) / abs(z), "at 1e-4", info["pobj_at_eps"],
        abs(info["pobj_at_eps"] - z) / abs(z), "iters", info["iters"], info["iters_fp64"], info["t_total_s"])
    assert k.rel_kkt <= 5e-6 * 1.001
    assert abs(k.pobj - z) <= 1e-6 * abs(z)


def kkt_points(lp, shape, rng):
    """Points at which the check kernels are compared: the simplex optimum and
    perturbations of it on the 30-bus grids, random points (bounds respected
    where finite, inequality duals of either sign) on the larger ones."""
    fixed = lp.lb == lp.ub
    if shape in ("tiny", "one_sided"):
        res = simplex_solve(lp)
        assert res.status == "optimal"
        for scale in (0.0, 1e-6, 1e-2):
            x = np.clip(res.x + scale * rng.normal(size=lp.n), lp.lb, lp.ub)
            x[fixed] = lp.lb[fixed]
            yield x, res.y + scale * rng.normal(size=lp.m)
        return
    lo = np.where(np.isfinite(lp.lb), lp.lb, -5.0)
    hi = np.where(np.isfinite(lp.ub), lp.ub, 5.0)
    for _ in range(2):
        x = lo + rng.random(lp.n) * (hi - lo)
        x[fixed] = lp.lb[fixed]
        yield x, rng.normal(0.0, 50.0, lp.m)


@pytest.mark.parametrize("shape,seed", [("tiny", 0), ("one_sided", 2), ("medium", 1), ("large", 0)])
def test_kkt_kernels_match_oracle(shape, seed):
    # every scalar of the FP64 check kernels (residual norms, objectives with
    # the bound-multiplier terms of boxed, one-sided and free columns, the
    # largest row violation) against the oracle's KKT evaluator
    lp = full_size_case()[0] if shape == "large" else (
        one_sided_instance(seed) if shape == "one_sided" else make_instance(shape, seed))
    say("case kkt", shape, seed)
    rng = np.random.default_rng(3)
    A = sp.csr_matrix((lp.val, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))
    absA = abs(A)
    nb, nc = np.linalg.norm(lp.b), np.linalg.norm(lp.c)
    with Handle(lp) as H:
        for x, y in kkt_points(lp, shape, rng):
            g = uclp.uc_lp_eval_kkt(H.h, x, y)
            o = kkt(lp, x, y)
            sp_scale = np.linalg.norm(absA @ np.abs(x) + np.abs(lp.b))
            sd_scale = np.linalg.norm(absA.T @ np.abs(y) + np.abs(lp.c))
            assert abs(g.rel_primal - o.rel_p) <= 1e-12 * (1 + sp_scale) / (1 + nb)
            assert abs(g.rel_dual - o.rel_d) <= 1e-12 * (1 + sd_scale) / (1 + nc)
            objscale = np.abs(lp.c) @ np.abs(x) + np.abs(lp.b) @ np.abs(y) + \
                np.nan_to_num(np.abs(lp.lb) + np.abs(lp.ub), posinf=0) @ (absA.T @ np.abs(y) + np.abs(lp.c))
            assert abs(g.pobj - o.pobj) <= 1e-12 * objscale
            assert abs(g.dobj - o.dobj) <= 1e-12 * objscale
            assert abs(g.abs_primal_inf - o.max_primal_violation) <= 1e-12 * (1 + np.max(absA @ np.abs(x)))
            gap = abs(o.pobj - o.dobj) / (1 + abs(o.pobj) + abs(o.dobj))
            assert abs(g.rel_gap - gap) <= 4e-12 * objscale / (1 + abs(o.pobj) + abs(o.dobj))


# ---------------------------------------------------------------------------
# standalone SpMV kernels on adversarial row-length mixes
# ---------------------------------------------------------------------------

def adversarial(kind, rng):
    if kind == "uc":
        lp = make_instance("medium", 0)
        return sp.csr_matrix((lp.val, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))
    if kind == "empty_rows":
        A = sp.random(3000, 2000, density=0.002, random_state=1, format="lil")
        A[::7, :] = 0
        return A.tocsr()
    if kind == "one_long_row":
        A = sp.random(5000, 120000, density=0.00002, random_state=2, format="lil")
        A[1234, :] = rng.normal(size=120000)
        return A.tocsr()
    if kind == "length_one":
        n = 70001
        return sp.csr_matrix((rng.normal(size=n), rng.integers(0, 5000, n), np.arange(n + 1)), shape=(n, 5000))
    if kind == "ragged":
        lens = rng.integers(0, 3000, 400)
        lens[::5] = 0
        rows = np.repeat(np.arange(400), lens)
        cols = np.concatenate([rng.choice(4000, L, replace=False) for L in lens])
        A = sp.csr_matrix((rng.normal(size=len(rows)), (rows, cols)), shape=(400, 4000))
        return A
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["uc", "empty_rows", "one_long_row", "length_one", "ragged"])
@pytest.mark.parametrize("algo", [uclp.UC_LP_SPMV_ROWSPLIT, uclp.UC_LP_SPMV_MERGEPATH])
def test_spmv_kernels(kind, algo):
    rng = np.random.default_rng(11)
    A = adversarial(kind, rng)
    A.sort_indices()
    A.sum_duplicates()
    say("case spmv", kind, algo, A.shape, A.nnz)
    x = rng.normal(size=A.shape[1])
    ref = ps.csr_matvec(A.indptr, A.indices, A.data, x)
    bound = abs(A) @ np.abs(x)
    k = max(int(np.diff(A.indptr).max()), 1)
    y64 = uclp.uc_spmv(A.shape[0], A.shape[1], A.indptr, A.indices, A.data, x, uclp.UC_LP_FP64, algo)
    assert np.all(np.abs(y64 - ref) <= 2 * k * U64 * bound + 1e-300)
    y32 = uclp.uc_spmv(A.shape[0], A.shape[1], A.indptr, A.indices, A.data, x, uclp.UC_LP_FP32_MIXED, algo)
    # inputs rounded to FP32 (relative 2u each), then k-term FP32 accumulation
    assert np.all(np.abs(y32 - ref) <= (k + 4) * U32 * 1.01 * bound + 1e-30)


# ---------------------------------------------------------------------------
# whole solves: objective against the oracle, KKT recomputed by the oracle
# ---------------------------------------------------------------------------

def solve(lp, **opts):
    x, y, info = uclp.solve(lp, uclp.uc_lp_opts_default(**opts), timeout_s=300)
    return x, y, info


@pytest.mark.parametrize("seed", range(10))
def test_tiny_fp64_matches_simplex_oracle(seed):
    lp = make_instance("tiny", seed)
    say("case tiny fp64", seed)
    z = GOLDEN[f"tiny/{seed}"]["obj"]
    x, y, info = solve(lp, precision=uclp.UC_LP_FP64, eps_rel=1e-8)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    k = kkt(lp, x, y)
    assert k.rel_kkt <= 1e-8 * 1.001
    assert abs(k.rel_kkt - info["rel_kkt"]) <= 1e-10
    assert abs(k.pobj - z) <= 1e-6 * abs(z)
    assert np.all(x >= lp.lb) and np.all(x <= lp.ub)


@pytest.mark.parametrize("gamma", [0.0, 0.5])
def test_tiny_partial_reflection_matches_simplex_oracle(gamma):
    # gamma < 1 stores the Halpern iterate every iteration instead of
    # rebuilding it from xbar; both paths reach the oracle's optimum
    lp = make_instance("tiny", 4)
    say("case tiny fp64 gamma", gamma)
    z = GOLDEN["tiny/4"]["obj"]
    x, y, info = solve(lp, precision=uclp.UC_LP_FP64, eps_rel=1e-8, halpern_gamma=gamma)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    k = kkt(lp, x, y)
    assert k.rel_kkt <= 1e-8 * 1.001
    assert abs(k.pobj - z) <= 1e-6 * abs(z)


def test_fp32_stall_continues_in_fp64():
    # a stall window of one check hands the solve to FP64 at the first check
    # without a 10% improvement; the FP64 phase still reaches the target
    lp = make_instance("medium", 1)
    say("case medium fp32 stall")
    z = GOLDEN["medium/1"]["obj"]
    x, y, info = solve(lp, precision=uclp.UC_LP_FP32_MIXED, fp32_stall_checks=1, eps_gap_rel=1e-7)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    assert 0 < info["iters_fp64"] < info["iters"]
    assert info["precision_now"] == uclp.UC_LP_FP64
    k = kkt(lp, x, y)
    assert k.rel_kkt <= 1e-4 * 1.001
    # the FP64 phase also closes the duality gap before it returns
    assert info["rel_gap"] <= 1e-7
    assert abs(k.pobj - z) <= 1e-6 * abs(z)


def test_weight_bound_of_one_fixes_the_primal_weight():
    # a change bound of 1 keeps the initial weight whatever the smoothing, so
    # two smoothings take the same iterates; unbounded, they do not
    lp = make_instance("tiny", 2)
    say("case tiny weight bound")
    _, _, a = solve(lp, precision=uclp.UC_LP_FP64, eps_rel=1e-6, pw_max_change=1.0, pw_smoothing=0.8)
    _, _, b = solve(lp, precision=uclp.UC_LP_FP64, eps_rel=1e-6, pw_max_change=1.0, pw_smoothing=0.5)
    _, _, c = solve(lp, precision=uclp.UC_LP_FP64, eps_rel=1e-6, pw_max_change=0.0, pw_smoothing=0.5)
    assert a["restarts"] > 0 and c["restarts"] > 0
    assert (a["iters"], a["pobj"], a["omega"]) == (b["iters"], b["pobj"], b["omega"])
    assert c["omega"] != a["omega"]


def test_columns_without_entries():
    # 600 columns that appear in no row fill whole row blocks of A^T with no
    # entries; each goes to the bound its cost points at, so the optimum
    # moves by the sum of the negative costs
    lp = make_instance("tiny", 6)
    z = GOLDEN["tiny/6"]["obj"]
    k = 600
    rng = np.random.default_rng(6)
    cx = rng.uniform(-2.0, 2.0, k)
    wide = LP(m=lp.m, n=lp.n + k, row_ptr=lp.row_ptr, col_idx=lp.col_idx, val=lp.val,
              c=np.append(lp.c, cx), b=lp.b, sense=lp.sense, lb=np.append(lp.lb, np.zeros(k)),
              ub=np.append(lp.ub, np.ones(k)))
    say("case tiny 6 with empty columns")
    x, y, info = solve(wide, precision=uclp.UC_LP_FP64, eps_rel=1e-8)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    zz = z + cx[cx < 0].sum()
    assert abs(info["pobj"] - zz) <= 1e-6 * abs(zz)
    xe = x[lp.n:]
    assert np.all((xe >= 0) & (xe <= 1))
    # a column whose cost is small next to the objective's scale may stop
    # short of its bound within the relative KKT tolerance; the others reach it
    big = np.abs(cx) > 0.1
    assert np.max(np.abs(xe[big] - (cx[big] < 0))) <= 1e-6


@pytest.mark.parametrize("prec", [uclp.UC_LP_FP64, uclp.UC_LP_FP32_MIXED])
def test_one_sided_bounds_solve_matches_simplex_oracle(prec):
    # columns with only a lower or only an upper bound take the kernels'
    # l = -inf / u = +inf paths in the projections and in the bound
    # multipliers of the check
    lp = one_sided_instance(2)
    say("case one-sided", prec)
    res = simplex_solve(lp)
    assert res.status == "optimal"
    eps = 1e-8 if prec == uclp.UC_LP_FP64 else 1e-4
    x, y, info = solve(lp, precision=prec, eps_rel=eps, eps_gap_rel=1e-7)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    k = kkt(lp, x, y)
    assert k.rel_kkt <= eps * 1.001
    assert abs(k.rel_kkt - info["rel_kkt"]) <= 1e-10 + 1e-6 * eps
    assert abs(k.pobj - res.obj) <= 1e-6 * abs(res.obj)
    assert np.all(x >= lp.lb) and np.all(x <= lp.ub)


def test_long_rows_solve_matches_simplex_oracle():
    # long rows of A and of A^T take the block-wide path in every kernel
    lp = ragged_instance(1)
    say("case ragged fp64")
    assert np.diff(lp.row_ptr).max() > 2048
    res = simplex_solve(lp)
    x, y, info = solve(lp, precision=uclp.UC_LP_FP64, eps_rel=1e-8)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    k = kkt(lp, x, y)
    assert k.rel_kkt <= 1e-8 * 1.001
    assert abs(k.pobj - res.obj) <= 1e-6 * abs(res.obj)


@pytest.mark.parametrize("seed", range(3))
def test_tiny_fp32_modes(seed):
    lp = make_instance("tiny", seed)
    say("case tiny fp32", seed)
    z = GOLDEN[f"tiny/{seed}"]["obj"]
    x, y, info = solve(lp, precision=uclp.UC_LP_FP32_MIXED, eps_gap_rel=1e-7)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    k = kkt(lp, x, y)
    assert k.rel_kkt <= 1e-4
    # past the 1e-4 milestone the solve closes the FP64 duality gap to 1e-7
    assert info["rel_gap"] <= 1e-7 and info["t_to_eps_s"] > 0
    assert abs(k.pobj - z) <= 1e-6 * abs(z)
    x, y, info = solve(lp, precision=uclp.UC_LP_FP32_MIXED_POLISH)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    k = kkt(lp, x, y)
    assert k.rel_kkt <= 1e-8 * 1.001
    assert abs(k.pobj - z) <= 1e-6 * abs(z)
    assert info["iters_fp64"] < info["iters"]


@pytest.mark.parametrize("seed", range(3))
def test_medium_polish_matches_highs_oracle(seed):
    lp = make_instance("medium", seed)
    say("case medium polish", seed)
    z = GOLDEN[f"medium/{seed}"]["obj"]
    t = time.time()
    # the FP64 polish to 1e-8 can need more than the paper's 100,000 iterations here
    x, y, info = solve(lp, precision=uclp.UC_LP_FP32_MIXED_POLISH, iter_limit=400000)
    say("  ", info["status_name"], info["iters"], info["iters_fp64"], info["t_total_s"], time.time() - t)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    k = kkt(lp, x, y)
    assert k.rel_kkt <= 1e-8 * 1.001
    assert abs(k.pobj - z) <= 1e-6 * abs(z)
    assert info["t_to_eps_s"] > 0 and info["rel_kkt_at_eps"] <= 1e-4


# ---------------------------------------------------------------------------
# boundary behaviour
# ---------------------------------------------------------------------------

def test_status_cancel_and_errors():
    lp = make_instance("medium", 0)
    h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP64, eps_rel=1e-12))
    try:
        with pytest.raises(uclp.UcLpError) as e:
            uclp.uc_lp_get_solution(h, lp.n, lp.m)
        assert e.value.code == uclp.UC_LP_ESTATE
        uclp.uc_lp_solve(h)
        with pytest.raises(uclp.UcLpError) as e:
            uclp.uc_lp_solve(h)
        assert e.value.code == uclp.UC_LP_ESTATE
        time.sleep(0.3)
        assert uclp.uc_lp_status(h).status == uclp.UC_LP_RUNNING
        uclp.uc_lp_cancel(h)
        assert uclp.uc_lp_wait(h, 30)
        info = uclp.uc_lp_status(h)
        assert info.status == uclp.UC_LP_CANCELLED and info.iters > 0
        x, y = uclp.uc_lp_get_solution(h, lp.n, lp.m)
        assert np.all(np.isfinite(x)) and np.all(np.isfinite(y))
    finally:
        uclp.uc_lp_destroy(h)


def test_iteration_limit_and_warm_start():
    lp = make_instance("tiny", 4)
    x, y, info = solve(lp, precision=uclp.UC_LP_FP64, iter_limit=128, eps_rel=1e-12)
    assert info["status"] == uclp.UC_LP_ITER_LIMIT and info["iters"] == 128
    # warm start from a converged point stops at the first check
    xs, ys, info = solve(lp, precision=uclp.UC_LP_FP64, eps_rel=1e-7)
    h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP64, eps_rel=1e-6))
    try:
        uclp.uc_lp_solve(h, xs, ys)
        uclp.uc_lp_wait(h, 60)
        assert uclp.uc_lp_status(h).iters == 64
    finally:
        uclp.uc_lp_destroy(h)


def test_update_data_and_infeasible_empty_row():
    lp = make_instance("tiny", 5)
    z = GOLDEN["tiny/5"]["obj"]
    h = uclp.uc_lp_create(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP64, eps_rel=1e-8))
    try:
        uclp.uc_lp_update_data(h, c=2.0 * lp.c)
        uclp.uc_lp_solve(h)
        uclp.uc_lp_wait(h, 120)
        info = uclp.uc_lp_status(h)
        assert info.status == uclp.UC_LP_OPTIMAL
        assert abs(info.pobj - 2 * z) <= 1e-6 * 2 * z
    finally:
        uclp.uc_lp_destroy(h)
    # an empty 'E' row with a non-zero right-hand side is infeasible
    A = sp.csr_matrix((lp.val, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))
    A = sp.vstack([A, sp.csr_matrix((1, lp.n))]).tocsr()
    bad = LP(m=lp.m + 1, n=lp.n, row_ptr=A.indptr, col_idx=A.indices, val=A.data, c=lp.c,
             b=np.append(lp.b, 1.0), sense=np.append(lp.sense, ord("E")).astype(np.uint8), lb=lp.lb, ub=lp.ub)
    x, y, info = solve(bad)
    assert info["status"] == uclp.UC_LP_INFEASIBLE


# ---------------------------------------------------------------------------
# crossover from the PDHG point to a vertex
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 5])
def test_crossover_from_the_pdhg_point_reaches_the_oracle_optimum(seed):
    # the library's FP32 + FP64-polish point (rel. KKT 1e-8) of the 30-bus
    # grid, then crossover on the host: an optimal vertex whose objective is
    # the oracle's optimum
    from paper_2607_03627_amd.crossover import crossover

    lp = make_instance("tiny", seed)
    say("case crossover", seed)
    z = GOLDEN[f"tiny/{seed}"]["obj"]
    x, y, info = solve(lp, precision=uclp.UC_LP_FP32_MIXED_POLISH, eps_polish=1e-8)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    r = crossover(lp, x, y)
    say("  ", r.status, r.obj, z, "pivots", r.pivots, r.phase1_pivots, "candidates", r.candidates, r.seconds)
    assert r.status == "optimal"
    assert abs(r.obj - z) <= 1e-9 * abs(z)
    k = kkt(lp, r.x, r.y)
    assert k.rel_kkt <= 1e-9
    assert np.all(r.x >= lp.lb - 1e-9) and np.all(r.x <= lp.ub + 1e-9)
