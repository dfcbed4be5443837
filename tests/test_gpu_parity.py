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


def instance_and_oracle(shape, seed):
    if shape == "large":
        assert seed == 0
        return full_size_case()
    lp = ragged_instance(seed) if shape == "ragged" else make_instance(shape, seed)
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


def test_full_size_solve_in_the_benchmark_configuration():
    # the benchmark's solve (FP32 iterates, FP64 checks, 1e-4, event timing
    # on); the oracle recomputes the KKT error of the returned point
    lp, _ = full_size_case()
    say("case large 0 solve")
    x, y, info = solve(lp, precision=uclp.UC_LP_FP32_MIXED, eps_rel=1e-4, timing=1)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    k = kkt(lp, x, y)
    say("large rel_kkt", k.rel_kkt, info["rel_kkt"], k.pobj)
    assert k.rel_kkt <= 1e-4 * 1.001
    assert abs(k.rel_kkt - info["rel_kkt"]) <= 1e-6
    assert np.all(x >= lp.lb) and np.all(x <= lp.ub)
    assert info["primal_kernel_us"] > 0 and info["dual_kernel_us"] > 0


def test_kkt_kernels_match_oracle():
    lp = make_instance("tiny", 0)
    say("case tiny 0 kkt")
    res = simplex_solve(lp)
    rng = np.random.default_rng(3)
    with Handle(lp) as H:
        for scale in (0.0, 1e-6, 1e-2):
            x = np.clip(res.x + scale * rng.normal(size=lp.n), lp.lb, lp.ub)
            fixed = lp.lb == lp.ub
            x[fixed] = lp.lb[fixed]
            y = res.y + scale * rng.normal(size=lp.m)
            g = uclp.uc_lp_eval_kkt(H.h, x, y)
            o = kkt(lp, x, y)
            nb, nc = np.linalg.norm(lp.b), np.linalg.norm(lp.c)
            A = sp.csr_matrix((lp.val, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))
            sp_scale = np.linalg.norm(abs(A) @ np.abs(x) + np.abs(lp.b))
            sd_scale = np.linalg.norm(abs(A).T @ np.abs(y) + np.abs(lp.c))
            assert abs(g.rel_primal - o.rel_p) <= 1e-12 * (1 + sp_scale) / (1 + nb)
            assert abs(g.rel_dual - o.rel_d) <= 1e-12 * (1 + sd_scale) / (1 + nc)
            objscale = np.abs(lp.c) @ np.abs(x) + np.abs(lp.b) @ np.abs(y) + \
                np.nan_to_num(np.abs(lp.lb) + np.abs(lp.ub), posinf=0) @ (abs(A).T @ np.abs(y) + np.abs(lp.c))
            assert abs(g.pobj - o.pobj) <= 1e-12 * objscale
            assert abs(g.dobj - o.dobj) <= 1e-12 * objscale
            assert abs(g.abs_primal_inf - o.max_primal_violation) <= 1e-12 * (1 + np.max(abs(A) @ np.abs(x)))


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
    x, y, info = solve(lp, precision=uclp.UC_LP_FP32_MIXED, fp32_stall_checks=1)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    assert 0 < info["iters_fp64"] < info["iters"]
    assert info["precision_now"] == uclp.UC_LP_FP64
    k = kkt(lp, x, y)
    assert k.rel_kkt <= 1e-4 * 1.001
    assert abs(k.pobj - z) <= 1e-3 * abs(z)


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
    x, y, info = solve(lp, precision=uclp.UC_LP_FP32_MIXED)
    assert info["status"] == uclp.UC_LP_OPTIMAL, info
    k = kkt(lp, x, y)
    assert k.rel_kkt <= 1e-4
    # a relative gap below 1e-4 bounds the objective error to the same order
    assert abs(k.pobj - z) <= 1e-3 * abs(z)
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
