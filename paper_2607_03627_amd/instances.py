"""Seeded synthetic DC unit-commitment LP relaxations.

The paper solves the continuous relaxation of a multi-period unit-commitment
MILP (Sec. II-A; Sec. II-C gives that LP relaxation to PDHG on the GPU and to
barrier on the CPU) on the 6,049-bus GO Challenge 3 system (Sec. II-E,
Table I).  Those data sets are not available here, so this module builds DC
unit-commitment LPs of the same structure from random draws:

  variables per period t (time-major column order)
      p_g  in [0, Pmax_g]      generator output (p.u.)
      u_g  in [0, 1]           commitment, relaxed from {0,1}
      v_g  in [0, 1]           start-up indicator, relaxed
      th_i free (th_ref = 0)   bus voltage angle
      f_l  in [-F_l, F_l]      line flow
      s_i  in [0, d_it]        load shed (value of lost load)
      and per contingency copy k: th_i^k, f_l^k (outaged line removed)
  rows per period t
      balance  (=)  sum_{g at i} p_g + s_i - sum_{l from i} f_l + sum_{l to i} f_l = d_it
      flow     (=)  f_l - B_l (th_from - th_to) = 0
      (the same two families again for every contingency copy, sharing p, s)
      pmin     (>=) p_g - Pmin_g u_g >= 0
      pmax     (>=) Pmax_g u_g - p_g >= 0
      ramp     (>=) p_t - p_{t-1} >= -R_g  and  p_{t-1} - p_t >= -R_g   (t >= 1)
      startup  (>=) v_t - u_t + u_{t-1} >= 0                            (u_{-1} = 0)
  objective
      sum_t dt * (100 c_g p_g + NL_g u_g) + SU_g v_g + dt * 100 * VOLL * s_i

This module holds only input generation: it draws data and assembles the CSR
arrays.  It contains no part of any solver, so both the CPU oracle and the
GPU path may consume what it produces.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

SENSE_E = ord("E")
SENSE_G = ord("G")
SENSE_L = ord("L")


@dataclass
class LP:
    """min c'x  s.t.  a_i'x (= or >=) b_i,  lb <= x <= ub  in CSR form.

    row_ptr/col_idx are int32, val/c/b/lb/ub float64, sense uint8 holding the
    ASCII codes 'E', 'G' (or 'L').  Column indices are sorted within a row and
    unique.  Infinite bounds are +-inf.
    """

    m: int
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    c: np.ndarray
    b: np.ndarray
    sense: np.ndarray
    lb: np.ndarray
    ub: np.ndarray
    meta: Dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def with_data(self, c=None, b=None, lb=None, ub=None) -> "LP":
        """Same matrix, replaced right-hand side, costs or bounds."""
        return replace(
            self,
            c=self.c if c is None else np.ascontiguousarray(c, dtype=np.float64),
            b=self.b if b is None else np.ascontiguousarray(b, dtype=np.float64),
            lb=self.lb if lb is None else np.ascontiguousarray(lb, dtype=np.float64),
            ub=self.ub if ub is None else np.ascontiguousarray(ub, dtype=np.float64),
        )


@dataclass(frozen=True)
class UCShape:
    """Distribution parameters of one synthetic grid family."""

    name: str
    n_bus: int
    n_extra_edges: int
    n_gen: int
    n_periods: int
    dt_hours: float
    load_noise_sd: float = 0.0
    n_contingencies: int = 0
    voll: float = 200.0       # $/MWh for shed load
    s_base: float = 100.0     # MVA per p.u.


def _extra_40pct(n_bus: int) -> int:
    return int(round(0.4 * (n_bus - 1)))


SHAPES: Dict[str, UCShape] = {
    # 30-bus meshed grid, 10 units, 24 hourly periods (~3.1k columns, ~2.8k rows)
    "tiny": UCShape("tiny", 30, 10, 10, 24, 1.0),
    # 500-bus grid with 40% extra edges, 120 units, 48 half-hour periods, load noise
    "medium": UCShape("medium", 500, _extra_40pct(500), 120, 48, 0.5, 0.05),
    # 6,049-bus-shaped grid: 8,500 branches, 700 units, 48 hourly periods,
    # three preventive line-outage copies (~3.18M columns, ~2.96M rows, ~9.8M nnz)
    "large": UCShape("large", 6049, 8500 - 6048, 700, 48, 1.0, 0.0, 3),
    # the same grid without contingency copies (~1.09M columns, ~2.7M nnz)
    "large_kc0": UCShape("large_kc0", 6049, 8500 - 6048, 700, 48, 1.0, 0.0, 0),
}


@dataclass
class Grid:
    n_bus: int
    line_from: np.ndarray   # int64 [L]
    line_to: np.ndarray     # int64 [L]
    line_b: np.ndarray      # susceptance, p.u.
    line_f: np.ndarray      # thermal limit, p.u.
    n_tree: int             # the first n_tree lines form a spanning tree


@dataclass
class Units:
    bus: np.ndarray
    pmin: np.ndarray
    pmax: np.ndarray
    cost: np.ndarray        # $/MWh
    noload: np.ndarray      # $/h
    startup: np.ndarray     # $
    ramp: np.ndarray        # p.u. per period


def draw_grid(rng: np.random.Generator, n_bus: int, n_extra: int) -> Grid:
    """Random recursive spanning tree plus uniform extra edges without duplicates."""
    if n_bus > 1:
        idx = np.arange(1, n_bus)
        parent = np.minimum((rng.random(n_bus - 1) * idx).astype(np.int64), idx - 1)
        frm = list(parent)
        to = list(idx)
    else:
        frm, to = [], []
    seen = {(min(a, b), max(a, b)) for a, b in zip(frm, to)}
    max_edges = n_bus * (n_bus - 1) // 2
    if len(seen) + n_extra > max_edges:
        raise ValueError("too many extra edges for this bus count")
    added = 0
    while added < n_extra:
        a, b = (int(v) for v in rng.integers(0, n_bus, size=2))
        if a == b:
            continue
        key = (min(a, b), max(a, b))
        if key in seen:
            continue
        seen.add(key)
        frm.append(a)
        to.append(b)
        added += 1
    L = len(frm)
    return Grid(
        n_bus=n_bus,
        line_from=np.asarray(frm, dtype=np.int64),
        line_to=np.asarray(to, dtype=np.int64),
        line_b=rng.uniform(5.0, 20.0, L),
        line_f=rng.uniform(0.5, 2.0, L),
        n_tree=max(n_bus - 1, 0),
    )


def draw_units(rng: np.random.Generator, n_bus: int, n_gen: int) -> Units:
    pmax = rng.uniform(0.5, 3.0, n_gen)
    return Units(
        bus=rng.integers(0, n_bus, n_gen).astype(np.int64),
        pmin=rng.uniform(0.1, 0.4, n_gen) * pmax,
        pmax=pmax,
        cost=rng.uniform(10.0, 60.0, n_gen),
        noload=rng.uniform(50.0, 200.0, n_gen),
        startup=rng.uniform(100.0, 500.0, n_gen),
        ramp=0.5 * pmax,
    )


def draw_loads(rng: np.random.Generator, n_bus: int, n_periods: int, dt: float,
               noise_sd: float) -> np.ndarray:
    """d[t, i] = base_i * (1 + 0.3 sin(2 pi h_t / 24) + noise), clipped at 0."""
    base = rng.uniform(0.1, 0.5, n_bus)
    h = np.arange(n_periods) * dt
    prof = 1.0 + 0.3 * np.sin(2.0 * math.pi * h / 24.0)
    fac = np.repeat(prof[:, None], n_bus, axis=1)
    if noise_sd > 0:
        fac = fac + rng.normal(0.0, noise_sd, size=fac.shape)
    return base[None, :] * np.maximum(fac, 0.0)


def build_uc_lp(grid: Grid, units: Units, loads: np.ndarray, dt: float, *,
                voll: float = 200.0, s_base: float = 100.0, ref_bus: int = 0,
                outages: Sequence[int] = (), include_ramp: bool = True,
                include_shed: bool = True) -> LP:
    """Assemble the DC-UC LP relaxation described in the module docstring."""
    T, N = loads.shape
    assert N == grid.n_bus
    G = len(units.pmax)
    L = len(grid.line_from)
    K = len(outages)
    keep = [np.setdiff1d(np.arange(L), [o]) for o in outages]

    # ---- column layout (per period block) ----
    off = {}
    o = 0
    for name, size in (("p", G), ("u", G), ("v", G), ("th", N), ("f", L)):
        off[name] = o
        o += size
    if include_shed:
        off["s"] = o
        o += N
    off_cont = []
    for k in range(K):
        off_cont.append((o, o + N))  # (theta_k, f_k)
        o += N + len(keep[k])
    ncol_t = o
    n = ncol_t * T

    # ---- row layout (per period block) ----
    roff = {}
    r = 0
    roff["bal"] = r; r += N
    roff["flow"] = r; r += L
    roff_cont = []
    for k in range(K):
        roff_cont.append((r, r + N))
        r += N + len(keep[k])
    roff["pmin"] = r; r += G
    roff["pmax"] = r; r += G
    nrow_first = r + G                      # startup rows, no ramp at t = 0
    roff_ramp = r
    nrow_t = r + (2 * G if include_ramp else 0) + G

    rows: List[np.ndarray] = []
    cols: List[np.ndarray] = []
    vals: List[np.ndarray] = []
    c = np.zeros(n)
    lb = np.zeros(n)
    ub = np.zeros(n)
    b_list: List[np.ndarray] = []
    sense_list: List[np.ndarray] = []
    row_base = 0

    def add(rr, cc, vv):
        rr = np.asarray(rr, dtype=np.int64)
        cc = np.asarray(cc, dtype=np.int64)
        vv = np.broadcast_to(np.asarray(vv, dtype=np.float64), rr.shape)
        rows.append(rr)
        cols.append(cc)
        vals.append(np.array(vv))

    gidx = np.arange(G)
    bidx = np.arange(N)
    period_row_base = []
    for t in range(T):
        cb = t * ncol_t
        rb = row_base
        period_row_base.append(rb)
        pc, uc, vc = cb + off["p"], cb + off["u"], cb + off["v"]
        thc, fc = cb + off["th"], cb + off["f"]
        # bounds and costs
        c[pc:pc + G] = dt * s_base * units.cost
        c[uc:uc + G] = dt * units.noload
        c[vc:vc + G] = units.startup
        lb[pc:pc + G], ub[pc:pc + G] = 0.0, units.pmax
        lb[uc:uc + G], ub[uc:uc + G] = 0.0, 1.0
        lb[vc:vc + G], ub[vc:vc + G] = 0.0, 1.0
        lb[thc:thc + N], ub[thc:thc + N] = -np.inf, np.inf
        lb[thc + ref_bus] = ub[thc + ref_bus] = 0.0
        lb[fc:fc + L], ub[fc:fc + L] = -grid.line_f, grid.line_f
        if include_shed:
            sc = cb + off["s"]
            c[sc:sc + N] = dt * s_base * voll
            lb[sc:sc + N], ub[sc:sc + N] = 0.0, loads[t]

        def network(rbal, rflow, th0, f0, lines):
            # balance rows
            add(rbal + units.bus, pc + gidx, 1.0)
            if include_shed:
                add(rbal + bidx, cb + off["s"] + bidx, 1.0)
            lf = grid.line_from[lines]
            lt = grid.line_to[lines]
            fcol = f0 + np.arange(len(lines))
            add(rbal + lf, fcol, -1.0)
            add(rbal + lt, fcol, 1.0)
            # flow definition rows
            frow = rflow + np.arange(len(lines))
            add(frow, fcol, 1.0)
            add(frow, th0 + lf, -grid.line_b[lines])
            add(frow, th0 + lt, grid.line_b[lines])

        network(rb + roff["bal"], rb + roff["flow"], thc, fc, np.arange(L))
        for k in range(K):
            th_k, f_k = off_cont[k]
            lb[cb + th_k:cb + th_k + N] = -np.inf
            ub[cb + th_k:cb + th_k + N] = np.inf
            lb[cb + th_k + ref_bus] = ub[cb + th_k + ref_bus] = 0.0
            kl = keep[k]
            lb[cb + f_k:cb + f_k + len(kl)] = -grid.line_f[kl]
            ub[cb + f_k:cb + f_k + len(kl)] = grid.line_f[kl]
            rbal_k, rflow_k = roff_cont[k]
            network(rb + rbal_k, rb + rflow_k, cb + th_k, cb + f_k, kl)

        bal_rhs = [loads[t]]
        e_count = N + L + sum(N + len(kk) for kk in keep)
        b_t = np.zeros(e_count)
        b_t[roff["bal"]:roff["bal"] + N] = loads[t]
        for k in range(K):
            rbal_k, _ = roff_cont[k]
            b_t[rbal_k:rbal_k + N] = loads[t]
        del bal_rhs
        # pmin / pmax
        add(rb + roff["pmin"] + gidx, pc + gidx, 1.0)
        add(rb + roff["pmin"] + gidx, uc + gidx, -units.pmin)
        add(rb + roff["pmax"] + gidx, pc + gidx, -1.0)
        add(rb + roff["pmax"] + gidx, uc + gidx, units.pmax)
        g_rhs = [np.zeros(G), np.zeros(G)]
        r_next = roff_ramp
        if include_ramp and t > 0:
            pprev = pc - ncol_t
            add(rb + r_next + gidx, pc + gidx, 1.0)
            add(rb + r_next + gidx, pprev + gidx, -1.0)
            add(rb + r_next + G + gidx, pc + gidx, -1.0)
            add(rb + r_next + G + gidx, pprev + gidx, 1.0)
            g_rhs += [-units.ramp, -units.ramp]
            r_next += 2 * G
        # startup
        add(rb + r_next + gidx, vc + gidx, 1.0)
        add(rb + r_next + gidx, uc + gidx, -1.0)
        if t > 0:
            add(rb + r_next + gidx, uc - ncol_t + gidx, 1.0)
        g_rhs.append(np.zeros(G))
        r_next += G
        b_list.append(b_t)
        b_list.append(np.concatenate(g_rhs))
        sense_list.append(np.full(e_count, SENSE_E, dtype=np.uint8))
        sense_list.append(np.full(r_next - roff["pmin"], SENSE_G, dtype=np.uint8))
        row_base += r_next

    m = row_base
    b = np.concatenate(b_list)
    sense = np.concatenate(sense_list)
    assert len(b) == m and len(sense) == m
    R = np.concatenate(rows)
    C = np.concatenate(cols)
    V = np.concatenate(vals)
    order = np.lexsort((C, R))
    R, C, V = R[order], C[order], V[order]
    if len(R) > 1:
        dup = (R[1:] == R[:-1]) & (C[1:] == C[:-1])
        if dup.any():
            raise AssertionError("duplicate matrix entry in generated LP")
    counts = np.bincount(R, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31 or n >= 2**31:
        raise ValueError("instance exceeds int32 indexing")
    meta = dict(T=T, N=N, G=G, L=L, K=K, ncol_t=ncol_t, col_off=off,
                cont_col_off=off_cont, row_off=roff, period_row_base=period_row_base,
                dt=dt, s_base=s_base, voll=voll, include_shed=include_shed,
                include_ramp=include_ramp, ref_bus=ref_bus)
    return LP(m=m, n=n, row_ptr=row_ptr.astype(np.int32), col_idx=C.astype(np.int32),
              val=V.astype(np.float64), c=c, b=b, sense=sense, lb=lb, ub=ub, meta=meta)


def make_instance(shape, seed: int, **overrides) -> LP:
    """Draw grid, units and loads for a named shape (or UCShape) and build the LP."""
    if isinstance(shape, str):
        shape = SHAPES[shape]
    if overrides:
        shape = replace(shape, **overrides)
    rng = np.random.default_rng(seed)
    grid = draw_grid(rng, shape.n_bus, shape.n_extra_edges)
    units = draw_units(rng, shape.n_bus, shape.n_gen)
    loads = draw_loads(rng, shape.n_bus, shape.n_periods, shape.dt_hours, shape.load_noise_sd)
    outages: List[int] = []
    if shape.n_contingencies:
        non_tree = np.arange(grid.n_tree, len(grid.line_from))
        if len(non_tree) < shape.n_contingencies:
            raise ValueError("not enough non-tree lines for the contingency copies")
        outages = sorted(int(v) for v in rng.choice(non_tree, shape.n_contingencies, replace=False))
    lp = build_uc_lp(grid, units, loads, shape.dt_hours, voll=shape.voll,
                     s_base=shape.s_base, outages=outages)
    lp.meta.update(shape=shape.name, seed=seed, outages=outages, grid=grid, units=units,
                   loads=loads)
    return lp


# ---------------------------------------------------------------------------
# Scenario variants sharing one matrix (load scaling + cost perturbation)
# ---------------------------------------------------------------------------

def scenario_data(lp: LP, seed: int, load_range=(0.85, 1.15), cost_range=(0.95, 1.05)):
    """One variant of a generated LP: per-bus load factor and per-unit cost factor.

    The matrix is untouched; the balance right-hand sides and the shed upper
    bounds follow the scaled loads, and every objective coefficient of a unit
    (output, no-load, start-up) is multiplied by that unit's factor.
    Returns (c, b, lb, ub).
    """
    meta = lp.meta
    rng = np.random.default_rng(seed)
    N, G, T, K = meta["N"], meta["G"], meta["T"], meta["K"]
    lf = rng.uniform(*load_range, N)
    cf = rng.uniform(*cost_range, G)
    c = lp.c.copy()
    b = lp.b.copy()
    ub = lp.ub.copy()
    off, roff = meta["col_off"], meta["row_off"]
    for t in range(T):
        cb = t * meta["ncol_t"]
        rb = meta["period_row_base"][t]
        for key in ("p", "u", "v"):
            c[cb + off[key]:cb + off[key] + G] *= cf
        b[rb + roff["bal"]:rb + roff["bal"] + N] *= lf
        # contingency balance rows sit right after the base flow rows
        r = rb + roff["flow"] + meta["L"]
        for k in range(K):
            b[r:r + N] *= lf
            r += N + meta["L"] - 1
        if meta["include_shed"]:
            ub[cb + off["s"]:cb + off["s"] + N] *= lf
    return c, b, lp.lb.copy(), ub


# ---------------------------------------------------------------------------
# Serving stream: Poisson arrivals of differently sized requests
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Request:
    index: int
    arrival_s: float
    shape: UCShape
    seed: int


def serving_stream(seed: int, n_requests: int = 64, mean_gap_s: float = 0.05,
                   bus_range=(300, 2000)) -> List[Request]:
    """Poisson arrivals, bus count log-uniform, 24 hourly or 48 half-hour periods,
    0.12 units per bus and a spanning tree with 40% extra edges."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(mean_gap_s, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    lo, hi = math.log(bus_range[0]), math.log(bus_range[1])
    for i in range(n_requests):
        nb = int(round(math.exp(rng.uniform(lo, hi))))
        if rng.random() < 0.5:
            T, dt = 24, 1.0
        else:
            T, dt = 48, 0.5
        shape = UCShape(f"req{i}", nb, _extra_40pct(nb), int(round(0.12 * nb)), T, dt)
        out.append(Request(i, float(arrivals[i]), shape, int(rng.integers(0, 2**31 - 1))))
    return out
