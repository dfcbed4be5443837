"""Write tests/golden/objectives.json: optimal objectives of the seeded
synthetic instances, computed by the CPU oracle only.

    python tests/golden/make_golden.py [--large [--large-method highs-ds]] [--only KEY] [--log]

Tiny grids (30 buses, 24 periods) use the oracle's bounded simplex; the
500-bus grids and the 6,049-bus-shaped grids, beyond the simplex's reach, use
the oracle's HiGHS call (interior point with crossover).  Every entry records
the method and the wall time.  Instances come from the seeded generator in
paper_2607_03627_amd/instances.py.
"""

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.kkt import kkt  # noqa: E402
from oracle.reference import highs_solve, host_threads  # noqa: E402
from oracle.simplex import simplex_solve  # noqa: E402
from paper_2607_03627_amd.instances import make_instance, scenario_data  # noqa: E402

OUT = os.path.join(HERE, "objectives.json")


def load():
    if os.path.exists(OUT):
        with open(OUT) as f:
            return json.load(f)
    return {}


def save(d):
    # merge with what is on disk, so that two runs writing different keys
    # (a long 6,049-bus job beside a short one) do not drop each other's
    disk = load()
    disk.update(d)
    d.update(disk)
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(disk, f, indent=1, sort_keys=True)
    os.replace(tmp, OUT)


def record(d, key, lp, method, disp=False):
    t0 = time.perf_counter()
    if method == "simplex":
        r = simplex_solve(lp)
        assert r.status == "optimal", (key, r.status)
        obj, x, y = r.obj, r.x, r.y
    else:
        st, obj, x, y, _ = highs_solve(lp, method, disp=disp)
        assert st == 0, (key, st)
    k = kkt(lp, x, y)
    d[key] = dict(obj=obj, method=method, rel_kkt=k.rel_kkt, m=lp.m, n=lp.n, nnz=lp.nnz,
                  seconds=round(time.perf_counter() - t0, 3), threads=host_threads())
    print(key, d[key], flush=True)
    save(d)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--large", action="store_true", help="also the 6,049-bus-shaped grids")
    ap.add_argument("--only", default=None)
    ap.add_argument("--large-method", default="highs-ipm", choices=["highs-ipm", "highs-ds"],
                    help="HiGHS method for the 6,049-bus-shaped grids")
    ap.add_argument("--log", action="store_true", help="HiGHS progress log on stdout")
    args = ap.parse_args()
    d = load()
    jobs = [(f"tiny/{s}", "tiny", s, "simplex") for s in range(10)]
    jobs += [(f"medium/{s}", "medium", s, "highs-ds") for s in range(3)]
    if args.large:
        jobs += [("large_kc0/0", "large_kc0", 0, args.large_method), ("large/0", "large", 0, args.large_method)]
    for key, shape, seed, method in jobs:
        if args.only and not key.startswith(args.only):
            continue
        if key in d:
            continue
        record(d, key, make_instance(shape, seed), method, args.log)
    # scenario variants of the 500-bus grid (shared matrix, perturbed c, b, ub)
    base = make_instance("medium", 0)
    for s in range(1, 5):
        key = f"medium_scen/0/{s}"
        if key in d or (args.only and not key.startswith(args.only)):
            continue
        c, b, lb, ub = scenario_data(base, s)
        record(d, key, base.with_data(c=c, b=b, lb=lb, ub=ub), "highs-ds")


if __name__ == "__main__":
    main()
