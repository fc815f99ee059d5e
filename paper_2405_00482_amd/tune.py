"""Autotuner of the batched form (pvfl_batch_*).

Sweeps the launch options of the batched step -- products sharing one key
stream per work item (group), diagonals per work item (chunk), evaluation
indices per thread (vec), and the work-item order (chunk_major) -- timing the
whole step replayed from its HIP graph, and keeps the fastest in a tuner
database keyed by the workload's signature (parameter set and product shapes).

    python -m paper_2405_00482_amd.tune --products 64     (tunes the C3 workload)
"""
from __future__ import annotations

import argparse
import hashlib
import itertools
import json
import os
import sys
import time

DEFAULT_DB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", "batch_mi355x.json")
GRID = {"group": (1, 2, 4), "chunk": (8, 16, 32, 64, 128), "vec": (1, 2), "chunk_major": (1, 0)}


def signature(config: str, shapes) -> str:
    h = hashlib.sha1(json.dumps([list(map(int, s)) for s in shapes]).encode()).hexdigest()[:16]
    return f"{config}:{len(shapes)}:{h}"


def lookup(sig: str, db_path: str = DEFAULT_DB):
    if not os.path.exists(db_path):
        return None
    with open(db_path) as f:
        return json.load(f).get(sig)


def store(sig: str, entry: dict, db_path: str = DEFAULT_DB):
    db = {}
    if os.path.exists(db_path):
        with open(db_path) as f:
            db = json.load(f)
    db[sig] = entry
    os.makedirs(os.path.dirname(os.path.abspath(db_path)), exist_ok=True)
    with open(db_path, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)


def tune_batch(ctx, plans, bufs: dict, keys, sk, seed: int, reps: int = 3, grid=GRID, log=print):
    """time every option set of `grid` (graph replay, median of reps steps);
    returns (best option dict, best ms, table of all)"""
    import numpy as np
    import torch
    from . import pvfl
    table = []
    names = list(grid)
    for vals in itertools.product(*(grid[k] for k in names)):
        o = dict(zip(names, vals))
        try:
            b = pvfl.Batch(ctx, plans, keys=keys, **bufs, group=o["group"], chunk=o["chunk"], vec=o["vec"],
                           chunk_major=bool(o["chunk_major"]))
        except pvfl.PvflError as e:
            table.append({**o, "ms": None, "error": str(e)})
            continue
        b.run(sk, seed, graph=True)          # capture + first replay
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            b.run(sk, seed, graph=True)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        ms = float(np.median(ts))
        table.append({**o, "ms": ms})
        log(f"[tune] group {o['group']} chunk {o['chunk']:4d} vec {o['vec']} chunk_major {o['chunk_major']}: "
            f"{ms:.3f} ms")
        del b
    ok = [t for t in table if t["ms"] is not None]
    best = min(ok, key=lambda t: t["ms"])
    return {k: best[k] for k in names}, best["ms"], table


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--products", type=int, default=64)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--db", default=DEFAULT_DB)
    a = ap.parse_args(argv)
    import torch
    from . import pvfl
    from . import workloads as W
    name = "C3"
    log = lambda s: print(s, flush=True)  # noqa: E731
    seeds = W.seeds(name)
    ctx = pvfl.Context.from_dict(W.params_dict(name))
    shapes = W.c3_shapes(a.products)
    plans = [ctx.plan(pvfl.PLAN_HYBRID, m, n, lazy=True) for (m, n) in shapes]
    sk = ctx.keygen(seeds["sk"])
    keys = ctx.rotkeys(sk, sorted(set(g for p in plans for g in p.galois())), seeds["rotkeys"])
    f64 = dict(dtype=torch.float64, device="cuda")
    bufs = {"X": [], "v": [], "pt": [], "ct": [], "out": [], "y": []}
    for k, (m, n) in enumerate(shapes):
        XT, r = W.c3_inputs(k, (m, n))
        p = plans[k]
        bufs["X"].append(torch.from_numpy(XT).cuda())
        bufs["v"].append(torch.from_numpy(r).cuda())
        bufs["pt"].append(torch.empty(p.bytes("pt") // 8, **f64))
        bufs["ct"].append(torch.empty(p.bytes("ct_in") // 8, **f64))
        bufs["out"].append(torch.empty(p.bytes("ct_out") // 8, **f64))
        bufs["y"].append(torch.empty(m, **f64))
    best, ms, table = tune_batch(ctx, plans, bufs, keys, sk, seeds["enc"], reps=a.reps, log=log)
    sig = signature(name, shapes)
    store(sig, {"opts": best, "ms": ms, "device": "MI355X", "table": table}, a.db)
    log(f"[tune] best for {sig}: {best} at {ms:.3f} ms")


if __name__ == "__main__":
    sys.exit(main())
