"""Plan selection: measured latencies, the two latency models, and regret.

    python -m paper_2405_00482_amd.planner collect --configs C1 C2 C3 C4 --shapes 64 --out DB.json
        times every candidate plan (encode of X plus the encrypted product,
        per call, on the current GPU) for seeded shapes of each parameter set
        and writes the records (shape, options, features, operation counts,
        milliseconds) -- the exhaustive tuning the planner is judged against.
    python -m paper_2405_00482_amd.planner evaluate DB.json
        trains the latency network on the training shapes (GPU kernels),
        fits the analytic model, and prints the regret of each on the
        held-out shapes.

Regret of a choice = its measured latency / the best measured latency of
that shape - 1.  Every computation on the plans runs in libpvfl; this module
only moves data, fits the analytic model's per-operation costs (non-negative
least squares over the training records) and drives the network's training
kernels.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import pvfl
from . import workloads as W

DEFAULT_DB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", "plan_latency_mi355x.json")

FEATURE_NAMES = ("log2_N", "limbs", "alpha", "beta", "K", "log2_m", "log2_n", "log2_mprime", "hybrid", "diag", "row",
                 "lazy", "ras_in_ct", "bsgs", "log2_bsgs", "lg_mult", "lg_add", "lg_rot", "lg_hstrot", "lg_modup",
                 "lg_moddown", "lg_pt_limbs", "lg_keys", "lg_blocks")
assert len(FEATURE_NAMES) == pvfl.PLAN_FEATURES


def counts_of(info: dict) -> list:
    """the analytic model's count vector (pvfl_plan_analytic_ms order)"""
    return [info["n_mult"], info["n_add"], info["n_rot"], info["n_hstrot"], info["n_modup"], info["n_moddown"],
            info["n_pts"] * info["pt_limbs"], 1]


def is_test_shape(idx: int) -> bool:
    return idx % 4 == 3


# ---------------------------------------------------------------------------
# exhaustive timing
# ---------------------------------------------------------------------------
def _time_plan(plan, X, ct, pt, out, ws, keys, torch, budget_ms: float = 60.0) -> float:
    s = torch.cuda.current_stream()

    def once():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        plan.encode_pt(X, pt)
        plan.matmul(ct, pt, keys, out, ws)
        e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1)

    first = once()                       # warm-up (also the estimate)
    if first > budget_ms:
        return once()
    reps = 5 if first < budget_ms / 10 else 2
    return float(np.median([once() for _ in range(reps)]))


def collect(names, count: int, log=print) -> list:
    import torch
    recs = []
    for name in names:
        ctx = pvfl.Context.from_dict(W.params_dict(name))
        sk = ctx.keygen(W.seeds(name)["sk"])
        shapes = W.planner_shapes(name, count)
        cands = [ctx.candidates(m, n) for (m, n) in shapes]
        plans = [[ctx.plan_from(o) for o in cs] for cs in cands]
        gal = sorted(set(g for ps in plans for p in ps for g in p.galois()))
        t0 = time.perf_counter()
        keys = ctx.rotkeys(sk, gal, W.seeds(name)["rotkeys"]) if gal else None
        torch.cuda.synchronize()
        log(f"[planner] {name}: {len(shapes)} shapes, {sum(len(c) for c in cands)} candidates, "
            f"{len(gal)} rotation keys ({time.perf_counter() - t0:.1f} s)")
        f64 = dict(dtype=torch.float64, device="cuda")
        for idx, ((m, n), cs, ps) in enumerate(zip(shapes, cands, plans)):
            Xh, yh = W.planner_inputs(name, idx, (m, n))
            X = torch.from_numpy(Xh).cuda()
            y = torch.from_numpy(yh).cuda()
            row = []
            for o, p in zip(cs, ps):
                pt = torch.empty(p.bytes("pt") // 8, **f64)
                ct = torch.empty(p.bytes("ct_in") // 8, **f64)
                out = torch.empty(p.bytes("ct_out") // 8, **f64)
                ws = torch.empty(max(1, p.bytes("workspace") // 8), **f64)
                p.encrypt(sk, y, 5 + idx, ct)
                ms = _time_plan(p, X, ct, pt, out, ws, keys, torch)
                rec = {"config": name, "idx": idx, "m": m, "n": n, "opts": o, "features": p.features(),
                       "counts": counts_of(p.info), "ms": ms}
                recs.append(rec)
                row.append(ms)
                del pt, ct, out, ws
            best = int(np.argmin(row))
            log(f"[planner] {name} #{idx} {m}x{n}: {len(cs)} candidates, best {row[best]:.3f} ms "
                f"({describe(cs[best])}), hybrid-lazy {row[0]:.3f} ms")
        del keys, plans
        torch.cuda.empty_cache()
    return recs


def describe(o: dict) -> str:
    kind = {0: "HYBRID", 1: "DIAG", 2: "ROW", 3: "CTMAT"}[o["kind"]]
    s = kind + ("" if o["kind"] == 2 else (" lazy" if o["lazy_moddown"] else " eager"))
    if o.get("bsgs"):
        s += f" bsgs{o['bsgs']}"
    if o.get("ras_in_ct"):
        s += " ras-in-ct"
    return s


# ---------------------------------------------------------------------------
# models
# ---------------------------------------------------------------------------
def split(recs):
    train = [r for r in recs if not is_test_shape(r["idx"])]
    test = [r for r in recs if is_test_shape(r["idx"])]
    return train, test


def fit_analytic(train) -> dict:
    """per parameter set: non-negative per-operation latencies (ms) minimising
    the squared relative error of sum(count x cost) over the training plans"""
    from scipy.optimize import nnls
    costs = {}
    for name in sorted(set(r["config"] for r in train)):
        rs = [r for r in train if r["config"] == name]
        A = np.array([r["counts"] for r in rs], dtype=np.float64)
        t = np.array([r["ms"] for r in rs])
        w = 1.0 / t                      # relative error
        c, _ = nnls(A * w[:, None], t * w)
        costs[name] = c.tolist()
    return costs


class Standardiser:
    def __init__(self, X, y):
        self.x_mean = X.mean(axis=0)
        sd = X.std(axis=0)
        self.x_std = np.where(sd > 1e-6, sd, 1.0)
        self.y_mean = float(y.mean())
        self.y_std = float(y.std()) or 1.0

    def x(self, X):
        return ((X - self.x_mean) / self.x_std).astype(np.float32)

    def y(self, y):
        return ((y - self.y_mean) / self.y_std).astype(np.float32)


def train_mlp(train, hidden: int = 64, steps: int = 4000, lr: float = 2e-3, seed: int = 0, log=None):
    """fit ln(ms) from the plan features with the library's GPU kernels
    (full-batch Adam, learning rate decayed tenfold over the run)"""
    import torch
    X = np.array([r["features"] for r in train], dtype=np.float64)
    y = np.log(np.array([r["ms"] for r in train]))
    st = Standardiser(X, y)
    net = pvfl.Mlp(X.shape[1], hidden, max_batch=len(train), seed=seed)
    xd = torch.from_numpy(st.x(X)).cuda()
    yd = torch.from_numpy(st.y(y)).cuda()
    for k in range(steps):
        loss = net.train_step(xd, yd, lr * (0.1 ** (k / steps)))
        if log and (k % 1000 == 0 or k == steps - 1):
            log(f"[planner] step {k}: loss {float(loss.item()):.4f}")
    return net, st


def mlp_predict_ms(net, st, recs) -> np.ndarray:
    import torch
    X = np.array([r["features"] for r in recs], dtype=np.float64)
    y = net.forward(torch.from_numpy(st.x(X)).cuda()).cpu().numpy().astype(np.float64)
    return np.exp(y * st.y_std + st.y_mean)


def analytic_predict_ms(costs, recs) -> np.ndarray:
    return np.array([float(np.dot(r["counts"], costs[r["config"]])) for r in recs])


def regrets(recs, pred) -> dict:
    """per shape: measured latency of the predicted-best candidate over the
    measured best, minus one"""
    by = {}
    for r, p in zip(recs, pred):
        by.setdefault((r["config"], r["idx"]), []).append((p, r["ms"], r))
    out = []
    for key, rows in sorted(by.items()):
        best = min(ms for _, ms, _ in rows)
        pick = min(rows, key=lambda t: t[0])
        out.append({"config": key[0], "idx": key[1], "regret": pick[1] / best - 1.0,
                    "chosen": describe(pick[2]["opts"]), "best": describe(min(rows, key=lambda t: t[1])[2]["opts"])})
    rg = np.array([o["regret"] for o in out])
    return {"mean": float(rg.mean()), "max": float(rg.max()), "geo": float(np.exp(np.mean(np.log1p(rg)))) - 1.0,
            "shapes": out}


def fixed_choice_regret(recs, pick) -> dict:
    """regret of always taking the candidate for which pick(opts) is True"""
    pred = np.array([0.0 if pick(r["opts"]) else 1.0 for r in recs])
    return regrets(recs, pred)


def evaluate(recs, log=print, steps: int = 4000) -> dict:
    train, test = split(recs)
    costs = fit_analytic(train)
    net, st = train_mlp(train, steps=steps, log=log)
    res = {
        "mlp": regrets(test, mlp_predict_ms(net, st, test)),
        "analytic": regrets(test, analytic_predict_ms(costs, test)),
        "paper_default": fixed_choice_regret(test, lambda o: o["kind"] == 0 and o["lazy_moddown"] and not o["bsgs"]),
        "costs": costs,
        "n_train": len(train), "n_test": len(test),
    }
    for k in ("mlp", "analytic", "paper_default"):
        log(f"[planner] {k:14s} regret on {len(res[k]['shapes'])} held-out shapes: mean {res[k]['mean']:.4f}, "
            f"max {res[k]['max']:.4f}")
    return res, net, st


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--configs", nargs="+", default=["C1", "C2", "C3", "C4"])
    c.add_argument("--shapes", type=int, default=64)
    c.add_argument("--out", default=DEFAULT_DB)
    e = sub.add_parser("evaluate")
    e.add_argument("db", nargs="?", default=DEFAULT_DB)
    e.add_argument("--steps", type=int, default=4000)
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)  # noqa: E731
    if a.cmd == "collect":
        recs = collect(a.configs, a.shapes, log=log)
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        with open(a.out, "w") as f:
            json.dump({"device": "MI355X", "what": "ms of encode_pt + matmul per call, median", "records": recs}, f)
        log(f"[planner] wrote {len(recs)} records to {a.out}")
    else:
        with open(a.db) as f:
            recs = json.load(f)["records"]
        evaluate(recs, log=log, steps=a.steps)


if __name__ == "__main__":
    sys.exit(main())
