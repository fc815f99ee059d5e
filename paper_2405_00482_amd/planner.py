"""Plan selection: measured latencies, the two latency models, and regret.

    python -m paper_2405_00482_amd.planner collect --out DB.json
        times every candidate plan on the current GPU for seeded shapes of
        each parameter set and writes the records (operand form, shape,
        options, batch, features, operation counts, milliseconds) -- the
        exhaustive tuning the planner is judged against.
          * X (m x n) times an encrypted vector: encode of X plus the product,
            per call (C1-C4 and C4's digit-count variants).
          * [[A]] (m x n) times W (n x n_out): Alg. 3 (encode W's packed
            columns plus the product) or the per-row form (encode W^T once,
            then the batched product over the m encrypted rows).
    python -m paper_2405_00482_amd.planner evaluate DB.json
        trains the latency network on the training shapes (GPU kernels),
        fits the analytic model, and prints the regret of each on the
        held-out shapes.

Regret of a choice = its measured latency / the best measured latency of
that shape - 1.  Shapes of C4 and its variants C4a1, C4a2 (one and two
special primes: six and three key-switch digits instead of two) are the
same seeded shapes, so their candidates are pooled: the choice includes the
digit count.  Every computation on the plans runs in libpvfl; this module
only moves data, fits the analytic model's per-operation costs
(non-negative least squares over the training records) and drives the
network's training kernels.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import pvfl
from . import workloads as W

DEFAULT_DB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", "plan_latency_mi355x.json")

FEATURE_NAMES = ("log2_N", "limbs", "alpha", "beta", "K", "log2_m", "log2_n", "log2_mprime", "hybrid", "diag", "row",
                 "ctmat", "lazy", "ras_in_ct", "bsgs", "log2_bsgs", "log2_pack", "log2_batch", "lg_mult", "lg_add",
                 "lg_rot", "lg_hstrot", "lg_modup", "lg_moddown", "lg_pt_limbs", "lg_keys", "lg_blocks")
assert len(FEATURE_NAMES) == pvfl.PLAN_FEATURES

VEC_CONFIGS = ["C1", "C2", "C3", "C4", "C4a1", "C4a2", "C5"]
MAT_CONFIGS = ["C4", "C4a1", "C4a2"]


def family(config: str) -> str:
    """digit-count variants of one parameter set share shapes (and a choice)"""
    return config[:2]


def counts_of(info: dict, batch: int = 1) -> list:
    """the analytic model's count vector (pvfl_plan_analytic_ms order)"""
    b = batch
    return [b * info["n_mult"], b * info["n_add"], b * info["n_rot"], b * info["n_hstrot"], b * info["n_modup"],
            b * info["n_moddown"], info["n_pts"] * info["pt_limbs"], 1]


def is_test_shape(idx: int) -> bool:
    return idx % 4 == 3


def mat_shapes(name: str, count: int):
    """[[A]] (m x n) times W (n x n_out) shapes of VFL layers: m (batch) ~
    logU[16, 1024], n (inputs) and n_out (outputs) ~ logU[8, 512]"""
    g = W.rng(name, 11)
    m = np.exp(g.uniform(np.log(16), np.log(1024), size=count)).astype(np.int64)
    n = np.exp(g.uniform(np.log(8), np.log(512), size=count)).astype(np.int64)
    k = np.exp(g.uniform(np.log(8), np.log(512), size=count)).astype(np.int64)
    return [(int(a), int(b), int(c)) for a, b, c in zip(m, n, k)]


# ---------------------------------------------------------------------------
# exhaustive timing
# ---------------------------------------------------------------------------
def _timed(fn, torch, budget_ms: float = 60.0) -> float:
    s = torch.cuda.current_stream()

    def once():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fn()
        e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1)

    first = once()                       # warm-up (also the estimate)
    if first > budget_ms:
        return once()
    reps = 5 if first < budget_ms / 10 else 2
    return float(np.median([once() for _ in range(reps)]))


def _record(operand, name, idx, shape, cand, plan, ms):
    b = cand.get("batch", 1)
    opts = {k: v for k, v in cand.items() if k != "batch"}
    return {"operand": operand, "config": name, "idx": idx, "m": shape[0], "n": shape[1],
            "n_out": shape[2] if len(shape) > 2 else 0, "opts": opts, "batch": b,
            "features": [round(x, 5) for x in plan.features(b)], "counts": counts_of(plan.info, b),
            "ms": round(float(ms), 5)}


def collect_vec(names, count: int, log=print) -> list:
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

                def run():
                    p.encode_pt(X, pt)
                    p.matmul(ct, pt, keys, out, ws)
                ms = _timed(run, torch)
                recs.append(_record(0, name, idx, (m, n), o, p, ms))
                row.append(ms)
                del pt, ct, out, ws
            best = int(np.argmin(row))
            log(f"[planner] {name} #{idx} {m}x{n}: {len(cs)} candidates, best {row[best]:.3f} ms "
                f"({describe(cs[best])}), hybrid-lazy {row[0]:.3f} ms")
        del keys, plans
        torch.cuda.empty_cache()
    return recs


def collect_mat(names, count: int, log=print) -> list:
    import torch
    recs = []
    for name in names:
        ctx = pvfl.Context.from_dict(W.params_dict(name))
        sd = W.seeds(name)
        sk = ctx.keygen(sd["sk"])
        shapes = mat_shapes(name, count)
        cands = [ctx.candidates(m, n, operand=pvfl.OPERAND_CT_MAT, n_out=k) for (m, n, k) in shapes]
        plans = [[ctx.plan_from(o) for o in cs] for cs in cands]
        gal = sorted(set(g for ps in plans for p in ps for g in p.galois()))
        keys = ctx.rotkeys(sk, gal, sd["rotkeys"]) if gal else None
        torch.cuda.synchronize()
        log(f"[planner] {name} [[A]]W: {len(shapes)} shapes, {sum(len(c) for c in cands)} candidates, "
            f"{len(gal)} rotation keys")
        f64 = dict(dtype=torch.float64, device="cuda")
        for idx, ((m, n, k), cs, ps) in enumerate(zip(shapes, cands, plans)):
            g = W.rng(name, 2000 + idx)
            A = torch.from_numpy(g.uniform(-1, 1, (m, n))).cuda()
            Wm = torch.from_numpy(g.standard_normal((n, k)) * 0.1).cuda()
            WT = Wm.t().contiguous()
            row = []
            for o, p in zip(cs, ps):
                if o["kind"] == pvfl.PLAN_CTMAT:
                    # Alg. 3: [[A]] sent as its diagonals (encryption is the key owner's, untimed)
                    pt = torch.empty(p.bytes("pt") // 8, **f64)
                    ct = torch.empty(p.bytes("ct_in") // 8, **f64)
                    out = torch.empty(p.bytes("ct_out") // 8, **f64)
                    p.encrypt(sk, A, 7 + idx, ct)

                    def run():
                        p.encode_pt(Wm, pt)
                        p.matmul(ct, pt, None, out)
                    ms = _timed(run, torch)
                    del pt, ct, out
                else:
                    # per-row form: W^T (k x n) times each encrypted row of A, one shared plaintext set
                    pt = torch.empty(p.bytes("pt") // 8, **f64)
                    cts = [torch.empty(p.bytes("ct_in") // 8, **f64) for _ in range(m)]
                    outs = [torch.empty(p.bytes("ct_out") // 8, **f64) for _ in range(m)]
                    rows = [A[r].contiguous() for r in range(m)]
                    b = pvfl.Batch(ctx, [p] * m, v=rows, pt=[pt] * m, ct=cts, out=outs, keys=keys)
                    b.encrypt(sk, 7 + idx)

                    def run():
                        p.encode_pt(WT, pt)
                        b.matmul()
                    ms = _timed(run, torch)
                    del b, pt, cts, outs, rows
                recs.append(_record(1, name, idx, (m, n, k), o, p, ms))
                row.append(ms)
            best = int(np.argmin(row))
            log(f"[planner] {name} [[A]]W #{idx} {m}x{n}x{k}: {len(cs)} candidates, best {row[best]:.3f} ms "
                f"({describe(cs[best])})")
        del keys, plans
        torch.cuda.empty_cache()
    return recs


def describe(o: dict) -> str:
    kind = {0: "HYBRID", 1: "DIAG", 2: "ROW", 3: "CTMAT"}[o["kind"]]
    if o["kind"] == 3:
        return f"CTMAT pack{o.get('pack', 1)}"
    s = kind + ("" if o["kind"] == 2 else (" lazy" if o["lazy_moddown"] else " eager"))
    if o.get("bsgs"):
        s += f" bsgs{o['bsgs']}"
    if o.get("unhoisted"):
        s += " O3"
    if o.get("ras_in_ct"):
        s += " ras-in-ct"
    if o.get("batch", 1) > 1:
        s += f" per-row x{o['batch']}"
    return s


def describe_rec(r: dict) -> str:
    return f"{r['config']} " + describe({**r["opts"], "batch": r.get("batch", 1)})


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


def shape_key(r) -> tuple:
    return (r.get("operand", 0), family(r["config"]), r["idx"])


def regrets(recs, pred) -> dict:
    """per shape (candidates of a parameter set's digit-count variants pooled):
    measured latency of the predicted-best candidate over the measured best,
    minus one"""
    by = {}
    for r, p in zip(recs, pred):
        by.setdefault(shape_key(r), []).append((p, r["ms"], r))
    out = []
    for key, rows in sorted(by.items()):
        best = min(ms for _, ms, _ in rows)
        pick = min(rows, key=lambda t: t[0])
        out.append({"operand": key[0], "config": key[1], "idx": key[2], "regret": pick[1] / best - 1.0,
                    "chosen": describe_rec(pick[2]), "best": describe_rec(min(rows, key=lambda t: t[1])[2])})
    rg = np.array([o["regret"] for o in out])
    return {"mean": float(rg.mean()), "max": float(rg.max()), "geo": float(np.exp(np.mean(np.log1p(rg)))) - 1.0,
            "shapes": out}


def fixed_choice_regret(recs, pick) -> dict:
    """regret of always taking the candidate for which pick(record) is True
    (shapes where no candidate qualifies take their first)"""
    pred = np.array([0.0 if pick(r) else 1.0 for r in recs])
    return regrets(recs, pred)


def paper_default(r) -> bool:
    """the paper's choices: the hybrid with hoisted rotations for X [[y]]
    (Sec. 4) and Alg. 3 for [[A]] W (Sec. 5), on the configured digit count"""
    o = r["opts"]
    if r["config"] not in ("C1", "C2", "C3", "C4", "C5"):
        return False
    if r.get("operand", 0) == 1:
        return o["kind"] == 3 and o.get("pack", 1) == 1
    return o["kind"] == 0 and o["lazy_moddown"] and not o.get("bsgs", 0)


def evaluate(recs, log=print, steps: int = 4000) -> dict:
    train, test = split(recs)
    costs = fit_analytic(train)
    net, st = train_mlp(train, steps=steps, log=log)
    pm = mlp_predict_ms(net, st, test)
    pa = analytic_predict_ms(costs, test)
    res = {"costs": costs, "n_train": len(train), "n_test": len(test)}
    for operand, label in ((None, "all"), (0, "X[[y]]"), (1, "[[A]]W")):
        sel = [i for i, r in enumerate(test) if operand is None or r.get("operand", 0) == operand]
        if not sel:
            continue
        sub = [test[i] for i in sel]
        res[label] = {"mlp": regrets(sub, pm[sel]), "analytic": regrets(sub, pa[sel]),
                      "paper_default": fixed_choice_regret(sub, paper_default)}
        for k in ("mlp", "analytic", "paper_default"):
            v = res[label][k]
            log(f"[planner] {label:7s} {k:14s} regret on {len(v['shapes'])} held-out shapes: mean {v['mean']:.4f}, "
                f"max {v['max']:.4f}")
    res["mlp"], res["analytic"], res["paper_default"] = (res["all"][k] for k in ("mlp", "analytic", "paper_default"))
    return res, net, st


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--vec-configs", nargs="*", default=VEC_CONFIGS)
    c.add_argument("--mat-configs", nargs="*", default=MAT_CONFIGS)
    c.add_argument("--shapes", type=int, default=64)
    c.add_argument("--mat-shapes", type=int, default=48)
    c.add_argument("--out", default=DEFAULT_DB)
    e = sub.add_parser("evaluate")
    e.add_argument("db", nargs="?", default=DEFAULT_DB)
    e.add_argument("--steps", type=int, default=4000)
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)  # noqa: E731
    if a.cmd == "collect":
        recs = collect_vec(a.vec_configs, a.shapes, log=log) + collect_mat(a.mat_configs, a.mat_shapes, log=log)
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        with open(a.out, "w") as f:
            json.dump({"device": "MI355X", "what": "ms per call of every candidate plan (median of repeats)",
                       "command": "python -m paper_2405_00482_amd.planner collect", "records": recs}, f,
                      separators=(",", ":"))
        log(f"[planner] wrote {len(recs)} records to {a.out}")
    else:
        with open(a.db) as f:
            recs = json.load(f)["records"]
        evaluate(recs, log=log, steps=a.steps)


if __name__ == "__main__":
    sys.exit(main())
